"""CPU oracle of the IMEX-DS hot path (ctypes binding of imexds_oracle.c).

TEST INFRASTRUCTURE ONLY: tests/, the package smoke check and the bench's
cpu_baseline leg may import this package; the product path never does.  The
C source is compiled here with gcc (-O2 -ffp-contract=off, OpenMP over
independent problems) and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "imexds_oracle.c")
SRC_EULER = os.path.join(_HERE, "euler_oracle.c")
DUAL_H = os.path.join(_HERE, "or_dual.h")
LIB = os.path.join(_HERE, "liboracle_imexds.so")
LIB_TAN = os.path.join(_HERE, "liboracle_imexds_tan.so")
# the same source with every formula as the paper prints it and the C
# library's log (OR_PLAIN; see the source's header)
LIB_PLAIN = os.path.join(_HERE, "liboracle_imexds_plain.so")

ST_NEWTON, ST_NONPHYS, ST_MESH, ST_OVERLAP, ST_VANISH = 1, 2, 4, 8, 16
FL_TINY_RIGHT, FL_MERGED, FL_REDO, FL_LMAX = 1, 2, 4, 8
FL_CROSS_L, FL_CROSS_R, FL_FAIL, FL_INACTIVE, FL_PAIR = 16, 32, 64, 128, 256


def build():
    """Compiles the oracle shared library, its tangent (dual-number) build
    and its plain-arithmetic build from the same source (always
    recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-shared", "-fPIC", "-o", tmp, SRC, SRC_EULER, "-lm"])
    os.replace(tmp, LIB)
    tmp = LIB_PLAIN + ".tmp"
    subprocess.check_call(["gcc", "-DOR_PLAIN", "-O2", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_PLAIN)
    tmp = LIB_TAN + ".tmp"
    subprocess.check_call(["g++", "-x", "c++", "-std=c++17", "-DOR_TANGENT", "-I", _HERE, "-O2",
                           "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
                           "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_TAN)


class _Mat(ctypes.Structure):
    _fields_ = [("a2v", ctypes.c_double), ("a2l", ctypes.c_double), ("p0", ctypes.c_double),
                ("rhol0", ctypes.c_double), ("tau", ctypes.c_double)]


class _Par(ctypes.Structure):
    _fields_ = [("cfl", ctypes.c_double), ("zone_half", ctypes.c_int),
                ("theta_nb", ctypes.c_double), ("tol_mode", ctypes.c_int),
                ("tol_nb", ctypes.c_double), ("tol_tiny", ctypes.c_double),
                ("tol_rel", ctypes.c_double), ("lmax", ctypes.c_int),
                ("alpha_floor", ctypes.c_double), ("merge_safety", ctypes.c_double),
                ("bc_left", ctypes.c_int), ("bc_right", ctypes.c_int),
                ("newton_maxit", ctypes.c_int), ("newton_rtol", ctypes.c_double),
                ("t_end", ctypes.c_double), ("zone_solver", ctypes.c_int),
                ("zn_maxit", ctypes.c_int), ("zn_rtol", ctypes.c_double)]


class _Iface(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("pl", "pr", "rl", "rr", "ul", "ur", "z", "w",
                                               "F0", "F1")] + [("iters", ctypes.c_int),
                                                               ("ok", ctypes.c_int)]


_lib = None
_lib_tan = None
_lib_plain = None


def _stale(path):
    return (not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC)
            or os.path.getmtime(path) < os.path.getmtime(DUAL_H)
            or os.path.getmtime(path) < os.path.getmtime(SRC_EULER))


def _run_argtypes(L):
    dp, ip, lp = (ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                  ctypes.POINTER(ctypes.c_longlong))
    run_args = [ctypes.POINTER(_Mat), ctypes.POINTER(_Par), ctypes.c_int, ip, dp, ip, ip, lp, ip,
                dp, dp, ip, dp, dp, dp, ip, lp, ctypes.c_int, ip, ip, ip, ip, ip, ip, ip,
                ctypes.c_int]
    L.oracle_run.restype = ctypes.c_int
    L.oracle_run.argtypes = run_args
    L.oracle_run_trace.restype = ctypes.c_int
    L.oracle_run_trace.argtypes = run_args + [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                              ctypes.c_int, ip]


def lib():
    global _lib
    if _lib is None:
        if _stale(LIB) or _stale(LIB_TAN) or _stale(LIB_PLAIN):
            build()
        L = ctypes.CDLL(LIB)
        dp, ip, lp = (ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                      ctypes.POINTER(ctypes.c_longlong))
        _run_argtypes(L)
        L.oracle_objective.restype = None
        L.oracle_objective.argtypes = [ctypes.c_int, ip, dp, dp, ip, lp, ip, dp, dp,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_iface_solve.restype = ctypes.c_int
        L.oracle_iface_solve.argtypes = [ctypes.POINTER(_Mat), ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(_Iface)]
        L.oracle_iface_G.restype = ctypes.c_int
        L.oracle_iface_G.argtypes = [ctypes.POINTER(_Mat), ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_block_tri.restype = ctypes.c_int
        L.oracle_block_tri.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        L.oracle_hll.restype = None
        L.oracle_hll.argtypes = [ctypes.POINTER(_Mat), ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_zone_fixed_point.restype = ctypes.c_int
        L.oracle_zone_fixed_point.argtypes = [ctypes.POINTER(_Mat), ctypes.POINTER(_Par),
                                              ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_int, dp, dp, ip, dp, dp, ip, ctypes.c_int,
                                              dp, dp, ip, dp]
        L.oracle_creation_rp.restype = ctypes.c_int
        L.oracle_creation_rp.argtypes = [ctypes.POINTER(_Mat), ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_double, dp]
        L.oracle_creation_batch.restype = None
        L.oracle_creation_batch.argtypes = [ctypes.POINTER(_Mat), ctypes.c_int, ip, dp, dp, dp, dp,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_double, ip, dp, ctypes.c_int]
        L.oracle_exp.restype = ctypes.c_double
        L.oracle_exp.argtypes = [ctypes.c_double]
        L.oracle_euler_riemann.restype = ctypes.c_int
        L.oracle_euler_riemann.argtypes = [ctypes.c_double, dp, dp, dp, dp, dp]
        L.oracle_euler_run.restype = ctypes.c_int
        L.oracle_euler_run.argtypes = ([ctypes.c_int, lp, ip] + [dp] * 6
                                       + [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int, dp, dp, dp, dp, ip, ip, lp, ctypes.c_int,
                                          ip, ip, ctypes.c_int])
        L.oracle_ct_run.restype = ctypes.c_int
        L.oracle_ct_run.argtypes = ([ctypes.POINTER(_Mat), ctypes.POINTER(_Par), ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ip, dp, ip, lp, dp, dp, ip,
                                     dp, dp, dp, dp, ip, ip, lp, ctypes.c_int, ip, ip,
                                     ctypes.c_int])
        _lib = L
    return _lib


def lib_plain():
    """The plain-arithmetic build (oracle_run, oracle_run_trace and the
    interface solve only)."""
    global _lib_plain
    if _lib_plain is None:
        lib()
        L = ctypes.CDLL(LIB_PLAIN)
        _run_argtypes(L)
        L.oracle_iface_solve.restype = ctypes.c_int
        L.oracle_iface_solve.argtypes = lib().oracle_iface_solve.argtypes
        _lib_plain = L
    return _lib_plain


def _mat(m):
    return _Mat(m.a2v, m.a2l, m.p0, m.rhol0, m.tau)


def _par(p):
    return _Par(p.cfl, p.zone_half, p.theta_nb, p.tol_mode, p.tol_nb, p.tol_tiny, p.tol_rel,
                p.lmax, p.alpha_floor, p.merge_safety, p.bc_left, p.bc_right, p.newton_maxit,
                p.newton_rtol, p.t_end, int(getattr(p, "zone_solver", 0)),
                int(getattr(p, "zn_maxit", 30)), float(getattr(p, "zn_rtol", 1e-10)))


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


class State:
    """Evolving state of a batch in the oracle (all host numpy arrays)."""

    def __init__(self, batch):
        self.batch = batch
        P, nif = batch.n_problems, batch.n_iface
        self.rho = np.ascontiguousarray(batch.rho, dtype=np.float64).copy()
        self.mom = np.ascontiguousarray(batch.mom, dtype=np.float64).copy()
        self.home = np.ascontiguousarray(batch.home, dtype=np.int32).copy()
        self.hl = np.ascontiguousarray(batch.hl, dtype=np.float64).copy()
        self.pw = np.zeros(2 * max(nif, 1), dtype=np.float64)
        self.warm = np.zeros(max(nif, 1), dtype=np.int32)
        self.t = np.zeros(P, dtype=np.float64)
        self.status = np.zeros(P, dtype=np.int32)
        self.steps = np.zeros(P, dtype=np.int64)

    def x_iface(self):
        b = self.batch
        out = np.empty(b.n_iface)
        for p in range(b.n_problems):
            for k in range(int(b.iface_off[p]), int(b.iface_off[p + 1])):
                out[k] = b.x_left[p] + self.home[k] * b.h[p] + self.hl[k]
        return out


def _geometry(b):
    return (np.ascontiguousarray(b.n_cells, dtype=np.int32),
            np.ascontiguousarray(b.h, dtype=np.float64),
            np.ascontiguousarray(b.phase_first, dtype=np.int32),
            np.ascontiguousarray(b.iface_off, dtype=np.int32),
            np.ascontiguousarray(b.slot_off, dtype=np.int64))


def run(state, material, params, n_steps, log=False, threads=1, replay=None, plain=False,
        trace=None):
    """Advances every problem of ``state`` by ``n_steps`` steps (or until
    t_end / failure).  Returns per-step logs (count, flags, zlo) of shape
    [n_steps, n_iface] if ``log`` (with log="full": also the CFL slot,
    [n_steps, n_problems]).  ``replay`` = a full log of an earlier run:
    its decisions are repeated instead of taken.  ``plain``: run the
    plain-arithmetic build.  ``trace`` = (problem, step, local interface):
    the dual time iterates of that zone solve are recorded and returned
    (see trace_record) as the last element of the result."""
    b = state.batch
    L = lib_plain() if plain else lib()
    m, p = _mat(material), _par(params)
    n_cells, h, pf, ioff, soff = _geometry(b)
    nif = b.n_iface
    lcp = lfp = lzp = lsp = None
    if log:
        lc = np.zeros((n_steps, max(nif, 1)), dtype=np.int32)
        lf = np.zeros_like(lc)
        lz = np.zeros_like(lc)
        ls = np.zeros((n_steps, b.n_problems), dtype=np.int32)
        lcp, lfp, lzp = (_ptr(lc, ctypes.c_int), _ptr(lf, ctypes.c_int), _ptr(lz, ctypes.c_int))
        lsp = _ptr(ls, ctypes.c_int)
    rcp = rfp = rsp = None
    if replay is not None:
        rc_, rf_, _, rs_ = replay
        assert rc_.shape[0] >= n_steps and rs_.shape[0] >= n_steps
        keep = [np.ascontiguousarray(np.pad(a[:n_steps], ((0, 0), (0, max(1, a.shape[1]) - a.shape[1]))),
                                     dtype=np.int32) for a in (rc_, rf_)]
        keep.append(np.ascontiguousarray(rs_[:n_steps], dtype=np.int32))
        rcp, rfp, rsp = (_ptr(a, ctypes.c_int) for a in keep)
    args = (ctypes.byref(m), ctypes.byref(p), b.n_problems, _ptr(n_cells, ctypes.c_int),
            _ptr(h, ctypes.c_double), _ptr(pf, ctypes.c_int), _ptr(ioff, ctypes.c_int),
            _ptr(soff, ctypes.c_longlong), _ptr(state.home, ctypes.c_int),
            _ptr(state.hl, ctypes.c_double), _ptr(state.pw, ctypes.c_double),
            _ptr(state.warm, ctypes.c_int), _ptr(state.rho, ctypes.c_double),
            _ptr(state.mom, ctypes.c_double), _ptr(state.t, ctypes.c_double),
            _ptr(state.status, ctypes.c_int), _ptr(state.steps, ctypes.c_longlong),
            int(n_steps), lcp, lfp, lzp, lsp, rcp, rfp, rsp, int(threads))
    rec = None
    if trace is None:
        rc = L.oracle_run(*args)
    else:
        tp, tstep, tk = (int(x) for x in trace)
        cap = 8 + 4 * 32 + (params.lmax + 2) * (2 * 32 + 1) + 64
        buf = np.zeros(cap)
        n = ctypes.c_int(0)
        rc = L.oracle_run_trace(*args, tp, tstep, tk, _ptr(buf, ctypes.c_double), cap,
                                ctypes.byref(n))
        assert n.value <= cap
        rec = trace_record(buf[:n.value])
    if rc != 0:
        raise ValueError(f"oracle_run rejected the parameters (rc={rc})")
    out = ()
    if log == "full":
        out = (lc[:, :nif], lf[:, :nif], lz[:, :nif], ls)
    elif log:
        out = (lc[:, :nif], lf[:, :nif], lz[:, :nif])
    if trace is not None:
        return out + (rec,)
    return out if log else None


def trace_record(buf):
    """Decodes one zone-solve record of oracle_run_trace: the zone's active
    cells (m), its tiny cell, the cell left of the phase boundary, dt, the
    dual time count and whether it stopped at lmax; per cell theta, h^n, the
    predicted end length and its motion (+1, -1, 0); the iterates W[l]
    (l = 0 .. count, shape [count+1, m, 2]) and the phase-boundary speed w[l]
    of the interface solve on W[l].  None if no zone was recorded."""
    if len(buf) == 0:
        return None
    m, tiny, ic = int(buf[0]), int(buf[1]), int(buf[2])
    dt, count, lmax_hit, nrec = float(buf[3]), int(buf[4]), bool(buf[5]), int(buf[6])
    cells = buf[8:8 + 4 * m].reshape(m, 4)
    it = buf[8 + 4 * m:8 + 4 * m + nrec * (2 * m + 1)].reshape(nrec, 2 * m + 1)
    return {"m": m, "tiny": tiny, "ic": ic, "dt": dt, "count": count, "lmax": lmax_hit,
            "theta": cells[:, 0].copy(), "hn": cells[:, 1].copy(), "hh": cells[:, 2].copy(),
            "mov": cells[:, 3].copy(), "W": it[:, :2 * m].reshape(nrec, m, 2).copy(),
            "w": it[:, 2 * m].copy()}


# objective of the adjoint: cx * sum of interface positions + mass in [wa, wb]
OBJ_CX, OBJ_WA, OBJ_WB = 1.0, 0.4, 0.6


def objective(state, cx=OBJ_CX, wa=OBJ_WA, wb=OBJ_WB):
    """Per-problem objective cx sum_k x_k + sum_s rho_s |slot_s ∩ [wa, wb]|."""
    b = state.batch
    n_cells, h, _, ioff, soff = _geometry(b)
    xl = np.ascontiguousarray(b.x_left, dtype=np.float64)
    out = np.zeros(b.n_problems)
    lib().oracle_objective(b.n_problems, _ptr(n_cells, ctypes.c_int), _ptr(h, ctypes.c_double),
                           _ptr(xl, ctypes.c_double), _ptr(ioff, ctypes.c_int),
                           _ptr(soff, ctypes.c_longlong), _ptr(state.home, ctypes.c_int),
                           _ptr(state.hl, ctypes.c_double), _ptr(state.rho, ctypes.c_double),
                           float(cx), float(wa), float(wb), _ptr(out, ctypes.c_double))
    return out


def lib_tan():
    global _lib_tan
    if _lib_tan is None:
        lib()
        L = ctypes.CDLL(LIB_TAN)
        dp, ip, lp = (ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                      ctypes.POINTER(ctypes.c_longlong))
        L.oracle_tan_run.restype = ctypes.c_int
        L.oracle_tan_run.argtypes = [dp, dp, ctypes.POINTER(_Par), ctypes.c_int, ip, dp, dp, ip, ip,
                                     lp, ip, dp, dp, dp, dp, ip, dp, dp, dp, dp, dp, dp, ip, lp,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, dp, ctypes.c_int]
        _lib_tan = L
    return _lib_tan


def tangent(state, material, params, n_steps, d_rho, d_mom, d_tau=0.0, d_hl=None,
            cx=OBJ_CX, wa=OBJ_WA, wb=OBJ_WB, threads=1):
    """Forward-mode derivative of the objective after ``n_steps`` steps along
    the direction (d_rho, d_mom, d_tau[, d_hl]) of the initial state and the
    kinetic coefficient (decisions frozen: those of the plain run).  Advances
    ``state`` like run(); returns (objective per problem, derivative per
    problem, final (d_rho, d_mom, d_hl))."""
    b = state.batch
    L = lib_tan()
    n_cells, h, pf, ioff, soff = _geometry(b)
    xl = np.ascontiguousarray(b.x_left, dtype=np.float64)
    nif = max(b.n_iface, 1)
    mat = np.array([material.a2v, material.a2l, material.p0, material.rhol0, material.tau])
    dmat = np.array([0.0, 0.0, 0.0, 0.0, float(d_tau)])
    dr = np.ascontiguousarray(d_rho, dtype=np.float64).copy()
    dm = np.ascontiguousarray(d_mom, dtype=np.float64).copy()
    dh = np.zeros(nif) if d_hl is None else np.ascontiguousarray(d_hl, dtype=np.float64).copy()
    dpw = np.zeros(2 * nif)
    dt = np.zeros(b.n_problems)
    obj = np.zeros(b.n_problems)
    dobj = np.zeros(b.n_problems)
    rc = L.oracle_tan_run(_ptr(mat, ctypes.c_double), _ptr(dmat, ctypes.c_double),
                          ctypes.byref(_par(params)), b.n_problems, _ptr(n_cells, ctypes.c_int),
                          _ptr(h, ctypes.c_double), _ptr(xl, ctypes.c_double),
                          _ptr(pf, ctypes.c_int), _ptr(ioff, ctypes.c_int),
                          _ptr(soff, ctypes.c_longlong), _ptr(state.home, ctypes.c_int),
                          _ptr(state.hl, ctypes.c_double), _ptr(dh, ctypes.c_double),
                          _ptr(state.pw, ctypes.c_double), _ptr(dpw, ctypes.c_double),
                          _ptr(state.warm, ctypes.c_int), _ptr(state.rho, ctypes.c_double),
                          _ptr(dr, ctypes.c_double), _ptr(state.mom, ctypes.c_double),
                          _ptr(dm, ctypes.c_double), _ptr(state.t, ctypes.c_double),
                          _ptr(dt, ctypes.c_double), _ptr(state.status, ctypes.c_int),
                          _ptr(state.steps, ctypes.c_longlong), int(n_steps), float(cx),
                          float(wa), float(wb), _ptr(obj, ctypes.c_double),
                          _ptr(dobj, ctypes.c_double), int(threads))
    if rc != 0:
        raise ValueError(f"oracle_tan_run rejected the parameters (rc={rc})")
    return obj, dobj, (dr, dm, dh[:b.n_iface])


def iface_solve(material, phl, rl, ul, phr, rr, ur, guess=None, maxit=50, rtol=1e-10):
    """Two-phase interface Riemann problem from primitive (rho, u) states."""
    out = _Iface()
    g = guess if guess is not None else (0.0, 0.0)
    ok = lib().oracle_iface_solve(ctypes.byref(_mat(material)), int(phl), float(rl),
                                  float(rl * ul), int(phr), float(rr), float(rr * ur),
                                  int(guess is not None), float(g[0]), float(g[1]), int(maxit),
                                  float(rtol), ctypes.byref(out))
    d = {n: getattr(out, n) for n, _ in _Iface._fields_}
    d["ok"] = bool(ok)
    return d


def iface_G(material, phl, rl, ul, phr, rr, ur, psl, psr):
    o = np.zeros(6)
    ok = lib().oracle_iface_G(ctypes.byref(_mat(material)), int(phl), float(rl), float(rl * ul),
                              int(phr), float(rr), float(rr * ur), float(psl), float(psr),
                              _ptr(o, ctypes.c_double))
    if not ok:
        return None
    return o[:2].copy(), o[2:].reshape(2, 2).copy()


CREATION_FIELDS = ("kind", "p1", "pa", "pb", "pc", "ra", "rb", "rc", "ua", "ub", "uc", "zl",
                   "zr", "wl", "wr", "Fl0", "Fl1", "Fr0", "Fr1", "iters")


def creation_rp(material, phase, rl, ml, rr, mr, p_min, p_tilde, maxit=50, rtol=1e-14):
    """Phase creation for a Riemann problem of one phase: (status, dict).
    status 0: no creation (dict['p1'] = star pressure without phase
    transition), 1: a layer of the other phase is created (five states:
    a | b (new phase) | c, boundaries at speeds wl, wr), -1: failure."""
    out = np.zeros(len(CREATION_FIELDS))
    st = lib().oracle_creation_rp(ctypes.byref(_mat(material)), int(phase), float(rl), float(ml),
                                  float(rr), float(mr), float(p_min), float(p_tilde), int(maxit),
                                  float(rtol), _ptr(out, ctypes.c_double))
    return st, dict(zip(CREATION_FIELDS, out.tolist()))


def creation_batch(material, phase, rl, ml, rr, mr, p_min, p_tilde, maxit=50, rtol=1e-14,
                   threads=1):
    """Vectorised creation_rp: (status [n], out [n, 20]) in CREATION_FIELDS order."""
    phase = np.ascontiguousarray(phase, dtype=np.int32)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rl, ml, rr, mr)]
    n = phase.shape[0]
    status = np.zeros(n, dtype=np.int32)
    out = np.zeros((n, len(CREATION_FIELDS)))
    lib().oracle_creation_batch(ctypes.byref(_mat(material)), n, _ptr(phase, ctypes.c_int),
                                *[_ptr(a, ctypes.c_double) for a in arrs], float(p_min),
                                float(p_tilde), int(maxit), float(rtol),
                                _ptr(status, ctypes.c_int), _ptr(out, ctypes.c_double),
                                int(threads))
    return status, out


def block_tri(D, L, U, r):
    """Block tridiagonal solve of the Newton zone solvers (block Thomas):
    D, L, U of shape [m, 2, 2] (L[0], U[m-1] unused), r of shape [m, 2];
    returns x of shape [m, 2], or None if a pivot block has no finite
    inverse or a result is not finite."""
    m = len(D)
    args = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (D, L, U, r)]
    x = np.zeros(2 * m)
    ok = lib().oracle_block_tri(int(m), *[_ptr(a, ctypes.c_double) for a in args],
                                _ptr(x, ctypes.c_double))
    return x.reshape(m, 2) if ok else None


def hll(material, phase, rl, ml, rr, mr):
    F = np.zeros(2)
    lib().oracle_hll(ctypes.byref(_mat(material)), int(phase), float(rl), float(ml), float(rr),
                     float(mr), _ptr(F, ctypes.c_double))
    return F


def zone_fixed_point(state, material, params, k=0):
    """For a single-problem state: Algorithm 2 Part 1 iterate vs a direct
    Newton solve of the zone's implicit system (see the C source)."""
    b = state.batch
    assert b.n_problems == 1
    Wd = np.zeros(64)
    Wn = np.zeros(64)
    m = np.zeros(1, dtype=np.int32)
    dt = np.zeros(1)
    rc = lib().oracle_zone_fixed_point(
        ctypes.byref(_mat(material)), ctypes.byref(_par(params)), int(b.n_cells[0]),
        float(b.h[0]), int(b.phase_first[0]), int(b.n_iface), _ptr(state.rho, ctypes.c_double),
        _ptr(state.mom, ctypes.c_double), _ptr(state.home, ctypes.c_int),
        _ptr(state.hl, ctypes.c_double), _ptr(state.pw, ctypes.c_double),
        _ptr(state.warm, ctypes.c_int), int(k), _ptr(Wd, ctypes.c_double),
        _ptr(Wn, ctypes.c_double), _ptr(m, ctypes.c_int), _ptr(dt, ctypes.c_double))
    n = 2 * int(m[0])
    return rc, Wd[:n].reshape(-1, 2), Wn[:n].reshape(-1, 2), float(dt[0])


# ---------------------------------------------------------------------------
# full Euler equations on a fixed mesh with one small cell (euler_oracle.c)
# ---------------------------------------------------------------------------

EU_ST_VACUUM, EU_ST_NEWTON, EU_ST_NONPHYS = 1, 2, 4
EU_FL_LMAX = 1


def exp(x):
    """The oracle's fixed-order exponential."""
    return lib().oracle_exp(float(x))


def euler_riemann(gamma, WL, WR):
    """Exact Riemann solution of the ideal-gas Euler equations for primitive
    data WL, WR = (rho, u, p): returns (status, W0, F, star) with W0 the state
    at x/t = 0, F its flux and star = (p*, u*, rho*_L, rho*_R)."""
    wl = np.ascontiguousarray(WL, dtype=np.float64)
    wr = np.ascontiguousarray(WR, dtype=np.float64)
    W0, F, star = np.zeros(3), np.zeros(3), np.zeros(4)
    st = lib().oracle_euler_riemann(float(gamma), _ptr(wl, ctypes.c_double),
                                    _ptr(wr, ctypes.c_double), _ptr(W0, ctypes.c_double),
                                    _ptr(F, ctypes.c_double), _ptr(star, ctypes.c_double))
    return st, W0, F, star


class EulerState:
    """Evolving state of an EulerBatch in the oracle."""

    def __init__(self, eb):
        self.batch = eb
        P = eb.n_problems
        self.rho = np.ascontiguousarray(eb.rho, dtype=np.float64).copy()
        self.mom = np.ascontiguousarray(eb.mom, dtype=np.float64).copy()
        self.ene = np.ascontiguousarray(eb.ene, dtype=np.float64).copy()
        self.t = np.zeros(P, dtype=np.float64)
        self.steps = np.zeros(P, dtype=np.int32)
        self.status = np.zeros(P, dtype=np.int32)
        self.iters = np.zeros(P, dtype=np.int64)


def euler_run(state, n_steps=None, threads=1, log=False):
    """Advances every problem by up to n_steps time steps (None: to t_end).
    With log=True returns (counts, flags), each [P, n_steps] (0 where a
    problem did not step)."""
    b = state.batch
    P = b.n_problems
    if n_steps is None:
        if log:
            raise ValueError("log=True needs n_steps")
        n_steps = 2**31 - 1
    off = np.ascontiguousarray(b.off[:-1], dtype=np.int64)
    N = np.ascontiguousarray(b.N, dtype=np.int32)
    per = [np.ascontiguousarray(getattr(b, f), dtype=np.float64)
           for f in ("h", "alpha", "theta_nb", "theta_k", "cfl", "t_end")]
    lc = lf = None
    if log:
        lc = np.zeros((P, n_steps), dtype=np.int32)
        lf = np.zeros((P, n_steps), dtype=np.int32)
    d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_longlong
    lib().oracle_euler_run(P, _ptr(off, l), _ptr(N, i), *[_ptr(a, d) for a in per],
                           float(b.gamma), float(b.tol_nb), float(b.tol_k), int(b.lmax),
                           _ptr(state.rho, d), _ptr(state.mom, d), _ptr(state.ene, d),
                           _ptr(state.t, d), _ptr(state.steps, i), _ptr(state.status, i),
                           _ptr(state.iters, l), int(n_steps),
                           _ptr(lc, i) if log else None, _ptr(lf, i) if log else None,
                           int(threads))
    if log:
        return lc, lf
    return None


CT_ST_NEWTON, CT_ST_NONPHYS, CT_ST_MESH, CT_ST_MULTI = 1, 2, 4, 8
CT_FL_CREATED, CT_FL_LMAX, CT_FL_INACTIVE = 1, 2, 4


class CTubeState:
    """Evolving state of a CTubeBatch (creation tubes) in the oracle: cell
    values, the face of the created cell (-1: none yet), its boundary
    offsets dl, dr from that face, the boundaries' warm starts pw [P, 4],
    time, status, steps and dual time iterations."""

    def __init__(self, cb):
        self.batch = cb
        P = cb.n_problems
        self.rho = np.ascontiguousarray(cb.rho, dtype=np.float64).copy()
        self.mom = np.ascontiguousarray(cb.mom, dtype=np.float64).copy()
        self.face = np.full(P, -1, dtype=np.int32)
        self.dl = np.zeros(P)
        self.dr = np.zeros(P)
        self.pw = np.zeros((P, 4))
        self.t = np.zeros(P)
        self.status = np.zeros(P, dtype=np.int32)
        self.steps = np.zeros(P, dtype=np.int32)
        self.iters = np.zeros(P, dtype=np.int64)


CT_SOLVER_DTS, CT_SOLVER_NEWTON = 0, 1


def ct_run(state, n_steps=None, threads=1, log=False, solver=CT_SOLVER_DTS, zn_maxit=30,
           zn_rtol=1e-10):
    """Advances every creation tube by up to n_steps steps (None: to t_end),
    the zone solved by Algorithm 2 (CT_SOLVER_DTS) or by Newton
    (CT_SOLVER_NEWTON: at most zn_maxit steps, tolerance zn_rtol).  With
    log=True returns (counts, flags), each [n_steps, P]."""
    b = state.batch
    P = b.n_problems
    if n_steps is None:
        if log:
            raise ValueError("log=True needs n_steps")
        n_steps = 2**31 - 1
    off = np.ascontiguousarray(b.off[:-1], dtype=np.int64)
    N = np.ascontiguousarray(b.N, dtype=np.int32)
    h = np.ascontiguousarray(b.h, dtype=np.float64)
    ph = np.ascontiguousarray(b.phase, dtype=np.int32)
    lc = lf = None
    if log:
        lc = np.zeros((n_steps, P), dtype=np.int32)
        lf = np.zeros((n_steps, P), dtype=np.int32)
    d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_longlong
    m, par = _mat(b.material), _par(b.params)
    rc = lib().oracle_ct_run(ctypes.byref(m), ctypes.byref(par), float(b.p_min),
                             float(b.p_tilde), int(solver), int(zn_maxit), float(zn_rtol), P,
                             _ptr(N, i), _ptr(h, d), _ptr(ph, i),
                             _ptr(off, l), _ptr(state.rho, d), _ptr(state.mom, d),
                             _ptr(state.face, i), _ptr(state.dl, d), _ptr(state.dr, d),
                             _ptr(state.pw, d), _ptr(state.t, d), _ptr(state.status, i),
                             _ptr(state.steps, i), _ptr(state.iters, l), int(n_steps),
                             _ptr(lc, i) if log else None, _ptr(lf, i) if log else None,
                             int(threads))
    if rc != 0:
        raise ValueError("oracle_ct_run: zone_half out of range")
    if log:
        return lc, lf
    return None
