"""ctypes binding of libimexds.so (include/imexds.h).

The ``imexds_*`` functions here mirror the C ABI one to one (argument
marshalling only); ``IMEXDS`` is a small convenience wrapper around them that
holds the context.  Device pointers come from torch tensors on cuda (FP64,
contiguous); torch is used only for device memory and streams.  There is no
fallback: if the library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimexds.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2211_00705_amd.build` "
                      "(the IMEX-DS path has no CPU fallback)")
_L = ctypes.CDLL(LIB_PATH)

OK, ERR_INVALID_ARG, ERR_OOM, ERR_HIP, ERR_NO_STATE, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
ST_NEWTON_FAIL, ST_NONPHYSICAL, ST_MESH_FAIL, ST_ZONE_OVERLAP, ST_PHASE_VANISH = 1, 2, 4, 8, 16
FL_TINY_RIGHT, FL_MERGED, FL_REDO, FL_LMAX = 1, 2, 4, 8
FL_CROSS_L, FL_CROSS_R, FL_FAIL, FL_INACTIVE, FL_PAIR = 16, 32, 64, 128, 256
TOL_PAPER, TOL_REL = 0, 1

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P_i32, P_i64, P_dbl = ctypes.POINTER(c_i32), ctypes.POINTER(c_i64), ctypes.POINTER(c_dbl)


class imexds_material(ctypes.Structure):
    _fields_ = [("a2_vap", c_dbl), ("a2_liq", c_dbl), ("p_sat", c_dbl), ("rho_liq_sat", c_dbl),
                ("tau", c_dbl)]


class imexds_params(ctypes.Structure):
    _fields_ = [("cfl", c_dbl), ("zone_half", c_i32), ("theta_nb", c_dbl), ("tol_mode", c_i32),
                ("tol_nb", c_dbl), ("tol_tiny", c_dbl), ("tol_rel", c_dbl), ("lmax", c_i32),
                ("alpha_floor", c_dbl), ("merge_safety", c_dbl), ("bc_left", c_i32),
                ("bc_right", c_i32), ("newton_maxit", c_i32), ("newton_rtol", c_dbl),
                ("t_end", c_dbl)]


class imexds_batch(ctypes.Structure):
    _fields_ = [("n_problems", c_i32), ("n_cells", P_i32), ("h", P_dbl), ("x_left", P_dbl),
                ("phase_first", P_i32), ("iface_off", P_i32), ("home", P_i32), ("hl", P_dbl)]


class imexds_stats(ctypes.Structure):
    _fields_ = [("steps", c_i64), ("cell_updates", c_i64), ("pseudo_iters", c_i64),
                ("merges", c_i64), ("lmax_hits", c_i64), ("n_failed", c_i32), ("n_active", c_i32),
                ("newton_iters", c_i64), ("iface_solves", c_i64), ("events", c_i64),
                ("gpu_ms", c_dbl), ("pair_zones", c_i64)]


def _sig(name, *args):
    f = getattr(_L, name)
    f.restype = c_i32
    f.argtypes = list(args)
    return f


_ctxpp = ctypes.POINTER(c_vp)
_create = _sig("imexds_create", _ctxpp, ctypes.POINTER(imexds_material),
               ctypes.POINTER(imexds_params), ctypes.POINTER(imexds_batch), c_vp)
_set_state = _sig("imexds_set_state", c_vp, c_vp, c_vp)
_step = _sig("imexds_step", c_vp, c_i32)
_run = _sig("imexds_run", c_vp, c_i32, c_i32, P_i32)
_step_pp = _sig("imexds_step_per_problem", c_vp, c_i32)
_get_state = _sig("imexds_get_state", c_vp, c_vp, c_vp)
_get_ifaces = _sig("imexds_get_interfaces", c_vp, P_i32, P_dbl, P_dbl)
_get_problems = _sig("imexds_get_problems", c_vp, P_dbl, P_i32, P_i64)
_enable_log = _sig("imexds_enable_log", c_vp, c_i32)
_get_log = _sig("imexds_get_log", c_vp, P_i32, P_i32, P_i32, P_i32)
_get_stats = _sig("imexds_get_stats", c_vp, ctypes.POINTER(imexds_stats))
_set_launch = _sig("imexds_set_launch", c_vp, c_i32, c_i32, c_i32, c_i32, c_i32)
_set_zone_solver = _sig("imexds_set_zone_solver", c_vp, c_i32, c_i32, c_dbl)
_autotune = _sig("imexds_autotune", c_vp, c_i32, P_i32, P_i32, P_i32, P_i32, P_dbl)
_get_sizes = _sig("imexds_get_sizes", c_vp, P_i32, P_i32, P_i64)
_last_timing = _sig("imexds_last_timing", c_vp, P_dbl, P_dbl)
_time_bulk = _sig("imexds_time_bulk", c_vp, c_i32)
_kernel_timing = _sig("imexds_kernel_timing", c_vp, P_dbl, P_dbl, P_i32)
_set_tau = _sig("imexds_set_tau", c_vp, c_dbl)
_forward_ckpt = _sig("imexds_forward_ckpt", c_vp, c_i32, c_i32)
_adjoint = _sig("imexds_adjoint", c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp)
_L.imexds_destroy.restype = None
_L.imexds_destroy.argtypes = [c_vp]
_L.imexds_strerror.restype = ctypes.c_char_p
_L.imexds_strerror.argtypes = [c_i32]

EXPORTED = ["imexds_create", "imexds_set_state", "imexds_step", "imexds_run",
            "imexds_step_per_problem", "imexds_get_state", "imexds_get_interfaces",
            "imexds_get_problems", "imexds_enable_log", "imexds_get_log", "imexds_get_stats",
            "imexds_set_launch", "imexds_set_zone_solver", "imexds_autotune", "imexds_get_sizes",
            "imexds_last_timing", "imexds_kernel_timing",
            "imexds_time_bulk", "imexds_set_tau", "imexds_forward_ckpt", "imexds_adjoint",
            "imexds_destroy", "imexds_strerror"]


class IMEXDSError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {imexds_strerror(code)} ({code})")
        self.code = code


def imexds_strerror(code: int) -> str:
    return _L.imexds_strerror(int(code)).decode()


def _check(rc, what):
    if rc != 0:
        raise IMEXDSError(rc, what)


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _dev_ptr(x, n=None):
    """Device address of a contiguous float64 GPU tensor of exactly n
    elements (the library reads or writes that many through it)."""
    import torch
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("expected a contiguous float64 tensor")
    if n is not None and x.numel() != n:
        raise ValueError(f"expected {n} elements, got {x.numel()}")
    if not x.is_cuda:
        raise ValueError("expected a tensor on the GPU")
    return ctypes.c_void_p(x.data_ptr())


# --- ABI functions (same names as include/imexds.h) -------------------------

def imexds_create(material, params, batch, stream=None):
    """Returns an opaque context handle (int).  ``material``/``params`` are the
    workloads dataclasses, ``batch`` a workloads.Batch; ``stream`` a torch
    stream (default: the current one)."""
    import torch
    m = imexds_material(material.a2v, material.a2l, material.p0, material.rhol0, material.tau)
    p = imexds_params(params.cfl, params.zone_half, params.theta_nb, params.tol_mode,
                      params.tol_nb, params.tol_tiny, params.tol_rel, params.lmax,
                      params.alpha_floor, params.merge_safety, params.bc_left, params.bc_right,
                      params.newton_maxit, params.newton_rtol, params.t_end)
    keep = [_np(batch.n_cells, np.int32), _np(batch.h, np.float64), _np(batch.x_left, np.float64),
            _np(batch.phase_first, np.int32), _np(batch.iface_off, np.int32),
            _np(batch.home, np.int32), _np(batch.hl, np.float64)]
    b = imexds_batch(batch.n_problems, _p(keep[0], c_i32), _p(keep[1], c_dbl), _p(keep[2], c_dbl),
                     _p(keep[3], c_i32), _p(keep[4], c_i32), _p(keep[5], c_i32),
                     _p(keep[6], c_dbl))
    s = stream if stream is not None else torch.cuda.current_stream()
    ctx = c_vp()
    _check(_create(ctypes.byref(ctx), ctypes.byref(m), ctypes.byref(p), ctypes.byref(b),
                   c_vp(s.cuda_stream)), "imexds_create")
    return ctx.value


def imexds_set_state(ctx, rho, mom):
    _, _, S = imexds_get_sizes(ctx)
    _check(_set_state(c_vp(ctx), _dev_ptr(rho, S), _dev_ptr(mom, S)), "imexds_set_state")


def imexds_step(ctx, n_steps):
    _check(_step(c_vp(ctx), int(n_steps)), "imexds_step")


def imexds_run(ctx, max_steps, check_every=256):
    done = c_i32(0)
    _check(_run(c_vp(ctx), int(max_steps), int(check_every), ctypes.byref(done)), "imexds_run")
    return done.value


def imexds_step_per_problem(ctx, n_steps):
    _check(_step_pp(c_vp(ctx), int(n_steps)), "imexds_step_per_problem")


def imexds_get_state(ctx, rho, mom):
    _, _, S = imexds_get_sizes(ctx)
    _check(_get_state(c_vp(ctx), _dev_ptr(rho, S), _dev_ptr(mom, S)), "imexds_get_state")


def imexds_get_sizes(ctx):
    P, N, S = c_i32(), c_i32(), c_i64()
    _check(_get_sizes(c_vp(ctx), ctypes.byref(P), ctypes.byref(N), ctypes.byref(S)),
           "imexds_get_sizes")
    return P.value, N.value, S.value


def imexds_get_interfaces(ctx):
    _, N, _ = imexds_get_sizes(ctx)
    home = np.zeros(max(N, 1), np.int32)
    hl = np.zeros(max(N, 1))
    x = np.zeros(max(N, 1))
    _check(_get_ifaces(c_vp(ctx), _p(home, c_i32), _p(hl, c_dbl), _p(x, c_dbl)),
           "imexds_get_interfaces")
    return home[:N], hl[:N], x[:N]


def imexds_get_problems(ctx):
    P, _, _ = imexds_get_sizes(ctx)
    t = np.zeros(max(P, 1))
    st = np.zeros(max(P, 1), np.int32)
    steps = np.zeros(max(P, 1), np.int64)
    _check(_get_problems(c_vp(ctx), _p(t, c_dbl), _p(st, c_i32), _p(steps, c_i64)),
           "imexds_get_problems")
    return t[:P], st[:P], steps[:P]


def imexds_enable_log(ctx, max_steps):
    _check(_enable_log(c_vp(ctx), int(max_steps)), "imexds_enable_log")


def imexds_get_log(ctx, max_rows):
    _, N, _ = imexds_get_sizes(ctx)
    n = max(int(max_rows) * N, 1)
    cnt = np.zeros(n, np.int32)
    fl = np.zeros(n, np.int32)
    zl = np.zeros(n, np.int32)
    rows = c_i32()
    _check(_get_log(c_vp(ctx), _p(cnt, c_i32), _p(fl, c_i32), _p(zl, c_i32), ctypes.byref(rows)),
           "imexds_get_log")
    r = rows.value
    return (cnt[:r * N].reshape(r, N), fl[:r * N].reshape(r, N), zl[:r * N].reshape(r, N))


def imexds_get_stats(ctx):
    s = imexds_stats()
    _check(_get_stats(c_vp(ctx), ctypes.byref(s)), "imexds_get_stats")
    return {n: getattr(s, n) for n, _ in imexds_stats._fields_}


def imexds_set_launch(ctx, tile_cells, zones_per_group, zone_groups, graph_steps, zone_lanes=1):
    _check(_set_launch(c_vp(ctx), int(tile_cells), int(zones_per_group), int(zone_groups),
                       int(graph_steps), int(zone_lanes)), "imexds_set_launch")


ZONE_DTS, ZONE_NEWTON = 0, 1


def imexds_set_zone_solver(ctx, solver, maxit=30, rtol=1e-10):
    _check(_set_zone_solver(c_vp(ctx), int(solver), int(maxit), float(rtol)),
           "imexds_set_zone_solver")


def imexds_autotune(ctx, steps_per_trial):
    t, z, g, n, ms = c_i32(), c_i32(), c_i32(), c_i32(), c_dbl()
    _check(_autotune(c_vp(ctx), int(steps_per_trial), ctypes.byref(t), ctypes.byref(z),
                     ctypes.byref(g), ctypes.byref(n), ctypes.byref(ms)), "imexds_autotune")
    return t.value, z.value, g.value, n.value, ms.value


def imexds_last_timing(ctx):
    a, b = c_dbl(), c_dbl()
    _check(_last_timing(c_vp(ctx), ctypes.byref(a), ctypes.byref(b)), "imexds_last_timing")
    return a.value, b.value


def imexds_time_bulk(ctx, on):
    _check(_time_bulk(c_vp(ctx), int(bool(on))), "imexds_time_bulk")


def imexds_kernel_timing(ctx):
    """(bulk ms, zone ms) per launch and the number of launches of the last
    step call made with imexds_time_bulk on."""
    b, z, n = c_dbl(), c_dbl(), c_i32()
    _check(_kernel_timing(c_vp(ctx), ctypes.byref(b), ctypes.byref(z), ctypes.byref(n)),
           "imexds_kernel_timing")
    return b.value, z.value, n.value


def imexds_set_tau(ctx, tau):
    _check(_set_tau(c_vp(ctx), float(tau)), "imexds_set_tau")


def imexds_forward_ckpt(ctx, n_steps, ckpt_every):
    _check(_forward_ckpt(c_vp(ctx), int(n_steps), int(ckpt_every)), "imexds_forward_ckpt")


def imexds_adjoint(ctx, gL_rho, gL_mom, gL_hl, g_rho0, g_mom0, g_hl0, g_tau):
    """All arguments are FP64 cuda tensors (gL_hl and g_hl0 may be None):
    n_slots elements for the state gradients, n_iface for the interface
    ones, one for g_tau."""
    _, N, S = imexds_get_sizes(ctx)
    opt = (lambda x: _dev_ptr(x, N) if x is not None else c_vp(None))
    _check(_adjoint(c_vp(ctx), _dev_ptr(gL_rho, S), _dev_ptr(gL_mom, S), opt(gL_hl),
                    _dev_ptr(g_rho0, S), _dev_ptr(g_mom0, S), opt(g_hl0), _dev_ptr(g_tau, 1)),
           "imexds_adjoint")


def imexds_destroy(ctx):
    if ctx:
        _L.imexds_destroy(c_vp(ctx))


class IMEXDS:
    """Context holder: a batch of problems, its state and its stepping."""

    def __init__(self, batch, material, params, stream=None):
        import torch
        self.batch = batch
        self.material = material
        self.params = params
        self.ctx = imexds_create(material, params, batch, stream)
        self.n_slots = batch.n_slots
        self._torch = torch
        # bumped by every call that replaces what a checkpointed forward
        # recorded, so that a backward can tell whether it still has its own
        self.generation = 0

    def set_state(self, rho=None, mom=None):
        torch = self._torch
        if rho is None:
            rho = torch.from_numpy(np.ascontiguousarray(self.batch.rho, np.float64)).cuda()
            mom = torch.from_numpy(np.ascontiguousarray(self.batch.mom, np.float64)).cuda()
        imexds_set_state(self.ctx, rho, mom)
        self.generation += 1

    def step(self, n):
        imexds_step(self.ctx, n)
        self.generation += 1

    def run(self, max_steps, check_every=256):
        self.generation += 1
        return imexds_run(self.ctx, max_steps, check_every)

    def step_per_problem(self, n):
        imexds_step_per_problem(self.ctx, n)
        self.generation += 1

    def state(self):
        torch = self._torch
        rho = torch.empty(self.n_slots, dtype=torch.float64, device="cuda")
        mom = torch.empty_like(rho)
        imexds_get_state(self.ctx, rho, mom)
        return rho, mom

    def state_numpy(self):
        rho, mom = self.state()
        self._torch.cuda.synchronize()
        return rho.cpu().numpy(), mom.cpu().numpy()

    def interfaces(self):
        return imexds_get_interfaces(self.ctx)

    def problems(self):
        return imexds_get_problems(self.ctx)

    def enable_log(self, max_steps):
        self._log_max = int(max_steps)
        imexds_enable_log(self.ctx, max_steps)

    def log(self):
        return imexds_get_log(self.ctx, getattr(self, "_log_max", 0))

    def stats(self):
        return imexds_get_stats(self.ctx)

    def set_launch(self, tile_cells=1024, zones_per_group=16, zone_groups=0, graph_steps=8,
                   zone_lanes=1):
        imexds_set_launch(self.ctx, tile_cells, zones_per_group, zone_groups, graph_steps,
                          zone_lanes)

    def set_zone_solver(self, solver, maxit=30, rtol=1e-10):
        imexds_set_zone_solver(self.ctx, solver, maxit, rtol)

    def autotune(self, steps_per_trial=10):
        return imexds_autotune(self.ctx, steps_per_trial)

    def last_timing(self):
        return imexds_last_timing(self.ctx)

    def time_bulk(self, on=True):
        imexds_time_bulk(self.ctx, on)

    def kernel_timing(self):
        return imexds_kernel_timing(self.ctx)

    def set_tau(self, tau):
        imexds_set_tau(self.ctx, tau)
        self.generation += 1

    def forward_ckpt(self, n_steps, ckpt_every):
        imexds_forward_ckpt(self.ctx, n_steps, ckpt_every)
        self.generation += 1

    def adjoint(self, g_rho, g_mom, g_hl=None):
        """dL/d(rho0, mom0, hl0, tau) of the last forward_ckpt, given dL/d of
        its end state (cuda FP64 tensors)."""
        torch = self._torch
        g_rho0 = torch.empty(self.n_slots, dtype=torch.float64, device="cuda")
        g_mom0 = torch.empty_like(g_rho0)
        n = max(self.batch.n_iface, 1)
        g_hl0 = torch.empty(n, dtype=torch.float64, device="cuda")
        g_tau = torch.empty(1, dtype=torch.float64, device="cuda")
        if g_hl is not None and self.batch.n_iface == 0:
            g_hl = None
        imexds_adjoint(self.ctx, g_rho.contiguous(), g_mom.contiguous(),
                       None if g_hl is None else g_hl.contiguous(), g_rho0, g_mom0,
                       g_hl0 if self.batch.n_iface else None, g_tau)
        return g_rho0, g_mom0, g_hl0[:self.batch.n_iface], g_tau

    def close(self):
        if self.ctx:
            imexds_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
