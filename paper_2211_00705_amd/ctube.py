"""ctypes binding of the creation-tube entry points of libimexds.so
(include/imexds_ctube.h): one function per C function, argument marshalling
only, and ``CreationTubes``, a holder of the context.  Device pointers come
from contiguous FP64 torch tensors on cuda.  There is no CPU fallback:
importing this module fails if the library is missing.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import imexds as _base

_L = _base._L
_check = _base._check
_dev_ptr = _base._dev_ptr
_np, _p = _base._np, _base._p
c_i32, c_i64, c_dbl, c_vp = _base.c_i32, _base.c_i64, _base.c_dbl, _base.c_vp
P_i32, P_i64, P_dbl = _base.P_i32, _base.P_i64, _base.P_dbl

ST_NEWTON, ST_NONPHYS, ST_MESH, ST_MULTI = 1, 2, 4, 8
FL_CREATED, FL_LMAX, FL_INACTIVE = 1, 2, 4
SOLVER_DTS, SOLVER_NEWTON = 0, 1


class imexds_ct_batch(ctypes.Structure):
    _fields_ = [("n_problems", c_i32), ("n_cells", P_i32), ("h", P_dbl), ("phase", P_i32)]


def _sig(name, *args):
    f = getattr(_L, name)
    f.restype = c_i32
    f.argtypes = list(args)
    return f


_create = _sig("imexds_ct_create", ctypes.POINTER(c_vp), ctypes.POINTER(_base.imexds_material),
               ctypes.POINTER(_base.imexds_params), c_dbl, c_dbl,
               ctypes.POINTER(imexds_ct_batch), c_vp)
_set_state = _sig("imexds_ct_set_state", c_vp, c_vp, c_vp)
_step = _sig("imexds_ct_step", c_vp, c_i32)
_step_pp = _sig("imexds_ct_step_per_problem", c_vp, c_i32)
_run = _sig("imexds_ct_run", c_vp, c_i32, c_i32, P_i32)
_get_state = _sig("imexds_ct_get_state", c_vp, c_vp, c_vp)
_get_problems = _sig("imexds_ct_get_problems", c_vp, P_dbl, P_i32, P_i32, P_i64, P_i32, P_dbl,
                     P_dbl)
_enable_log = _sig("imexds_ct_enable_log", c_vp, c_i32)
_get_log = _sig("imexds_ct_get_log", c_vp, P_i32, P_i32, P_i32)
_set_launch = _sig("imexds_ct_set_launch", c_vp, c_i32, c_i32)
_set_solver = _sig("imexds_ct_set_solver", c_vp, c_i32, c_i32, c_dbl)
_get_sizes = _sig("imexds_ct_get_sizes", c_vp, P_i32, P_i64)
_time_kernels = _sig("imexds_ct_time_kernels", c_vp, c_i32)
_last_timing = _sig("imexds_ct_last_timing", c_vp, P_dbl, P_dbl, P_dbl)
_L.imexds_ct_destroy.restype = None
_L.imexds_ct_destroy.argtypes = [c_vp]

EXPORTED = ["imexds_ct_create", "imexds_ct_set_state", "imexds_ct_step",
            "imexds_ct_step_per_problem", "imexds_ct_run",
            "imexds_ct_get_state", "imexds_ct_get_problems", "imexds_ct_enable_log",
            "imexds_ct_get_log", "imexds_ct_set_launch", "imexds_ct_set_solver",
            "imexds_ct_get_sizes",
            "imexds_ct_time_kernels", "imexds_ct_last_timing", "imexds_ct_destroy"]


def imexds_ct_create(batch, stream=None):
    """``batch``: a ctube_workloads.CTubeBatch.  Returns the context handle."""
    import torch
    m, pr = batch.material, batch.params
    mat = _base.imexds_material(m.a2v, m.a2l, m.p0, m.rhol0, m.tau)
    par = _base.imexds_params(pr.cfl, pr.zone_half, pr.theta_nb, pr.tol_mode, pr.tol_nb,
                              pr.tol_tiny, pr.tol_rel, pr.lmax, pr.alpha_floor, pr.merge_safety,
                              pr.bc_left, pr.bc_right, pr.newton_maxit, pr.newton_rtol, pr.t_end)
    keep = [_np(batch.N, np.int32), _np(batch.h, np.float64), _np(batch.phase, np.int32)]
    b = imexds_ct_batch(batch.n_problems, _p(keep[0], c_i32), _p(keep[1], c_dbl),
                        _p(keep[2], c_i32))
    s = stream if stream is not None else torch.cuda.current_stream()
    ctx = c_vp()
    _check(_create(ctypes.byref(ctx), ctypes.byref(mat), ctypes.byref(par), float(batch.p_min),
                   float(batch.p_tilde), ctypes.byref(b), c_vp(s.cuda_stream)),
           "imexds_ct_create")
    return ctx.value


def imexds_ct_set_state(ctx, rho, mom):
    _, n = imexds_ct_get_sizes(ctx)
    _check(_set_state(c_vp(ctx), _dev_ptr(rho, n), _dev_ptr(mom, n)), "imexds_ct_set_state")


def imexds_ct_step(ctx, n_steps):
    _check(_step(c_vp(ctx), int(n_steps)), "imexds_ct_step")


def imexds_ct_step_per_problem(ctx, n_steps):
    _check(_step_pp(c_vp(ctx), int(n_steps)), "imexds_ct_step_per_problem")


def imexds_ct_run(ctx, max_steps, check_every=64):
    done = c_i32(0)
    _check(_run(c_vp(ctx), int(max_steps), int(check_every), ctypes.byref(done)),
           "imexds_ct_run")
    return done.value


def imexds_ct_get_state(ctx, rho, mom):
    _, n = imexds_ct_get_sizes(ctx)
    _check(_get_state(c_vp(ctx), _dev_ptr(rho, n), _dev_ptr(mom, n)), "imexds_ct_get_state")


def imexds_ct_get_sizes(ctx):
    P, n = c_i32(), c_i64()
    _check(_get_sizes(c_vp(ctx), ctypes.byref(P), ctypes.byref(n)), "imexds_ct_get_sizes")
    return P.value, n.value


def imexds_ct_get_problems(ctx):
    """(t, status, steps, iters, face, dl, dr), numpy arrays of n_problems."""
    P, _ = imexds_ct_get_sizes(ctx)
    n = max(P, 1)
    t, dl, dr = np.zeros(n), np.zeros(n), np.zeros(n)
    st, steps, face = np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32)
    iters = np.zeros(n, np.int64)
    _check(_get_problems(c_vp(ctx), _p(t, c_dbl), _p(st, c_i32), _p(steps, c_i32),
                         _p(iters, c_i64), _p(face, c_i32), _p(dl, c_dbl), _p(dr, c_dbl)),
           "imexds_ct_get_problems")
    return t[:P], st[:P], steps[:P], iters[:P], face[:P], dl[:P], dr[:P]


def imexds_ct_enable_log(ctx, max_steps):
    _check(_enable_log(c_vp(ctx), int(max_steps)), "imexds_ct_enable_log")


def imexds_ct_get_log(ctx, max_rows):
    P, _ = imexds_ct_get_sizes(ctx)
    n = max(int(max_rows) * P, 1)
    cnt = np.zeros(n, np.int32)
    fl = np.zeros(n, np.int32)
    rows = c_i32()
    _check(_get_log(c_vp(ctx), _p(cnt, c_i32), _p(fl, c_i32), ctypes.byref(rows)),
           "imexds_ct_get_log")
    r = rows.value
    return cnt[:r * P].reshape(r, P), fl[:r * P].reshape(r, P)


def imexds_ct_set_launch(ctx, zone_lanes, zone_problems_per_wave):
    _check(_set_launch(c_vp(ctx), int(zone_lanes), int(zone_problems_per_wave)),
           "imexds_ct_set_launch")


def imexds_ct_set_solver(ctx, solver, maxit=30, rtol=1e-10):
    _check(_set_solver(c_vp(ctx), int(solver), int(maxit), float(rtol)), "imexds_ct_set_solver")


def imexds_ct_time_kernels(ctx, on):
    _check(_time_kernels(c_vp(ctx), int(bool(on))), "imexds_ct_time_kernels")


def imexds_ct_last_timing(ctx):
    a, b, s = c_dbl(), c_dbl(), c_dbl()
    _check(_last_timing(c_vp(ctx), ctypes.byref(a), ctypes.byref(b), ctypes.byref(s)),
           "imexds_ct_last_timing")
    return a.value, b.value, s.value


def imexds_ct_destroy(ctx):
    if ctx:
        _L.imexds_ct_destroy(c_vp(ctx))


class CreationTubes:
    """Context holder for a CTubeBatch."""

    def __init__(self, batch, stream=None):
        import torch
        self.batch = batch
        self.ctx = imexds_ct_create(batch, stream)
        self.n_slots = batch.n_slots
        self._torch = torch
        self._log_max = 0

    def set_state(self, rho=None, mom=None):
        torch = self._torch
        if rho is None:
            rho, mom = (torch.from_numpy(np.ascontiguousarray(getattr(self.batch, f),
                                                              np.float64)).cuda()
                        for f in ("rho", "mom"))
        imexds_ct_set_state(self.ctx, rho, mom)

    def step(self, n):
        imexds_ct_step(self.ctx, n)

    def step_per_problem(self, n):
        imexds_ct_step_per_problem(self.ctx, n)

    def run(self, max_steps=1 << 30, check_every=64):
        return imexds_ct_run(self.ctx, max_steps, check_every)

    def state(self):
        torch = self._torch
        out = [torch.empty(self.n_slots, dtype=torch.float64, device="cuda") for _ in range(2)]
        imexds_ct_get_state(self.ctx, *out)
        return tuple(out)

    def state_numpy(self):
        out = self.state()
        self._torch.cuda.synchronize()
        return tuple(x.cpu().numpy() for x in out)

    def problems(self):
        return imexds_ct_get_problems(self.ctx)

    def enable_log(self, max_steps):
        self._log_max = int(max_steps)
        imexds_ct_enable_log(self.ctx, max_steps)

    def log(self):
        return imexds_ct_get_log(self.ctx, self._log_max)

    def set_launch(self, zone_lanes=4, zone_problems_per_wave=2):
        imexds_ct_set_launch(self.ctx, zone_lanes, zone_problems_per_wave)

    def set_solver(self, solver, maxit=30, rtol=1e-10):
        imexds_ct_set_solver(self.ctx, solver, maxit, rtol)

    def time_kernels(self, on=True):
        imexds_ct_time_kernels(self.ctx, on)

    def last_timing(self):
        return imexds_ct_last_timing(self.ctx)

    def close(self):
        if self.ctx:
            imexds_ct_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
