"""ctypes binding of the full-Euler entry points of libimexds.so
(include/imexds_euler.h): one function per C function, argument marshalling
only, and ``EulerIMEXDS``, a holder of the context.  Device pointers come from
contiguous FP64 torch tensors on cuda.  There is no CPU fallback: importing
this module fails if the library is missing.
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

ST_VACUUM, ST_NEWTON, ST_NONPHYS = 1, 2, 4
FL_LMAX = 1


class imexds_eu_params(ctypes.Structure):
    _fields_ = [("gamma", c_dbl), ("tol_nb", c_dbl), ("tol_k", c_dbl), ("lmax", c_i32)]


class imexds_eu_batch(ctypes.Structure):
    _fields_ = [("n_problems", c_i32), ("N", P_i32), ("h", P_dbl), ("alpha", P_dbl),
                ("theta_nb", P_dbl), ("theta_k", P_dbl), ("cfl", P_dbl), ("t_end", P_dbl)]


def _sig(name, *args):
    f = getattr(_L, name)
    f.restype = c_i32
    f.argtypes = list(args)
    return f


_create = _sig("imexds_eu_create", ctypes.POINTER(c_vp), ctypes.POINTER(imexds_eu_params),
               ctypes.POINTER(imexds_eu_batch), c_vp)
_set_state = _sig("imexds_eu_set_state", c_vp, c_vp, c_vp, c_vp)
_step = _sig("imexds_eu_step", c_vp, c_i32)
_run = _sig("imexds_eu_run", c_vp, c_i32, c_i32, P_i32)
_step_pp = _sig("imexds_eu_step_per_problem", c_vp, c_i32)
_get_state = _sig("imexds_eu_get_state", c_vp, c_vp, c_vp, c_vp)
_get_problems = _sig("imexds_eu_get_problems", c_vp, P_dbl, P_i32, P_i32, P_i64)
_enable_log = _sig("imexds_eu_enable_log", c_vp, c_i32)
_get_log = _sig("imexds_eu_get_log", c_vp, P_i32, P_i32, P_i32)
_set_launch = _sig("imexds_eu_set_launch", c_vp, c_i32, c_i32, c_i32)
_get_sizes = _sig("imexds_eu_get_sizes", c_vp, P_i32, P_i64)
_time_kernels = _sig("imexds_eu_time_kernels", c_vp, c_i32)
_last_timing = _sig("imexds_eu_last_timing", c_vp, P_dbl, P_dbl, P_dbl)
_L.imexds_eu_destroy.restype = None
_L.imexds_eu_destroy.argtypes = [c_vp]

EXPORTED = ["imexds_eu_create", "imexds_eu_set_state", "imexds_eu_step",
            "imexds_eu_step_per_problem", "imexds_eu_run",
            "imexds_eu_get_state", "imexds_eu_get_problems", "imexds_eu_enable_log",
            "imexds_eu_get_log", "imexds_eu_set_launch", "imexds_eu_get_sizes",
            "imexds_eu_time_kernels", "imexds_eu_last_timing", "imexds_eu_destroy"]


def imexds_eu_create(batch, stream=None):
    """``batch``: an euler_workloads.EulerBatch.  Returns the context handle."""
    import torch
    par = imexds_eu_params(batch.gamma, batch.tol_nb, batch.tol_k, int(batch.lmax))
    keep = [_np(batch.N, np.int32)] + [_np(getattr(batch, f), np.float64) for f in
                                       ("h", "alpha", "theta_nb", "theta_k", "cfl", "t_end")]
    b = imexds_eu_batch(batch.n_problems, _p(keep[0], c_i32),
                        *[_p(a, c_dbl) for a in keep[1:]])
    s = stream if stream is not None else torch.cuda.current_stream()
    ctx = c_vp()
    _check(_create(ctypes.byref(ctx), ctypes.byref(par), ctypes.byref(b), c_vp(s.cuda_stream)),
           "imexds_eu_create")
    return ctx.value


def imexds_eu_set_state(ctx, rho, mom, ene):
    _, n = imexds_eu_get_sizes(ctx)
    _check(_set_state(c_vp(ctx), _dev_ptr(rho, n), _dev_ptr(mom, n), _dev_ptr(ene, n)),
           "imexds_eu_set_state")


def imexds_eu_step(ctx, n_steps):
    _check(_step(c_vp(ctx), int(n_steps)), "imexds_eu_step")


def imexds_eu_step_per_problem(ctx, n_steps):
    _check(_step_pp(c_vp(ctx), int(n_steps)), "imexds_eu_step_per_problem")


def imexds_eu_run(ctx, max_steps, check_every=64):
    done = c_i32(0)
    _check(_run(c_vp(ctx), int(max_steps), int(check_every), ctypes.byref(done)),
           "imexds_eu_run")
    return done.value


def imexds_eu_get_state(ctx, rho, mom, ene):
    _, n = imexds_eu_get_sizes(ctx)
    _check(_get_state(c_vp(ctx), _dev_ptr(rho, n), _dev_ptr(mom, n), _dev_ptr(ene, n)),
           "imexds_eu_get_state")


def imexds_eu_get_sizes(ctx):
    P, n = c_i32(), c_i64()
    _check(_get_sizes(c_vp(ctx), ctypes.byref(P), ctypes.byref(n)), "imexds_eu_get_sizes")
    return P.value, n.value


def imexds_eu_get_problems(ctx):
    P, _ = imexds_eu_get_sizes(ctx)
    t = np.zeros(max(P, 1))
    st = np.zeros(max(P, 1), np.int32)
    steps = np.zeros(max(P, 1), np.int32)
    iters = np.zeros(max(P, 1), np.int64)
    _check(_get_problems(c_vp(ctx), _p(t, c_dbl), _p(st, c_i32), _p(steps, c_i32),
                         _p(iters, c_i64)), "imexds_eu_get_problems")
    return t[:P], st[:P], steps[:P], iters[:P]


def imexds_eu_enable_log(ctx, max_steps):
    _check(_enable_log(c_vp(ctx), int(max_steps)), "imexds_eu_enable_log")


def imexds_eu_get_log(ctx, max_rows):
    P, _ = imexds_eu_get_sizes(ctx)
    n = max(int(max_rows) * P, 1)
    cnt = np.zeros(n, np.int32)
    fl = np.zeros(n, np.int32)
    rows = c_i32()
    _check(_get_log(c_vp(ctx), _p(cnt, c_i32), _p(fl, c_i32), ctypes.byref(rows)),
           "imexds_eu_get_log")
    r = rows.value
    return cnt[:r * P].reshape(r, P), fl[:r * P].reshape(r, P)


def imexds_eu_set_launch(ctx, tile_cells, zone_lanes, zone_problems_per_wave):
    _check(_set_launch(c_vp(ctx), int(tile_cells), int(zone_lanes), int(zone_problems_per_wave)),
           "imexds_eu_set_launch")


def imexds_eu_time_kernels(ctx, on):
    _check(_time_kernels(c_vp(ctx), int(bool(on))), "imexds_eu_time_kernels")


def imexds_eu_last_timing(ctx):
    a, b, s = c_dbl(), c_dbl(), c_dbl()
    _check(_last_timing(c_vp(ctx), ctypes.byref(a), ctypes.byref(b), ctypes.byref(s)),
           "imexds_eu_last_timing")
    return a.value, b.value, s.value


def imexds_eu_destroy(ctx):
    if ctx:
        _L.imexds_eu_destroy(c_vp(ctx))


class EulerIMEXDS:
    """Context holder for an EulerBatch."""

    def __init__(self, batch, stream=None):
        import torch
        self.batch = batch
        self.ctx = imexds_eu_create(batch, stream)
        self.n_cells = batch.n_cells
        self._torch = torch
        self._log_max = 0

    def set_state(self, rho=None, mom=None, ene=None):
        torch = self._torch
        if rho is None:
            rho, mom, ene = (torch.from_numpy(np.ascontiguousarray(getattr(self.batch, f),
                                                                   np.float64)).cuda()
                             for f in ("rho", "mom", "ene"))
        imexds_eu_set_state(self.ctx, rho, mom, ene)

    def step(self, n):
        imexds_eu_step(self.ctx, n)

    def step_per_problem(self, n):
        imexds_eu_step_per_problem(self.ctx, n)

    def run(self, max_steps=1 << 30, check_every=64):
        return imexds_eu_run(self.ctx, max_steps, check_every)

    def state(self):
        torch = self._torch
        out = [torch.empty(self.n_cells, dtype=torch.float64, device="cuda") for _ in range(3)]
        imexds_eu_get_state(self.ctx, *out)
        return tuple(out)

    def state_numpy(self):
        out = self.state()
        self._torch.cuda.synchronize()
        return tuple(x.cpu().numpy() for x in out)

    def problems(self):
        return imexds_eu_get_problems(self.ctx)

    def enable_log(self, max_steps):
        self._log_max = int(max_steps)
        imexds_eu_enable_log(self.ctx, max_steps)

    def log(self):
        return imexds_eu_get_log(self.ctx, self._log_max)

    def set_launch(self, tile_cells=1024, zone_lanes=2, zone_problems_per_wave=32):
        imexds_eu_set_launch(self.ctx, tile_cells, zone_lanes, zone_problems_per_wave)

    def time_kernels(self, on=True):
        imexds_eu_time_kernels(self.ctx, on)

    def last_timing(self):
        return imexds_eu_last_timing(self.ctx)

    def close(self):
        if self.ctx:
            imexds_eu_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
