"""ctypes binding of imexds_creation_rp (include/imexds_creation.h): argument
marshalling only.  Inputs and outputs are contiguous torch tensors on cuda;
there is no CPU fallback."""
from __future__ import annotations

import ctypes

from . import imexds as _base

_L = _base._L
c_i32, c_dbl, c_vp = _base.c_i32, _base.c_dbl, _base.c_vp

FIELDS = ("kind", "p1", "pa", "pb", "pc", "ra", "rb", "rc", "ua", "ub", "uc", "zl", "zr", "wl",
          "wr", "Fl0", "Fl1", "Fr0", "Fr1", "iters")

_creation = getattr(_L, "imexds_creation_rp")
_creation.restype = c_i32
_creation.argtypes = [ctypes.POINTER(_base.imexds_material), c_i32, c_vp, c_vp, c_vp, c_vp, c_vp,
                      c_dbl, c_dbl, c_i32, c_dbl, c_vp, c_vp, c_vp]

_creation_na = getattr(_L, "imexds_creation_rp_noalloc")
_creation_na.restype = c_i32
_creation_na.argtypes = _creation.argtypes

EXPORTED = ["imexds_creation_rp", "imexds_creation_rp_noalloc"]

# largest problem count of imexds_creation_rp_noalloc
NOALLOC_MAX = 1 << 20


def _dev(x, dtype, n):
    """Device address of a contiguous GPU tensor of that dtype and exactly n
    elements (the library reads or writes that many through it)."""
    import torch
    if not isinstance(x, torch.Tensor) or x.dtype != dtype or not x.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor")
    if x.numel() != n:
        raise ValueError(f"expected {n} elements, got {x.numel()}")
    if not x.is_cuda:
        raise ValueError("expected a tensor on the GPU")
    return c_vp(x.data_ptr())


def imexds_creation_rp(material, phase, rho_l, mom_l, rho_r, mom_r, p_min, p_tilde, maxit=50,
                       rtol=1e-14, status=None, out=None, stream=None):
    """Returns (status int32 [n], out float64 [n, 20]) as cuda tensors."""
    return _call(_creation, "imexds_creation_rp", material, phase, rho_l, mom_l, rho_r, mom_r,
                 p_min, p_tilde, maxit, rtol, status, out, stream)


def imexds_creation_rp_noalloc(material, phase, rho_l, mom_l, rho_r, mom_r, p_min, p_tilde,
                               maxit=50, rtol=1e-14, status=None, out=None, stream=None):
    """As imexds_creation_rp, through the entry point that allocates no
    device memory (its scratch is a fixed array of the library; at most
    NOALLOC_MAX problems).  Pass preallocated ``status`` and ``out`` where
    allocation must be avoided altogether."""
    return _call(_creation_na, "imexds_creation_rp_noalloc", material, phase, rho_l, mom_l,
                 rho_r, mom_r, p_min, p_tilde, maxit, rtol, status, out, stream)


def _call(fn, name, material, phase, rho_l, mom_l, rho_r, mom_r, p_min, p_tilde, maxit, rtol,
          status, out, stream):
    import torch
    n = int(phase.shape[0])
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device="cuda")
    if out is None:
        out = torch.empty((n, len(FIELDS)), dtype=torch.float64, device="cuda")
    m = _base.imexds_material(material.a2v, material.a2l, material.p0, material.rhol0,
                              material.tau)
    s = stream if stream is not None else torch.cuda.current_stream()
    d = torch.float64
    nf = n * len(FIELDS)
    _base._check(fn(ctypes.byref(m), n, _dev(phase, torch.int32, n), _dev(rho_l, d, n),
                    _dev(mom_l, d, n), _dev(rho_r, d, n), _dev(mom_r, d, n), float(p_min),
                    float(p_tilde), int(maxit), float(rtol), _dev(status, torch.int32, n),
                    _dev(out, d, nf), c_vp(s.cuda_stream)), name)
    return status, out
