"""The entry point that allocates nothing (imexds_creation_rp_noalloc),
through the C ABI: on two calls in a row, the second with fewer problems, its
statuses and output records are bitwise those of imexds_creation_rp on the
same inputs; more problems than its fixed scratch holds are refused before
anything is launched."""
import numpy as np
import pytest

from paper_2211_00705_amd import workloads as W

pytestmark = pytest.mark.gpu

M = W.WATER_363K


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _inputs(b):
    import torch
    return (_dev(b.phase, torch.int32), _dev(b.rho_l, torch.float64),
            _dev(b.mom_l, torch.float64), _dev(b.rho_r, torch.float64),
            _dev(b.mom_r, torch.float64))


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    import torch
    from paper_2211_00705_amd.creation import (NOALLOC_MAX, imexds_creation_rp,
                                               imexds_creation_rp_noalloc)
    for seed, n in ((11, NOALLOC_MAX), (12, 5000)):
        print(f"noalloc: seed {seed}, {n} problems", flush=True)
        b = W.creation_batch(M, seed=seed, n=n)
        args = _inputs(b)
        # outputs preallocated and poisoned, so that stale values would show
        st_na = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        out_na = torch.full((n, 20), float("nan"), dtype=torch.float64, device="cuda")
        imexds_creation_rp_noalloc(M, *args, W.P_MIN, W.P_TILDE, status=st_na, out=out_na)
        st, out = imexds_creation_rp(M, *args, W.P_MIN, W.P_TILDE)
        torch.cuda.synchronize()
        st_na, out_na, st, out = (x.cpu().numpy() for x in (st_na, out_na, st, out))
        assert np.array_equal(st_na, st)
        assert np.array_equal(out_na.view(np.uint64), out.view(np.uint64))
        # both phases create and both do not, so every queue is used
        for ph in (W.LIQ, W.VAP):
            for s in (0, 1):
                assert np.sum((b.phase == ph) & (st == s)) > 0


def test_noalloc_refuses_more_than_its_maximum():
    import torch
    from paper_2211_00705_amd.creation import NOALLOC_MAX, imexds_creation_rp_noalloc
    from paper_2211_00705_amd.imexds import IMEXDSError
    n = NOALLOC_MAX + 1
    z = torch.ones(n, dtype=torch.float64, device="cuda")
    ph = torch.zeros(n, dtype=torch.int32, device="cuda")
    st = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(IMEXDSError, match="fixed maximum"):
        imexds_creation_rp_noalloc(M, ph, z, z, z, z, W.P_MIN, W.P_TILDE, status=st)
    torch.cuda.synchronize()
    assert bool((st == -7).all())  # nothing ran
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    s0, o0 = imexds_creation_rp_noalloc(M, torch.zeros(0, dtype=torch.int32, device="cuda"), e,
                                        e, e, e, W.P_MIN, W.P_TILDE)
    assert s0.shape == (0,) and o0.shape == (0, 20)
