"""Counters of imexds_get_stats and the kernel timing of imexds_time_bulk /
imexds_kernel_timing on the GPU, checked against the per-step logs (which
are themselves compared with the oracle in the parity tests) and against
each other across the two zone kernels, which make the same interface
solves in the same order."""
import numpy as np
import pytest

from parity import run_gpu, run_oracle
from paper_2211_00705_amd import workloads as W

pytestmark = pytest.mark.gpu

FL_MERGED, FL_REDO, FL_CROSS_L, FL_CROSS_R, FL_FAIL, FL_INACTIVE = 2, 4, 16, 32, 64, 128


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_00705_amd import imexds  # noqa: F401


def _events(flags):
    ok = (flags & (FL_FAIL | FL_INACTIVE)) == 0
    f = flags[ok]
    return (int(np.sum((f & FL_MERGED) > 0)), int(np.sum((f & FL_REDO) > 0)),
            int(np.sum((f & (FL_CROSS_L | FL_CROSS_R)) > 0)))


@pytest.mark.parametrize("work", ["random", "bubble"])
def test_counters_match_the_logs_and_both_zone_kernels(material, work):
    if work == "random":
        b = W.random_batch(seed=12, n_problems=48, nmin=64, nmax=2000)
        P = W.random_batch_params()
    else:
        b = W.bubble_batch(seed=3, n_problems=12, n=512)
        P = W.bubble_batch_params()
    n = 200
    runs = [run_gpu(b, material, P, n, lanes=lanes) for lanes in (1, 8)]
    o = run_oracle(b, material, P, n)
    merges, redos, crosses = _events(o["flags"])
    assert merges > 0
    for g in runs:
        st = g["stats"]
        assert st["pseudo_iters"] == int(np.sum(o["count"]))
        assert st["merges"] == merges
        assert st["events"] == merges + redos + crosses
        assert st["lmax_hits"] == int(np.sum((o["flags"] & 8) > 0))
        # one solve for the prediction, one per dual time iteration and one
        # for Part 2 per zone step; a redone zone adds its first attempt's
        active = int(np.sum((o["flags"] & (FL_FAIL | FL_INACTIVE)) == 0))
        base = int(np.sum(o["count"])) + 2 * active
        assert st["iface_solves"] >= base
        if redos == 0:
            assert st["iface_solves"] == base
        # every solve evaluates G at its start point and after each step but
        # the last (which is applied to first order)
        assert st["iface_solves"] <= st["newton_iters"] <= 8 * st["iface_solves"]
        assert st["gpu_ms"] > 0.0
    for key in ("pseudo_iters", "merges", "events", "iface_solves", "newton_iters"):
        assert runs[0]["stats"][key] == runs[1]["stats"][key], key


def test_kernel_timing_and_device_time(material):
    import torch
    from paper_2211_00705_amd.imexds import IMEXDS
    b = W.random_batch(seed=5, n_problems=64, nmin=256, nmax=4096)
    s = IMEXDS(b, material, W.random_batch_params())
    try:
        s.set_launch(zone_lanes=8)
        s.set_state()
        s.time_bulk(True)
        s.step(30)
        torch.cuda.synchronize()
        total, bulk1 = s.last_timing()
        bulk, zone, n = s.kernel_timing()
        assert n == 30 and bulk > 0.0 and zone > 0.0
        assert bulk == pytest.approx(bulk1, rel=1e-9)
        assert 30 * (bulk + zone) <= total * 1.05
        s.time_bulk(False)
        s.step(20)
        torch.cuda.synchronize()
        t2, _ = s.last_timing()
        st = s.stats()
        # device time of both stepping calls since set_state
        assert st["gpu_ms"] == pytest.approx(total + t2, rel=0.05)
    finally:
        s.close()
