"""HIP path vs CPU oracle, element by element, through the C ABI.

Bar: rel-L1 <= 1e-10 per problem and component (FP64), identical interface
cells, statuses, step counts, dual-time iteration counts, event flags and
zone partitions for every step and interface.
"""
import math

import numpy as np
import pytest

from parity import assert_parity, run_gpu, run_oracle, take_problems
from paper_2211_00705_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_00705_amd import imexds  # noqa: F401  (fails loudly if the library is missing)


def test_constant_states_are_preserved_bitwise(material):
    b = W.single_phase_problem(1000, lambda x: np.full(x.shape, 970.0), lambda x: np.zeros(x.shape))
    g = run_gpu(b, material, W.Params(), 50, log=False)
    assert np.array_equal(g["rho"], b.rho) and np.array_equal(g["mom"], b.mom)
    assert g["steps"][0] == 50


def test_single_phase_matches_oracle_bitwise(material):
    b = W.single_phase_problem(3000, lambda x: 900.0 + 80.0 * np.sin(6 * x) ** 2,
                               lambda x: 20.0 * np.cos(9 * x))
    P = W.Params(bc_left=1, bc_right=0)
    g = run_gpu(b, material, P, 120)
    o = run_oracle(b, material, P, 120)
    assert np.array_equal(g["rho"], o["rho"]) and np.array_equal(g["mom"], o["mom"])
    assert_parity(b, g, o)


LANES = [1, 8]  # lanes per zone: k_zone, k_zone8


@pytest.mark.parametrize("lanes", LANES)
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_single_cut_problem(material, seed, lanes):
    """200 cells, cut fraction 1e-4, relative-update dual time stepping."""
    b = W.single_cut_problem(seed)
    P = W.single_cut_params()
    g = run_gpu(b, material, P, 400, lanes=lanes)
    o = run_oracle(b, material, P, 400)
    assert np.all(o["status"] == 0)
    assert_parity(b, g, o)


@pytest.mark.parametrize("lanes", LANES)
@pytest.mark.parametrize("zone_half", [1, 2, 3])
def test_random_batch(material, zone_half, lanes):
    """Uneven problems spanning several tiles with ragged tails, paper's
    stopping rule, interfaces crossing cells and tiny pieces merging."""
    b = W.random_batch(seed=3 + zone_half, n_problems=40, nmin=64, nmax=3000)
    P = W.random_batch_params().replace(zone_half=zone_half)
    g = run_gpu(b, material, P, 300, lanes=lanes)
    o = run_oracle(b, material, P, 300)
    assert np.all(o["status"] == 0)
    ev = (o["flags"] & 2) > 0  # merged
    assert ev.sum() > 20  # merges happened
    assert_parity(b, g, o)


@pytest.mark.parametrize("lanes", LANES)
def test_bubble_batch(material, lanes):
    b = W.bubble_batch(seed=7, n_problems=12, n=512)
    P = W.bubble_batch_params()
    g = run_gpu(b, material, P, 300, lanes=lanes)
    o = run_oracle(b, material, P, 300)
    assert_parity(b, g, o)


def test_launch_forms_agree_bitwise(material):
    """Batched graph replay, direct launches, per-problem launches and every
    tile size give bit-identical results."""
    b = W.random_batch(seed=21, n_problems=16, nmin=100, nmax=5000)
    P = W.random_batch_params()
    ref = run_gpu(b, material, P, 64, launch=(1024, 16, 0, 8))
    for launch in [(256, 1, 0, 0), (512, 64, 0, 2), (2048, 7, 1, 16), (1024, 4, 3, 0),
                   (1024, 16, 0, 0), (1024, 16, 0, 8, 8), (512, 1, 1, 0, 8), (256, 1, 3, 4, 8),
                   (1024, 4, 0, 0, 8), (2048, 2, 5, 2, 8)]:
        g = run_gpu(b, material, P, 64, launch=launch)
        assert np.array_equal(g["rho"], ref["rho"]) and np.array_equal(g["mom"], ref["mom"]), launch
        assert np.array_equal(g["count"], ref["count"])
    g = run_gpu(b, material, P, 64, per_problem=True)
    assert np.array_equal(g["rho"], ref["rho"]) and np.array_equal(g["mom"], ref["mom"])
    assert np.array_equal(g["count"], ref["count"])


def test_run_to_end_time(material):
    b = W.random_batch(seed=5, n_problems=6, nmin=64, nmax=400)
    P = W.random_batch_params().replace(t_end=2e-4)
    import torch
    from paper_2211_00705_amd.imexds import IMEXDS
    s = IMEXDS(b, material, P)
    s.set_state()
    n = s.run(100000, check_every=64)
    torch.cuda.synchronize()
    t, st, steps = s.problems()
    rho, mom = s.state_numpy()
    home, hl, _ = s.interfaces()
    s.close()
    assert np.all(t == 2e-4) and np.all(st == 0)
    o = run_oracle(b, material, P, int(steps.max()) + 5)
    g = dict(rho=rho, mom=mom, home=home, hl=hl, t=t, status=st, steps=steps)
    assert_parity(b, g, o, logs=False)
    assert n >= steps.max()


@pytest.mark.parametrize("lanes", LANES)
def test_failures_are_flagged_and_confined(material, lanes):
    """Host-forced failures (a NaN density, a negative density, Newton limited
    to one iteration) freeze exactly their problems with the oracle's status."""
    good = W.random_batch(seed=11, n_problems=4, nmin=64, nmax=128)
    bad = good.copy()
    so = bad.slot_off
    bad.rho[so[1] + 5] = float("nan")
    bad.rho[so[3] + 2] = -1.0
    P = W.random_batch_params()
    g = run_gpu(bad, material, P, 20, lanes=lanes)
    o = run_oracle(bad, material, P, 20)
    assert g["status"][1] == 2 and g["steps"][1] == 0
    assert g["status"][3] == 2 and g["steps"][3] == 0
    assert_parity(bad.subset([0, 2]), {k: take_problems(bad, v, k, [0, 2]) for k, v in g.items()},
                  {k: take_problems(bad, v, k, [0, 2]) for k, v in o.items()}, logs=False)
    np.testing.assert_array_equal(g["status"], o["status"])
    g2 = run_gpu(good, material, P.replace(newton_maxit=1), 5, lanes=lanes)
    assert np.all(g2["status"] == 1) and np.all(g2["t"] == 0)


@pytest.mark.parametrize("lanes", LANES)
def test_forced_small_limits_match_oracle(material, lanes):
    """l_max = 1 (every zone stops at once) and Newton limited to 3 steps per
    start: the same results, statuses and logs as the oracle."""
    b = W.random_batch(seed=13, n_problems=8, nmin=64, nmax=600)
    for P in (W.random_batch_params().replace(lmax=1),
              W.random_batch_params().replace(newton_maxit=3)):
        g = run_gpu(b, material, P, 60, lanes=lanes)
        o = run_oracle(b, material, P, 60)
        assert_parity(b, g, o)


@pytest.mark.parametrize("lanes", LANES)
def test_edge_cases(material, lanes):
    """Empty batch; a problem without interfaces next to ones with them; an
    interface in the first and last background cells; pieces of exactly zero
    and of full length."""
    P = W.Params(bc_left=0, bc_right=1)
    empty = W._assemble([], [], [], [], [], [], [], name="empty")
    g = run_gpu(empty, material, P, 3, log=False, lanes=lanes)
    assert g["rho"].size == 0
    st = lambda x, q: (np.where(q == W.LIQ, 965.0 + 5 * x, 0.05 + 0.01 * x), 0.3 * np.ones(x.shape))
    b = W._assemble([30, 20, 25, 40], [1 / 30, 1 / 20, 1 / 25, 1 / 40], [0, 0, 0, 0],
                    [W.LIQ, W.VAP, W.LIQ, W.VAP], [[], [0], [24], [10, 30]],
                    [[], [0.3 / 20], [0.5 / 25], [0.0, 1 / 40]], [st] * 4, name="edges")
    g = run_gpu(b, material, P, 40, lanes=lanes)
    o = run_oracle(b, material, P, 40)
    assert_parity(b, g, o)


def _sampled_logs(b, g, idx):
    """The per-step logs of the interfaces of problems idx (in order)."""
    io = b.iface_off
    cols = np.concatenate([np.arange(io[p], io[p + 1]) for p in idx]).astype(np.int64)
    return {k: g[k][:, cols] for k in ("count", "flags", "zlo")}


@pytest.mark.parametrize("launch", [(1024, 8, 0, 10, 8), (1024, 16, 64, 10, 1)])
def test_full_size_batch_sampled(material, launch):
    """The benchmarked batch at full size (4096 problems, about 1.6e7 cells,
    1000 steps) in the launch form bench.py times (eight lanes per zone, eight
    zones per wave, all zones at once) and in a persistent one-lane form; 16
    sampled problems, including the 8 with the most dual time iterations,
    recomputed by the oracle on their own, logs (every step's dual time
    count, flags and zone) included."""
    b = W.random_batch()
    P = W.random_batch_params()
    g = run_gpu(b, material, P, 1000, launch=launch, log=True)
    rng = np.random.default_rng(1)
    heavy = np.argsort(-g["count"].sum(axis=0))[:8]
    idx = sorted(set(rng.choice(b.n_problems, size=8, replace=False).tolist())
                 | set(heavy.tolist()))
    sub = b.subset(idx)
    o = run_oracle(sub, material, P, 1000)
    gs = {k: take_problems(b, v, k, idx) for k, v in g.items()
          if k not in ("stats", "count", "flags", "zlo")}
    gs.update(_sampled_logs(b, g, idx))
    assert (o["flags"] & 8).any()  # the sample holds zones stopped at l_max
    assert_parity(sub, gs, o, logs=True)
    assert np.all(g["steps"] == 1000)
    assert g["stats"]["cell_updates"] == 1000 * b.n_slots
    assert g["stats"]["pseudo_iters"] == int(g["count"].sum())


def test_single_cut_run_to_end_time(material):
    """The single problem at full length: 200 cells, cut piece 1e-4 h, run to
    t = 0.1 (about 33,000 steps, the last one clipped) with relative-update
    dual time stepping to 1e-12 (up to 1e4 pseudo steps)."""
    b = W.single_cut_problem(seed=0)
    P = W.single_cut_params()
    n = 33000
    g = run_gpu(b, material, P, n, lanes=8)
    o = run_oracle(b, material, P, n)
    assert o["t"][0] == P.t_end and g["t"][0] == P.t_end
    assert_parity(b, g, o)


def test_large_problem_full_size(material):
    """One problem of 2^20 cells, 2000 steps, paper stop rule, zone of 5 cells."""
    b = W.large_smooth_problem()
    P = W.large_smooth_params()
    n = 2000
    g = run_gpu(b, material, P, n, lanes=8)
    o = run_oracle(b, material, P, n)
    assert np.all(o["status"] == 0)
    assert_parity(b, g, o)


def test_bubble_batch_full_size_sampled(material):
    """1024 bubble problems of 4096 cells (two interfaces each), 2000 steps;
    6 sampled problems recomputed by the oracle on their own."""
    b = W.bubble_batch()
    P = W.bubble_batch_params()
    n = 2000
    g = run_gpu(b, material, P, n, log=True, lanes=8)
    rng = np.random.default_rng(4)
    idx = set(rng.choice(b.n_problems, size=6, replace=False).tolist())
    # problems whose two zones were joined at some step
    paired = np.nonzero(((g["flags"] & 256) != 0).any(axis=0))[0] // 2
    idx |= set(paired[:3].tolist())
    # In this configuration some bubbles close: compressed liquid condenses
    # the vapour, the two zones join into one, and the problem is frozen when
    # the vapour vanishes (PHASE_VANISH); one reaches a non-physical state.
    # No zones overlap outside a pair.  Two problems of every frozen status
    # are recomputed too: the oracle must freeze them with the same status at
    # the same step.
    assert not np.any(g["status"] & 8)
    assert g["stats"]["pair_zones"] > 0
    for st in np.unique(g["status"]):
        if st != 0:
            idx |= set(np.nonzero(g["status"] == st)[0][:2].tolist())
    idx = sorted(idx)
    sub = b.subset(idx)
    o = run_oracle(sub, material, P, n)
    gs = {k: take_problems(b, v, k, idx) for k, v in g.items()
          if k not in ("stats", "count", "flags", "zlo")}
    gs.update(_sampled_logs(b, g, idx))
    assert_parity(sub, gs, o, logs=True)
