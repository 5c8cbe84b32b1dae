"""GPU parity of the full-Euler path (ideal gas, fixed mesh with one small
cell per problem) against the CPU oracle, through the C ABI: states, times,
step and dual time iteration counts, per-step logs and status bits must be
identical (the two sides evaluate the same IEEE expressions in the same
order, so the comparison is bitwise)."""
import numpy as np
import pytest

import oracle
from paper_2211_00705_amd import euler_workloads as EW

pytestmark = pytest.mark.gpu


def run_gpu(b, n_steps=None, tile=1024, lanes=2, log_rows=None, ppw=32):
    import torch
    from paper_2211_00705_amd.euler import EulerIMEXDS
    s = EulerIMEXDS(b)
    try:
        s.set_launch(tile, lanes, ppw)
        s.set_state()
        if log_rows:
            s.enable_log(log_rows)
        if n_steps is None:
            s.run()
        else:
            s.step(n_steps)
        torch.cuda.synchronize()
        rho, mom, ene = s.state_numpy()
        t, status, steps, iters = s.problems()
        out = dict(rho=rho, mom=mom, ene=ene, t=t, status=status, steps=steps, iters=iters)
        if log_rows:
            out["count"], out["flags"] = s.log()
        return out
    finally:
        s.close()


def run_oracle(b, n_steps=None, log_rows=None, threads=8):
    st = oracle.EulerState(b)
    out = {}
    if log_rows:
        lc, lf = oracle.euler_run(st, log_rows, threads=threads, log=True)
        out["count"], out["flags"] = lc.T, lf.T
    else:
        oracle.euler_run(st, n_steps, threads=threads)
    out.update(rho=st.rho, mom=st.mom, ene=st.ene, t=st.t, status=st.status, steps=st.steps,
               iters=st.iters)
    return out


def assert_same(b, g, o, rows=None):
    ok = g["status"] == 0
    assert np.array_equal(g["status"], o["status"]), (g["status"], o["status"])
    assert np.array_equal(g["steps"], o["steps"])
    assert np.array_equal(g["iters"], o["iters"])
    assert np.array_equal(g["t"], o["t"])
    off = b.off
    for p in np.flatnonzero(ok):
        sl = slice(off[p], off[p + 1])
        for f in ("rho", "mom", "ene"):
            assert np.array_equal(g[f][sl], o[f][sl]), (p, f, np.max(np.abs(g[f][sl] - o[f][sl])))
    if rows:
        r = g["count"].shape[0]
        assert np.array_equal(g["count"], o["count"][:r])
        assert np.array_equal(g["flags"], o["flags"][:r])


@pytest.mark.parametrize("lanes", [1, 2])
def test_lax_study_to_end_time(lanes):
    """The paper's Lax tube configurations (theta_{k+-1} = 0.9, 0.1 with
    alpha down to 1e-6, and theta_{k+-1} = alpha = 1e-2) run to t_end = 1."""
    entries = [e for e in EW.LAX_STUDY if e[0] is not None] + [(None, N, 1e-2)
                                                                 for N in (100, 200, 400)]
    b = EW.lax_study(entries)
    rows = 240
    g = run_gpu(b, lanes=lanes, log_rows=rows)
    o = run_oracle(b, log_rows=rows)
    assert np.all(g["status"] == 0) and np.all(g["t"] == 1.0)
    assert_same(b, g, o, rows)
    avg = dict(zip(entries, g["iters"] / g["steps"]))
    assert avg[(0.9, 100, 1e-6)] > avg[(0.9, 100, 1e-2)]


@pytest.mark.parametrize("tile,lanes,ppw", [(256, 2, 4), (512, 1, 64), (1024, 2, 32), (256, 1, 1),
                                            (512, 2, 7)])
def test_lax_batch_matches_oracle(tile, lanes, ppw):
    """A seeded ensemble of Lax-type tubes (N in 100..400, alpha log-uniform in
    [1e-6, 1e-2], theta_{k+-1} in {0.9, 0.1}, perturbed states), stepped 60
    times: ragged problem ends, tiles spanning problem boundaries."""
    b = EW.lax_batch(seed=5, n_problems=96)
    g = run_gpu(b, 60, tile=tile, lanes=lanes, log_rows=60, ppw=ppw)
    o = run_oracle(b, 60, log_rows=60)
    assert np.all(g["status"] == 0)
    assert_same(b, g, o, 60)


def test_lax_batch_full_size():
    """The benchmark ensemble (4096 tubes, about 1.2 M cells) to t_end,
    compared cell by cell with the oracle."""
    b = EW.lax_batch()
    g = run_gpu(b)
    o = run_oracle(b, threads=16)
    assert np.all(g["status"] == 0) and np.all(g["t"] == b.t_end)
    assert_same(b, g, o)


def test_failures_and_limits_match_oracle():
    """Vacuum from the initial data, a negative pressure in a bulk cell, l_max
    reached (a flag) and an unconverged small cell whose Part 2 is not
    physical, next to healthy problems."""
    specs = [EW.lax_spec(20, 1e-2, 0.9, left=(1.0, -8.0, 0.4), right=(1.0, 8.0, 0.4)),
             EW.lax_spec(40, 1e-3, 0.9), EW.lax_spec(20, 1e-2, 0.9), EW.lax_spec(20, 1e-1, 0.9),
             EW.lax_spec(100, 1e-5, 0.1)]
    b = EW._concat(specs, "faults")
    b.ene[b.off[2] + 3] = 0.01  # negative pressure in a bulk cell of problem 2
    for lmax in (3, 1_000_000):
        bb = b.replace(lmax=lmax)
        g = run_gpu(bb, 30, lanes=2, log_rows=30)
        o = run_oracle(bb, 30, log_rows=30)
        assert g["status"][0] & oracle.EU_ST_VACUUM
        assert g["status"][2] & oracle.EU_ST_NONPHYS
        assert_same(bb, g, o, 30)
        if lmax == 3:
            n3 = g["steps"][3]
            assert g["status"][3] == 0 and n3 > 0 and np.all(g["flags"][:n3, 3] & oracle.EU_FL_LMAX)
            assert g["status"][1] == oracle.EU_ST_NONPHYS


def test_edge_cases():
    import torch
    from paper_2211_00705_amd.euler import EulerIMEXDS
    # empty batch
    b = EW._concat([], "empty")
    s = EulerIMEXDS(b)
    s.set_state(*(torch.zeros(0, dtype=torch.float64, device="cuda") for _ in range(3)))
    s.step(3)
    assert s.problems()[0].shape == (0,)
    s.close()
    # the smallest mesh (N = 4: the zone touches both boundary neighbours),
    # t_end = 0 (nothing to do) and one very short run, with a regular batch
    specs = [EW.lax_spec(4, 0.5, 0.9), EW.lax_spec(6, 1e-3, 0.5, t_end=0.0),
             EW.lax_spec(8, 1.0, 1.0, theta_k=1.0, t_end=0.05)]
    b = EW._concat(specs, "edges")
    g = run_gpu(b, 40, log_rows=40)
    o = run_oracle(b, 40, log_rows=40)
    assert g["steps"][1] == 0 and g["t"][1] == 0.0
    assert_same(b, g, o, 40)


def test_api_errors():
    import torch
    from paper_2211_00705_amd import euler as E
    from paper_2211_00705_amd.imexds import IMEXDSError
    b = EW.lax_tube(10, 1e-2, 0.9)
    for bad in (b.replace(N=np.array([7], np.int32)), b.replace(alpha=np.array([0.0])),
                b.replace(theta_nb=np.array([1.5])), b.replace(gamma=1.0),
                b.replace(lmax=-1), b.replace(cfl=np.array([np.nan]))):
        with pytest.raises(IMEXDSError):
            E.EulerIMEXDS(bad)
    s = E.EulerIMEXDS(b)
    with pytest.raises(IMEXDSError):
        s.step(1)  # no state yet
    for bad in ((300, 2, 4), (256, 3, 4), (256, 2, 0), (256, 2, 33), (256, 1, 65)):
        with pytest.raises(IMEXDSError):
            s.set_launch(*bad)
    s.close()


@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.2])
def test_other_gases_match_oracle(gamma):
    """Other ratios of specific heats change every exponent of the exact
    Riemann solver ((gamma-1)/(2 gamma), 1/gamma, 2/(gamma-1), ...)."""
    rng = np.random.default_rng(17)
    specs = [EW.lax_spec(int(rng.choice([20, 64, 100])), float(10 ** rng.uniform(-5, -2)),
                         float(rng.choice([0.9, 0.3])), t_end=0.4) for _ in range(24)]
    b = EW._concat(specs, f"gamma_{gamma:.3f}", gamma=gamma)
    g = run_gpu(b, log_rows=80)
    o = run_oracle(b, log_rows=80)
    assert np.all(g["status"] == 0) and np.all(g["t"] == 0.4)
    assert_same(b, g, o, 80)


def test_per_problem_launches_match_batched():
    """The unbatched form (sweep, dual time kernel and bookkeeping launched
    problem by problem) gives the batched results bit for bit."""
    import torch
    from paper_2211_00705_amd.euler import EulerIMEXDS
    b = EW.lax_batch(seed=9, n_problems=24)
    out = []
    for per_problem in (False, True):
        s = EulerIMEXDS(b)
        s.set_state()
        if per_problem:
            s.step_per_problem(40)
        else:
            s.step(40)
        torch.cuda.synchronize()
        out.append((s.state_numpy(), s.problems()))
        s.close()
    (sa, pa), (sb, pb) = out
    for x, y in zip(sa + tuple(pa), sb + tuple(pb)):
        assert np.array_equal(x, y)
