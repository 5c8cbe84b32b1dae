"""Pins of the oracle's tangent build (the reference for the GPU adjoint).

The tangent build is the oracle's own source compiled with dual numbers, so
it differentiates exactly the discrete map the oracle executes, with every
decision (pseudo-iteration count, merge, crossing, CFL cell, HLL branch)
that of the plain run.  These tests pin it to things other than itself:

* its value parts are the plain oracle's, bit for bit;
* the scheme conserves mass exactly with walls (Sec. 3.4: the moving cut
  cells update h U conservatively, eq. godunov_meth:nonunif), so the
  derivative of the total mass after any number of steps along any
  direction is the initial slot lengths dotted with the density direction;
* central differences of the plain oracle with the decisions replayed agree
  with it to the differencing error;
* a replay of a run's own decisions reproduces that run bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2211_00705_amd import workloads as W


def _slot_lengths(b):
    out = []
    so = b.slot_off
    for p in range(b.n_problems):
        Lp = np.full(int(so[p + 1] - so[p]), b.h[p])
        for kk, k in enumerate(range(int(b.iface_off[p]), int(b.iface_off[p + 1]))):
            Lp[b.home[k] + kk] = b.hl[k]
            Lp[b.home[k] + kk + 1] = b.h[p] - b.hl[k]
        out.append(Lp)
    return np.concatenate(out)


CASES = {
    "single_cut": (lambda: W.single_cut_problem(seed=3), lambda: W.single_cut_params(), 300),
    "random_batch": (lambda: W.random_batch(n_problems=16, nmax=1024), W.random_batch_params, 200),
    "bubble_batch": (lambda: W.bubble_batch(n_problems=8, n=256), W.bubble_batch_params, 200),
}


def _direction(b, material, rng):
    dr = rng.standard_normal(b.n_slots) * b.rho
    dm = rng.standard_normal(b.n_slots) * np.maximum(np.abs(b.mom), 1e-3 * b.rho)
    return dr, dm, rng.standard_normal() * material.tau


@pytest.mark.parametrize("case", sorted(CASES))
def test_tangent_values_are_the_plain_oracle(material, case):
    mk, mp, n = CASES[case]
    b, P = mk(), mp()
    a = oracle.State(b)
    oracle.run(a, material, P, n, threads=4)
    s = oracle.State(b)
    rng = np.random.default_rng(7)
    dr, dm, dtau = _direction(b, material, rng)
    obj, _, _ = oracle.tangent(s, material, P, n, dr, dm, dtau, threads=4)
    for f in ("rho", "mom", "hl", "home", "pw", "t", "status", "steps"):
        assert np.array_equal(getattr(a, f), getattr(s, f)), f
    assert np.array_equal(obj, oracle.objective(a))


@pytest.mark.parametrize("case", ["random_batch", "bubble_batch"])
def test_tangent_of_total_mass_is_the_initial_lengths(material, case):
    mk, mp, n = CASES[case]
    b, P = mk(), mp()
    assert P.bc_left == 0 and P.bc_right == 0
    rng = np.random.default_rng(11)
    dr = rng.standard_normal(b.n_slots)
    dm = 100.0 * rng.standard_normal(b.n_slots)
    s = oracle.State(b)
    lo, hi = float(np.min(b.x_left)) - 1.0, float(np.max(b.x_left + b.n_cells * b.h)) + 1.0
    _, dobj, _ = oracle.tangent(s, material, P, n, dr, dm, 0.3 * material.tau, cx=0.0, wa=lo,
                                wb=hi, threads=4)
    assert np.all(s.status == 0) and np.all(s.steps == n)
    lens = _slot_lengths(b)
    exact = np.add.reduceat(dr * lens, b.slot_off[:-1])
    np.testing.assert_allclose(dobj, exact, rtol=1e-12)


@pytest.mark.parametrize("case", sorted(CASES))
def test_replay_reproduces_the_run(material, case):
    mk, mp, n = CASES[case]
    b, P = mk(), mp()
    a = oracle.State(b)
    lg = oracle.run(a, material, P, n, log="full", threads=4)
    r = oracle.State(b)
    lg2 = oracle.run(r, material, P, n, log="full", threads=4, replay=lg)
    for f in ("rho", "mom", "hl", "home", "pw", "t"):
        assert np.array_equal(getattr(a, f), getattr(r, f)), f
    # a replay takes its counts and merges from the log: it reports no
    # l_max or redo event of its own
    own = ~np.int32(oracle.FL_LMAX | oracle.FL_REDO)
    assert np.array_equal(lg[0], lg2[0]) and np.array_equal(lg[2], lg2[2])
    assert np.array_equal(lg[3], lg2[3])
    assert np.array_equal(lg[1] & own, lg2[1] & own)


@pytest.mark.parametrize("case", sorted(CASES))
def test_tangent_matches_replayed_central_differences(material, case):
    mk, mp, n = CASES[case]
    b, P = mk(), mp()
    base = oracle.State(b)
    lg = oracle.run(base, material, P, n, log="full", threads=4)
    flags = lg[1]
    if case != "single_cut":  # the batches exercise merges and both crossings
        assert np.any(flags & oracle.FL_MERGED) and np.any(flags & oracle.FL_CROSS_L)
        assert np.any(flags & oracle.FL_CROSS_R)
    eps = 1e-7
    rng = np.random.default_rng(5)
    for _ in range(2):
        dr, dm, dtau = _direction(b, material, rng)
        s = oracle.State(b)
        _, dobj, _ = oracle.tangent(s, material, P, n, dr, dm, dtau, threads=4)
        fd = []
        for sg in (1.0, -1.0):
            bb = b.copy()
            bb.rho = b.rho + sg * eps * dr
            bb.mom = b.mom + sg * eps * dm
            mp_ = W.Material(tau=material.tau + sg * eps * dtau)
            sp = oracle.State(bb)
            oracle.run(sp, mp_, P, n, threads=4, replay=lg)
            fd.append(oracle.objective(sp))
        fdv = (fd[0] - fd[1]) / (2 * eps)
        # differencing error: O(eps^2) truncation plus the objective's
        # rounding (a few ulp of |L|) over 2 eps
        noise = 5e-16 * np.abs(fd[0]) / eps
        assert np.all(np.abs(dobj - fdv) <= 2e-6 * np.abs(dobj) + noise)


def test_tangent_in_the_kinetic_coefficient(material):
    """d objective / d tau alone (the kinetic relation eq. isoT:kin_rel1 is
    the only place tau enters)."""
    b, P, n = W.bubble_batch(n_problems=4, n=256), W.bubble_batch_params(), 150
    base = oracle.State(b)
    lg = oracle.run(base, material, P, n, log="full")
    s = oracle.State(b)
    z = np.zeros(b.n_slots)
    _, dobj, _ = oracle.tangent(s, material, P, n, z, z, material.tau)
    eps = 1e-6
    fd = []
    for sg in (1.0, -1.0):
        sp = oracle.State(b)
        oracle.run(sp, W.Material(tau=material.tau * (1 + sg * eps)), P, n, replay=lg)
        fd.append(oracle.objective(sp))
    fdv = (fd[0] - fd[1]) / (2 * eps)
    assert np.all(np.abs(dobj) > 0)
    noise = 5e-16 * np.abs(fd[0]) / eps
    assert np.all(np.abs(dobj - fdv) <= 1e-5 * np.abs(dobj) + noise)
    # the same map with tau frozen has no tau sensitivity
    s2 = oracle.State(b)
    _, d0, _ = oracle.tangent(s2, material, P, n, z, z, 0.0)
    assert np.all(d0 == 0.0)


def test_objective_by_brute_force():
    """Window mass by explicit slot intervals and interface positions."""
    b = W.bubble_batch(n_problems=3, n=64)
    s = oracle.State(b)
    got = oracle.objective(s, cx=1.0, wa=0.4, wb=0.6)
    lens = _slot_lengths(b)
    for p in range(b.n_problems):
        x = b.x_left[p]
        tot = 0.0
        for sl in range(int(b.slot_off[p]), int(b.slot_off[p + 1])):
            a, e = x, x + lens[sl]
            tot += b.rho[sl] * max(0.0, min(e, 0.6) - max(a, 0.4))
            x = e
        ks = range(int(b.iface_off[p]), int(b.iface_off[p + 1]))
        tot += sum(b.x_left[p] + b.home[k] * b.h[p] + b.hl[k] for k in ks)
        assert got[p] == pytest.approx(tot, rel=1e-13)
