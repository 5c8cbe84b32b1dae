"""Zones holding two phase boundaries on the GPU (k_zone_pair) against the
CPU oracle, through the C ABI: when the zones of two neighbouring interfaces
overlap they are solved as one zone (Algorithm 2 with two interface solves
per pseudo iteration), and a merge that would leave the phase between the
two boundaries as a single cell freezes the problem with PHASE_VANISH.  Bar:
bitwise in practice, rel-L1 <= 1e-10, identical statuses, steps, dual time
counts, flags and zones at every step."""
import math

import numpy as np
import pytest

import oracle
from parity import assert_parity, run_gpu, run_oracle
from paper_2211_00705_amd import workloads as W

pytestmark = pytest.mark.gpu

LANES = [1, 8]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_00705_amd import imexds  # noqa: F401  (fails loudly if the library is missing)


def _states(rl, ul, rv, uv, split=None):
    def st(x, q):
        if q == W.LIQ:
            u = np.full(x.shape, ul) if split is None else np.where(x < split, ul, -ul)
            return np.full(x.shape, rl), u
        return np.full(x.shape, rv), np.full(x.shape, uv)
    return st


def _close_pair():
    return W._assemble([40], [0.025], [0.0], [W.LIQ], [[10, 12]], [[0.01, 0.01]],
                       [_states(966.0, 0.0, 0.4, 0.0)], name="close")


@pytest.mark.parametrize("lanes", LANES)
def test_close_pair_every_step(material, lanes):
    b = _close_pair()
    g = run_gpu(b, material, W.Params(), 40, lanes=lanes)
    o = run_oracle(b, material, W.Params(), 40)
    assert np.all(o["flags"] & oracle.FL_PAIR) and np.all(o["status"] == 0)
    assert_parity(b, g, o)
    assert g["stats"]["pair_zones"] == 40


def _condensing_bubble(material, a_left, width, n=60, j=24):
    """Liquid moving in on a supersaturated vapour bubble at rest (rho_V =
    0.45 kg/m^3) with the liquid state that makes each phase boundary an exact
    condensing front, so that the bubble collapses with every state kept."""
    from scipy.optimize import brentq
    M = material
    rV = 0.45
    pV, vV = M.a2v * rV, 1.0 / rV
    gV = M.a2v * math.log(rV / (M.p0 / M.a2v))

    def resid(rL):
        pL = M.p0 + M.a2l * (rL - M.rhol0)
        vL = 1.0 / rL
        z2 = (pL - pV) / (vV - vL)
        z = math.sqrt(max(z2, 0.0))
        gL = M.a2l * math.log(rL / M.rhol0)
        return z - M.tau * pV * ((gV - gL) + 0.5 * z2 * (vV**2 - vL**2))

    r_lo = M.rhol0 + (pV - M.p0) / M.a2l
    xs = np.linspace(r_lo * (1 + 1e-15), r_lo + 1.0, 2001)
    fs = [resid(x) for x in xs]
    i = next(i for i in range(len(xs) - 1) if fs[i] * fs[i + 1] < 0)
    rL = brentq(resid, xs[i], xs[i + 1], xtol=1e-14, rtol=1e-15)
    pL = M.p0 + M.a2l * (rL - M.rhol0)
    z = math.sqrt((pL - pV) / (vV - 1.0 / rL))
    w = z * vV
    uL = w - z / rL
    h = 0.01
    xa = (j + a_left) * h
    xb = xa + width * h
    ja, jb = int(xa // h), int(xb // h)
    return W._assemble([n], [h], [0.0], [W.LIQ], [[ja, jb]], [[xa - ja * h, xb - jb * h]],
                       [_states(rL, uL, rV, 0.0, split=0.5 * (xa + xb))], name="collapse")


@pytest.mark.parametrize("a_left", [0.35, 0.93])
@pytest.mark.parametrize("lanes", LANES)
def test_bubble_collapse_to_phase_vanish(material, a_left, lanes):
    b = _condensing_bubble(material, a_left, 5.3)
    P = W.Params(bc_left=1, bc_right=1)
    n = 400
    g = run_gpu(b, material, P, n, lanes=lanes)
    o = run_oracle(b, material, P, n)
    assert o["status"][0] == oracle.ST_VANISH and 100 < o["steps"][0] < n
    assert (o["flags"][:, 0] & oracle.FL_PAIR).sum() >= 5
    assert_parity(b, g, o)


@pytest.mark.parametrize("lanes", LANES)
def test_travelling_pair_at_saturation(material, lanes):
    rV0 = material.p0 / material.a2v
    b = W._assemble([50], [0.01], [0.0], [W.VAP], [[20, 22]], [[0.006, 0.003]],
                    [_states(material.rhol0, 3.0, rV0, 3.0)], name="sat")
    P = W.Params(bc_left=1, bc_right=1)
    g = run_gpu(b, material, P, 300, lanes=lanes)
    o = run_oracle(b, material, P, 300)
    assert (o["flags"] & oracle.FL_PAIR).any() and (o["flags"] & oracle.FL_CROSS_R).any()
    assert_parity(b, g, o)


@pytest.mark.parametrize("lanes", LANES)
def test_bubble_batch_with_pairs(material, lanes):
    """48 bubble problems of 512 cells for 1500 steps: bubbles collapse, their
    zones join, and some reach PHASE_VANISH; the other problems run beside
    them in the same launches."""
    b = W.bubble_batch(seed=7, n_problems=48, n=512)
    P = W.bubble_batch_params()
    n = 1500
    g = run_gpu(b, material, P, n, lanes=lanes)
    o = run_oracle(b, material, P, n)
    assert (o["flags"] & oracle.FL_PAIR).sum() > 100
    assert np.sum(o["status"] == oracle.ST_VANISH) >= 2
    assert not np.any(o["status"] & oracle.ST_OVERLAP)
    assert_parity(b, g, o)


def test_pairs_under_every_launch_form(material):
    """Graph replay, direct launches, per-problem launches and the timing
    mode give the same bits with pairs present."""
    import torch
    from paper_2211_00705_amd.imexds import IMEXDS
    b = W.bubble_batch(seed=7, n_problems=48, n=512)
    P = W.bubble_batch_params()
    n = 1200
    o = run_oracle(b, material, P, n)
    ref = None
    for form in ("graph", "direct", "per_problem", "timed"):
        s = IMEXDS(b, material, P)
        try:
            s.set_launch(zone_lanes=8, graph_steps=0 if form == "direct" else 8)
            s.set_state()
            if form == "timed":
                s.time_bulk(True)
            if form == "per_problem":
                s.step_per_problem(n)
            else:
                s.step(n)
            torch.cuda.synchronize()
            rho, mom = s.state_numpy()
            _, status, steps = s.problems()
        finally:
            s.close()
        assert np.array_equal(status, o["status"]) and np.array_equal(steps, o["steps"])
        if ref is None:
            ref = (rho, mom)
        assert np.array_equal(rho, ref[0]) and np.array_equal(mom, ref[1]), form


def test_overlaps_outside_a_pair_freeze(material):
    """Three mutually overlapping zones freeze their problem (ZONE_OVERLAP),
    as does any overlap under the Newton zone solver; the next problem runs."""
    st = _states(966.0, 0.0, 0.4, 0.0)
    b = W._assemble([40, 50], [0.025, 0.02], [0.0, 0.0], [W.LIQ, W.LIQ], [[10, 12, 14], [20]],
                    [[0.01, 0.01, 0.01], [0.005]], [st, st], name="three")
    g = run_gpu(b, material, W.Params(), 10)
    o = run_oracle(b, material, W.Params(), 10)
    assert g["status"][0] == oracle.ST_OVERLAP and g["status"][1] == 0
    assert_parity(b, g, o)
    b2 = _close_pair()
    P = W.Params(zone_solver=1)
    g2 = run_gpu(b2, material, P, 5)
    o2 = run_oracle(b2, material, P, 5)
    assert g2["status"][0] == oracle.ST_OVERLAP
    assert_parity(b2, g2, o2)


def test_adjoint_refuses_a_forward_with_pairs(material):
    import torch
    from paper_2211_00705_amd.imexds import IMEXDS, IMEXDSError
    b = _close_pair()
    s = IMEXDS(b, material, W.Params())
    try:
        s.set_launch(zone_lanes=8)
        s.set_state()
        s.forward_ckpt(10, 5)
        z = torch.zeros(b.n_slots, dtype=torch.float64, device="cuda")
        with pytest.raises(IMEXDSError, match="unsupported"):
            s.adjoint(z, z)
    finally:
        s.close()
