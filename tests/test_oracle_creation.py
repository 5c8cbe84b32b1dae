"""Pins of the oracle's phase creation (cavitation and nucleation): the
five-state Riemann problem solved from the initial data of the paper's two
tests reproduces the printed exact star states and phase-boundary speeds;
closed forms for the single-phase problem of step (i); the two phase
boundaries satisfy the (separately pinned) two-phase interface problem;
textbook outer waves; mirror symmetry."""
import json
import math
import os

import pytest

import oracle
from paper_2211_00705_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def gold(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


M = W.WATER_363K
LIM = gold("eos_limits.json")
P_MIN, P_TILDE = LIM["p_min_Pa"], LIM["p_tilde_Pa"]


def rho(ph, p):
    # the phase pressure laws of Sec. 4, inverted
    return p / M.a2v if ph == W.VAP else M.rhol0 + (p - M.p0) / M.a2l


def solve(ph, pl, ul, pr, ur):
    rl, rr = rho(ph, pl), rho(ph, pr)
    return oracle.creation_rp(M, ph, rl, rl * ul, rr, rr * ur, P_MIN, P_TILDE)


def test_cavitation_exact_row():
    """Sec. 4 cavitation test: liquid at 60000 Pa pulled apart at -/+4 m/s."""
    g = gold("cavitation_star_states.json")
    st, d = solve(W.LIQ, 60000.0, -4.0, 60000.0, 4.0)
    assert st == 1 and d["kind"] == 1.0 and d["p1"] < P_MIN
    assert abs(d["pa"] - g["pL_star_minus_Pa"]) < 1e-3
    assert abs(d["pc"] - g["pL_star_plus_Pa"]) < 1e-3
    assert abs(d["pb"] - g["pV_star_Pa"]) < 1e-3
    assert d["ua"] == pytest.approx(g["uL_star_minus"], abs=1e-6)
    assert d["uc"] == pytest.approx(g["uL_star_plus"], abs=1e-6)
    assert abs(d["ub"]) < 1e-9
    assert d["wr"] == pytest.approx(g["w_right"], abs=1e-6)
    assert d["wl"] == pytest.approx(-g["w_right"], abs=1e-6)
    # the created vapour layer after the first step, (w_r - w_l) dt with the
    # CFL step of the initial data (|u| + a_L = 4 + a_L, C = 0.5, h = 1e-2)
    dt = g["cfl"] * g["h"] / (g["initial_liquid_speed"] + math.sqrt(M.a2l))
    assert (d["wr"] - d["wl"]) * dt == pytest.approx(g["h_V_created"], rel=2e-4)


def test_nucleation_exact_row():
    """Sec. 4 nucleation test: vapour at 70000 Pa compressed at +/-2.7 m/s."""
    g = gold("nucleation_star_states.json")
    st, d = solve(W.VAP, 70000.0, 2.7, 70000.0, -2.7)
    assert st == 1 and d["kind"] == 2.0 and d["p1"] > P_TILDE
    assert abs(d["pa"] - g["pV_star_minus_Pa"]) < 1e-3
    assert abs(d["pc"] - g["pV_star_plus_Pa"]) < 1e-3
    assert abs(d["pb"] - g["pL_star_Pa"]) < 1e-3
    assert d["ua"] == pytest.approx(g["uV_star_minus"], abs=1e-6)
    assert d["uc"] == pytest.approx(g["uV_star_plus"], abs=1e-6)
    assert abs(d["ub"]) < 1e-9
    assert abs(d["wl"]) == pytest.approx(g["w_abs"], abs=5e-7)
    assert d["wl"] < 0 < d["wr"]


def test_single_phase_problem_closed_forms():
    """Step (i) without creation: symmetric isothermal rarefactions
    rho* = rho exp(-du/(2a)) (Riemann invariant) and symmetric shocks
    x - 1/x = u/a with x^2 = rho*/rho (Rankine-Hugoniot)."""
    a_l, a_v = math.sqrt(M.a2l), math.sqrt(M.a2v)
    r = rho(W.LIQ, 1e5)
    st, d = solve(W.LIQ, 1e5, -1e-3, 1e5, 1e-3)
    want = M.p0 + M.a2l * (r * math.exp(-2e-3 / (2 * a_l)) - M.rhol0)
    assert st == 0 and d["p1"] == pytest.approx(want, abs=1e-6)
    r = rho(W.VAP, 60000.0)
    st, d = solve(W.VAP, 60000.0, 1.0, 60000.0, -1.0)
    y = 1.0 / a_v
    x = 0.5 * (y + math.sqrt(y * y + 4.0))
    assert st == 0 and d["p1"] == pytest.approx(M.a2v * r * x * x, rel=1e-12)
    # liquid pulled apart but staying above p_min, vapour compressed but
    # staying below p_tilde: no creation
    assert solve(W.LIQ, 2e6, -0.5, 2e6, 0.5)[0] == 0
    assert solve(W.VAP, 60000.0, 2.0, 60000.0, -2.0)[0] == 0


@pytest.mark.parametrize("p_star", [5000.0, 1.0, -1.0, -5000.0])
def test_step_i_decides_near_p_min(p_star):
    """Symmetric rarefactions built to reach a given star pressure near
    p_min = 0: the single-phase solve must converge there (the liquid
    resolves p* only to about 1e-7 Pa) and decide by the sign."""
    a = math.sqrt(M.a2l)
    r = rho(W.LIQ, 60000.0)
    r_star = rho(W.LIQ, p_star)
    du = 2.0 * a * math.log(r / r_star)
    st, d = solve(W.LIQ, 60000.0, -0.5 * du, 60000.0, 0.5 * du)
    assert d["p1"] == pytest.approx(p_star, abs=1e-3)
    assert st == (1 if p_star < P_MIN else 0)


def _textbook_f(ph, r, r_star):
    """Velocity change across an isothermal wave of p = a^2 rho + const."""
    a = math.sqrt(M.a2v if ph == W.VAP else M.a2l)
    if r_star > r:
        return a * (r_star - r) / math.sqrt(r * r_star)
    return a * math.log(r_star / r)


@pytest.mark.parametrize("case", [
    (W.LIQ, 50000.0, -3.0, 65000.0, 5.0),
    (W.LIQ, 69000.0, 0.5, 30000.0, 9.0),
    (W.VAP, 69500.0, 6.0, 70100.0, -4.0),
    (W.VAP, 70300.0, 4.0, 69000.0, -6.0),
])
def test_asymmetric_creation_is_consistent(case):
    """Outer waves by the textbook formulas; each phase boundary satisfies the
    two-phase problem of the interface solver (G = 0 with the star states as
    outer states); mass conservation across both boundaries."""
    ph, pl, ul, pr, ur = case
    st, d = solve(ph, pl, ul, pr, ur)
    assert st == 1
    rl, rr = rho(ph, pl), rho(ph, pr)
    assert d["ua"] == pytest.approx(ul - _textbook_f(ph, rl, d["ra"]), abs=1e-9)
    assert d["uc"] == pytest.approx(ur + _textbook_f(ph, rr, d["rc"]), abs=1e-9)
    nph = 1 - ph
    for (phl, rL, uL, pL, phr, rR, uR, pR, z) in (
            (ph, d["ra"], d["ua"], d["pa"], nph, d["rb"], d["ub"], d["pb"], d["zl"]),
            (nph, d["rb"], d["ub"], d["pb"], ph, d["rc"], d["uc"], d["pc"], d["zr"])):
        G, _ = oracle.iface_G(M, phl, rL, uL, phr, rR, uR, pL, pR)
        scale = max(abs(pL), abs(pR))
        assert abs(G[0]) < 1e-9 * scale and abs(G[1]) < 1e-9
    for rK, uK, w in ((d["ra"], d["ua"], d["wl"]), (d["rc"], d["uc"], d["wr"])):
        assert rK * (uK - w) == pytest.approx(d["rb"] * (d["ub"] - w), rel=1e-9, abs=1e-12)


def test_mirror_symmetry():
    st, d = solve(W.LIQ, 50000.0, -3.0, 65000.0, 5.0)
    st2, e = solve(W.LIQ, 65000.0, -5.0, 50000.0, 3.0)
    assert st == st2 == 1
    assert e["pa"] == pytest.approx(d["pc"], rel=1e-12)
    assert e["pb"] == pytest.approx(d["pb"], rel=1e-12)
    assert e["ua"] == pytest.approx(-d["uc"], rel=1e-10)
    assert e["wl"] == pytest.approx(-d["wr"], rel=1e-9)


def test_invalid_input():
    assert oracle.creation_rp(M, W.LIQ, -1.0, 0.0, 900.0, 0.0, P_MIN, P_TILDE)[0] == -1
