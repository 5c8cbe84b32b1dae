"""Self-similar exact solution of the two-phase Riemann problem.

Test helper.  Star states come from the oracle's interface solver (pinned on
its own against the paper's printed star states); the outer waves are the
textbook isothermal wave curves with a constant sound speed per phase:
shock speed from mass conservation across the jump, rarefaction fans from the
Riemann invariants u +- a ln(rho) along the characteristics u -+ a.
"""
import math

import numpy as np

import oracle


def star(material, left, right, phases):
    r = oracle.iface_solve(material, phases[0], left[0], left[1], phases[1], right[0], right[1])
    assert r["ok"]
    return r


def sample(material, left, right, phases, xi, st=None):
    """(rho, u) of the exact solution at x/t = xi (array)."""
    if st is None:
        st = star(material, left, right, phases)
    a2 = {0: material.a2l, 1: material.a2v}
    al, ar = math.sqrt(a2[phases[0]]), math.sqrt(a2[phases[1]])
    rl, ul = left
    rr, ur = right
    rls, uls, rrs, urs, w = st["rl"], st["ul"], st["rr"], st["ur"], st["w"]
    xi = np.asarray(xi, dtype=float)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    # left wave
    lm = xi < w
    if rls > rl:  # shock
        s = (rls * uls - rl * ul) / (rls - rl)
        a = lm & (xi < s)
        rho[a], u[a] = rl, ul
        b = lm & (xi >= s)
        rho[b], u[b] = rls, uls
    else:  # rarefaction
        head, tail = ul - al, uls - al
        a = lm & (xi < head)
        rho[a], u[a] = rl, ul
        b = lm & (xi >= head) & (xi <= tail)
        u[b] = xi[b] + al
        rho[b] = rl * np.exp((ul - u[b]) / al)
        c = lm & (xi > tail)
        rho[c], u[c] = rls, uls
    rm = ~lm
    if rrs > rr:
        s = (rrs * urs - rr * ur) / (rrs - rr)
        a = rm & (xi > s)
        rho[a], u[a] = rr, ur
        b = rm & (xi <= s)
        rho[b], u[b] = rrs, urs
    else:
        head, tail = ur + ar, urs + ar
        a = rm & (xi > head)
        rho[a], u[a] = rr, ur
        b = rm & (xi <= head) & (xi >= tail)
        u[b] = xi[b] - ar
        rho[b] = rr * np.exp((u[b] - ur) / ar)
        c = rm & (xi < tail)
        rho[c], u[c] = rrs, urs
    return rho, u
