"""Material constants of the paper's isothermal water model, derived.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

* Vapour: ideal gas p = (k T0 / m) rho with the printed Boltzmann constant and
  molecule mass (Sec. 4, eq. eos:isoT_idgas).
* Kinetic coefficient tau = (2 pi)^(-1/2) (m / (k T0))^(3/2) (Sec. 4).
* Liquid: linear Tait law, read as p = p0 + K0 (rho/rho0 - 1) (the printed
  "- p0" inside the bracket is dimensionally inconsistent).  rho0 and K0 come
  from steam tables in the paper and are not printed; they are recovered
  here from what is printed: the liquid branch ends at p_min = 0 Pa at
  rho_min (table of maximum vapour / minimum liquid pressure), the vapour
  branch at p~ (same table), the two are joined linearly in density, and the
  Maxwell equal-area rule holds (Sec. 2.1 and the sentence after the Tait
  law).  The equal-area integral is evaluated in closed form, piece by piece.
"""
from __future__ import annotations

import math

K_BOLTZMANN = 1.380658e-23  # J/K, printed with eq. eos:isoT_idgas
T0 = 363.15  # K, saturation-values table of the cavitation test
M_WATER = (2 * 1.0079 + 15.9994) / 6.02205e26  # kg, printed with eq. eos:isoT_idgas
P0 = 70182.360745  # Pa, printed saturation pressure at T0
P_TILDE = 70388.660656  # Pa, maximum vapour pressure (table)
RHO_TILDE_PRINTED = 0.419977  # kg/m^3 (table)
P_MIN = 0.0  # Pa, minimum liquid pressure (table)
RHO_MIN = 965.289008  # kg/m^3 (table)


def a2_vapour():
    return K_BOLTZMANN * T0 / M_WATER


def kinetic_tau():
    return (1.0 / math.sqrt(2.0 * math.pi)) * (M_WATER / (K_BOLTZMANN * T0)) ** 1.5


def equal_area(rho0, a2v=None):
    """Integral of (p(v) - p0) dv over the isotherm from the liquid to the
    vapour saturation volume, in closed form, for a liquid branch through
    (rho_min, p_min) with saturation density rho0."""
    a2v = a2_vapour() if a2v is None else a2v
    rv0 = P0 / a2v
    rt = P_TILDE / a2v
    a2l = (P0 - P_MIN) / (rho0 - RHO_MIN)  # p_L(rho_min) = p_min with p_L = p0 + a2l (rho - rho0)
    # in density: dv = -drho / rho^2, so the integral is  int_{rv0}^{rho0} (p - p0)/rho^2 drho
    vap = a2v * math.log(rt / rv0) + P0 * (1.0 / rt - 1.0 / rv0)
    s = (P_MIN - P_TILDE) / (RHO_MIN - rt)
    c = P_TILDE - s * rt - P0
    conn = c * (1.0 / rt - 1.0 / RHO_MIN) + s * math.log(RHO_MIN / rt)
    liq = a2l * math.log(rho0 / RHO_MIN) + a2l * rho0 * (1.0 / rho0 - 1.0 / RHO_MIN)
    return vap + conn + liq


def derive_liquid():
    """(rho0, a2l = K0/rho0) such that the equal-area integral vanishes."""
    lo, hi = RHO_MIN + 1e-3, RHO_MIN + 1.0
    flo = equal_area(lo)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = equal_area(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
        if hi - lo < 1e-13:
            break
    rho0 = 0.5 * (lo + hi)
    a2l = (P0 - P_MIN) / (rho0 - RHO_MIN)
    return rho0, a2l


def derive():
    """All five material numbers as a dict."""
    rho0, a2l = derive_liquid()
    return {"a2v": a2_vapour(), "a2l": a2l, "p0": P0, "rhol0": rho0, "tau": kinetic_tau()}
