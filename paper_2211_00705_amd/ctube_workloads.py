"""Seeded synthetic inputs for creation tubes: the cavitation and nucleation
tests of Sec. 4 run through the whole scheme (phase creation on a face, then
a created cell between two phase boundaries), and ensembles around them.

Like ``workloads``, this module only lays out grids, initial data and run
parameters; the HIP path and the CPU oracle consume the same arrays.

Tube p: ``N[p]`` regular cells of length ``h[p]`` from ``x_left[p]``, all of
phase ``phase[p]`` (0 liquid, 1 vapour), the initial jump on the face
``N[p] // 2``; ``N[p] + 1`` slots from ``off[p]`` in the flat (rho, rho u)
arrays, the last one holding the created cell once there is one (zero
before).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

from .workloads import LIQ, P_MIN, P_TILDE, VAP, WATER_363K, Params, _rho_of_p

# the Sec. 4 runs: C_CFL = 0.5, h = 1e-2 m on [-2, 2] m, t_end = 5e-4 s;
# zone of the created cell +- 1 cell, the paper's stop rule
CT_PARAMS = Params(cfl=0.5, zone_half=1, theta_nb=0.9, tol_mode=0, tol_nb=1e-3, tol_tiny=1e-1,
                   lmax=100_000, bc_left=1, bc_right=1, t_end=5e-4)

# initial data (p, u) left and right of x = 0
CAVITATION = (LIQ, (60000.0, -4.0), (60000.0, 4.0))
NUCLEATION = (VAP, (70000.0, 2.7), (70000.0, -2.7))


@dataclass
class CTubeBatch:
    N: np.ndarray        # int32 [P] regular cells (even)
    h: np.ndarray        # f64 [P]
    x_left: np.ndarray   # f64 [P]
    phase: np.ndarray    # int32 [P] phase of the regular cells
    rho: np.ndarray      # f64 [slots]
    mom: np.ndarray
    params: Params = field(default_factory=lambda: CT_PARAMS)
    p_min: float = P_MIN
    p_tilde: float = P_TILDE
    material: object = WATER_363K
    name: str = "ctube"
    meta: dict = field(default_factory=dict)

    @property
    def n_problems(self) -> int:
        return int(self.N.shape[0])

    @property
    def off(self) -> np.ndarray:
        o = np.zeros(self.n_problems + 1, dtype=np.int64)
        np.cumsum(self.N.astype(np.int64) + 1, out=o[1:])
        return o

    @property
    def n_slots(self) -> int:
        return int(self.off[-1])

    def copy(self) -> "CTubeBatch":
        return dataclasses.replace(
            self, **{f.name: np.array(getattr(self, f.name), copy=True)
                     for f in dataclasses.fields(self)
                     if isinstance(getattr(self, f.name), np.ndarray)})

    def replace(self, **kw) -> "CTubeBatch":
        return dataclasses.replace(self, **kw)

    def with_params(self, **kw) -> "CTubeBatch":
        return dataclasses.replace(self, params=self.params.replace(**kw))

    def subset(self, idx) -> "CTubeBatch":
        idx = np.asarray(idx, dtype=np.int64)
        o = self.off
        cells = lambda a: (np.concatenate([a[o[p]:o[p + 1]] for p in idx])
                           if len(idx) else a[:0].copy())
        per = {f: getattr(self, f)[idx].copy() for f in ("N", "h", "x_left", "phase")}
        return dataclasses.replace(self, **per, rho=cells(self.rho), mom=cells(self.mom),
                                   name=f"{self.name}[subset]")


def _tube(material, N, phase, left, right):
    if N < 4 or N % 2:
        raise ValueError("N must be even and at least 4")
    k = N // 2
    p = np.empty(N)
    u = np.empty(N)
    p[:k], u[:k] = left
    p[k:], u[k:] = right
    r = np.zeros(N + 1)
    m = np.zeros(N + 1)
    r[:N] = _rho_of_p(material, phase, p)
    m[:N] = r[:N] * u
    return r, m


def concat(specs, name, params=CT_PARAMS, material=WATER_363K, meta=None):
    """specs: dicts with N, h, phase, left = (p, u), right = (p, u); the
    domain is centred on the jump (x_left = -N h / 2)."""
    rho, mom = [], []
    for s in specs:
        r, m = _tube(material, s["N"], s["phase"], s["left"], s["right"])
        rho.append(r)
        mom.append(m)
    cat = lambda a: np.concatenate(a) if a else np.zeros(0)
    N = np.asarray([s["N"] for s in specs], dtype=np.int32)
    h = np.asarray([s["h"] for s in specs], dtype=np.float64)
    return CTubeBatch(N, h, -0.5 * N * h, np.asarray([s["phase"] for s in specs], dtype=np.int32),
                      cat(rho), cat(mom), params=params, material=material, name=name,
                      meta=dict(meta or {}))


def spec(case, N=400, h=1e-2):
    ph, left, right = case
    return dict(N=int(N), h=float(h), phase=int(ph), left=tuple(left), right=tuple(right))


def cavitation_tube(N=400, h=1e-2, **kw):
    """The cavitation test of Sec. 4: liquid at 60000 Pa pulled apart at
    -/+4 m/s, [-2, 2] m with h = 1e-2 m for N = 400."""
    return concat([spec(CAVITATION, N, h)], name=f"cavitation_N{N}", **kw)


def nucleation_tube(N=400, h=1e-2, **kw):
    """The nucleation test of Sec. 4: vapour at 70000 Pa compressed at
    +/-2.7 m/s."""
    return concat([spec(NUCLEATION, N, h)], name=f"nucleation_N{N}", **kw)


def ctube_batch(seed=20261202, n_problems=4096, Ns=(200, 400, 800), h=1e-2, params=None):
    """Tubes around the two tests, alternating: liquid ones with p ~ U[4e4,
    9e4] Pa on each side pulled apart at u_l = -U[1, 6], u_r = U[1, 6] m/s
    (cavitation), vapour ones with p ~ U[6.998e4, 7.01e4] Pa compressed at
    u_l = U[2.6, 3], u_r = -U[2.6, 3] m/s (nucleation: the single-phase star
    pressure exceeds p~, close to the paper's test); N drawn from Ns with h
    fixed, so every phase boundary stays inside its neighbour cells up to
    t_end = 5e-4 s."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_problems):
        N = int(rng.choice(Ns))
        if i % 2 == 0:
            pl, pr = rng.uniform(4e4, 9e4, 2)
            ul, ur = -rng.uniform(1.0, 6.0), rng.uniform(1.0, 6.0)
            specs.append(dict(N=N, h=h, phase=LIQ, left=(pl, ul), right=(pr, ur)))
        else:
            pl, pr = rng.uniform(6.998e4, 7.01e4, 2)
            ul, ur = rng.uniform(2.6, 3.0), -rng.uniform(2.6, 3.0)
            specs.append(dict(N=N, h=h, phase=VAP, left=(pl, ul), right=(pr, ur)))
    return concat(specs, name=f"ctube_batch_P{n_problems}_seed{seed}",
                  params=params or CT_PARAMS, meta={"seed": seed, "Ns": tuple(Ns), "h": h})
