"""Seeded synthetic inputs for the full-Euler instance of the method: ideal gas
on a fixed mesh with one small cell (the first test of Sec. 4, the Lax shock
tube with the local pseudo time step factors theta_i).

Like ``workloads``, this module only lays out grids, initial data and run
parameters; the HIP path and the CPU oracle consume the same arrays.

Mesh of problem b (Fig. 1 with alpha h small cell): ``N[b]`` regular cells of
length ``h[b]`` and one small cell of length ``alpha[b] h[b]`` at position
``N[b] // 2``, whose left face is at x = 0; ``N[b] + 1`` cells from
``off[b]`` in the flattened conserved arrays (rho, m = rho u, E).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4

# initial data of the Lax shock tube, (rho, u, p) left and right of x = 0
LAX_LEFT = (0.445, 0.698, 3.528)
LAX_RIGHT = (0.5, 0.0, 0.571)


@dataclass
class EulerBatch:
    N: np.ndarray        # int32 [P] regular cells (even)
    h: np.ndarray        # f64 [P] regular cell length
    x_left: np.ndarray   # f64 [P] left end of the domain
    alpha: np.ndarray    # f64 [P] small-cell length / h
    theta_nb: np.ndarray  # f64 [P] theta_{k-1} = theta_{k+1}
    theta_k: np.ndarray  # f64 [P] theta_k
    cfl: np.ndarray      # f64 [P] C_CFL
    t_end: np.ndarray    # f64 [P]
    rho: np.ndarray      # f64 [cells]
    mom: np.ndarray
    ene: np.ndarray
    gamma: float = GAMMA
    tol_nb: float = 1e-3
    tol_k: float = 1e-1
    lmax: int = 10_000_000
    name: str = "euler"
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
    def n_cells(self) -> int:
        return int(self.off[-1])

    def copy(self) -> "EulerBatch":
        return dataclasses.replace(
            self, **{f.name: np.array(getattr(self, f.name), copy=True)
                     for f in dataclasses.fields(self)
                     if isinstance(getattr(self, f.name), np.ndarray)})

    def replace(self, **kw) -> "EulerBatch":
        return dataclasses.replace(self, **kw)

    def subset(self, idx) -> "EulerBatch":
        idx = np.asarray(idx, dtype=np.int64)
        o = self.off
        cells = lambda a: (np.concatenate([a[o[p]:o[p + 1]] for p in idx])
                           if len(idx) else a[:0].copy())
        per = {f: getattr(self, f)[idx].copy() for f in
               ("N", "h", "x_left", "alpha", "theta_nb", "theta_k", "cfl", "t_end")}
        return dataclasses.replace(self, **per, rho=cells(self.rho), mom=cells(self.mom),
                                   ene=cells(self.ene), name=f"{self.name}[subset]")


def conserved(gamma, rho, u, p):
    """(rho, rho u, E) of primitive ideal-gas data, E = p/(gamma-1) + rho u^2/2."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    return rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u


def _tube(N, alpha, left, right, x_l=-5.0, x_r=5.0, gamma=GAMMA):
    if N < 4 or N % 2:
        raise ValueError("N must be even and at least 4")
    k = N // 2
    prim = np.empty((N + 1, 3))
    prim[:k] = left
    prim[k:] = right
    r, m, e = conserved(gamma, prim[:, 0], prim[:, 1], prim[:, 2])
    return (x_r - x_l) / N, r, m, e


def _concat(specs, name, gamma=GAMMA, meta=None, **glob):
    """specs: list of dicts with N, alpha, theta_nb, theta_k, cfl, t_end, left,
    right, x_l, x_r."""
    cols = {f: [] for f in ("N", "h", "x_left", "alpha", "theta_nb", "theta_k", "cfl", "t_end")}
    rho, mom, ene = [], [], []
    for s in specs:
        h, r, m, e = _tube(s["N"], s["alpha"], s["left"], s["right"], s["x_l"], s["x_r"], gamma)
        cols["N"].append(s["N"])
        cols["h"].append(h)
        cols["x_left"].append(s["x_l"])
        for f in ("alpha", "theta_nb", "theta_k", "cfl", "t_end"):
            cols[f].append(s[f])
        rho.append(r)
        mom.append(m)
        ene.append(e)
    cat = lambda a: np.concatenate(a) if a else np.zeros(0)
    return EulerBatch(np.asarray(cols["N"], dtype=np.int32),
                      *(np.asarray(cols[f], dtype=np.float64) for f in
                        ("h", "x_left", "alpha", "theta_nb", "theta_k", "cfl", "t_end")),
                      cat(rho), cat(mom), cat(ene), gamma=gamma, name=name,
                      meta=dict(meta or {}), **glob)


def lax_spec(N=100, alpha=1e-2, theta_nb=0.9, theta_k=None, cfl=0.8, t_end=1.0,
             left=LAX_LEFT, right=LAX_RIGHT, x_l=-5.0, x_r=5.0):
    return dict(N=int(N), alpha=float(alpha), theta_nb=float(theta_nb),
                theta_k=float(alpha if theta_k is None else theta_k), cfl=float(cfl),
                t_end=float(t_end), left=tuple(left), right=tuple(right), x_l=x_l, x_r=x_r)


def lax_tube(N=100, alpha=1e-2, theta_nb=0.9, theta_k=None, **kw):
    """The Lax shock tube of Sec. 4 on [-5, 5 + alpha h], C_CFL = 0.8,
    t_end = 1, theta_k = alpha unless given."""
    return _concat([lax_spec(N, alpha, theta_nb, theta_k, **kw)], name=f"lax_N{N}_a{alpha:g}")


# the configurations of the paper's table of average dual time iterations
# (Sec. 4, Lax shock tube): (theta_{k+-1}, N, alpha), theta_{k+-1} = None
# meaning theta_{k+-1} = alpha
LAX_STUDY = ([(th, N, a) for th in (0.9, 0.1) for N in (100, 200, 400) for a in (1e-2, 1e-4, 1e-6)]
             + [(None, N, a) for N in (100, 200, 400) for a in (1e-2, 1e-4, 1e-5)])


def lax_study(entries=None):
    """One problem per configuration (theta_nb, N, alpha), LAX_STUDY by default."""
    entries = list(LAX_STUDY) if entries is None else list(entries)
    specs = [lax_spec(N, a, a if th is None else th) for th, N, a in entries]
    return _concat(specs, name="lax_study", meta={"entries": entries})


def lax_batch(seed=20261202, n_problems=4096, Ns=(100, 200, 400), alpha_lo=1e-6, alpha_hi=1e-2,
              thetas=(0.9, 0.1), spread=0.25):
    """An ensemble of Lax-type shock tubes: N drawn from Ns, alpha log-uniform
    in [alpha_lo, alpha_hi], theta_{k+-1} drawn from thetas, theta_k = alpha,
    and each of rho, p on both sides scaled by a factor log-uniform in
    [1/(1+spread), 1+spread] and u_L by one uniform in [1-spread, 1+spread]."""
    rng = np.random.default_rng(seed)
    specs = []
    lo, hi = math.log(1.0 / (1.0 + spread)), math.log(1.0 + spread)
    for _ in range(n_problems):
        N = int(rng.choice(Ns))
        a = float(math.exp(rng.uniform(math.log(alpha_lo), math.log(alpha_hi))))
        th = float(rng.choice(thetas))
        f = np.exp(rng.uniform(lo, hi, 4))
        left = (LAX_LEFT[0] * f[0], LAX_LEFT[1] * rng.uniform(1 - spread, 1 + spread),
                LAX_LEFT[2] * f[1])
        right = (LAX_RIGHT[0] * f[2], LAX_RIGHT[1], LAX_RIGHT[2] * f[3])
        specs.append(lax_spec(N, a, th, None, left=left, right=right))
    return _concat(specs, name=f"lax_batch_P{n_problems}_seed{seed}",
                   meta={"seed": seed, "Ns": tuple(Ns), "alpha": (alpha_lo, alpha_hi),
                         "thetas": tuple(thetas), "spread": spread})
