"""Seeded synthetic inputs for the IMEX-DS hot path.

This module only draws numbers: grids, interface positions, phase states and
run parameters.  It holds none of the method's arithmetic, so both the HIP
path and the CPU oracle consume exactly the same inputs from it.

Material constants (water at T0 = 363.15 K) are stored as numbers with their
provenance:

* ``a2v = k T0 / m`` with Boltzmann's constant and the molecule mass printed
  with the ideal-gas law (Sec. 4, eq. eos:isoT_idgas);
* ``p0`` is the printed saturation pressure (cavitation initial-data table);
* ``tau = (2 pi)^(-1/2) (m / k T0)^(3/2)`` (Sec. 4, kinetic coefficient);
* ``rhol0`` and ``a2l = K0 / rho0`` of the linear Tait law are not printed (the
  paper takes them from steam tables); they are recovered from the printed
  p_min = 0 Pa at rho_min = 965.289008 kg/m^3 and the Maxwell equal-area rule
  with a connector linear in density (Sec. 4, table of p~, rho~, p_min,
  rho_min).  The derivation lives with the CPU oracle and a test checks these
  numbers against it.

Each generator's docstring states the shapes and distributions it draws.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

LIQ = 0
VAP = 1


@dataclass(frozen=True)
class Material:
    a2v: float = 167601.31868960848  # m^2/s^2, vapour: p = a2v * rho
    a2l: float = 2188937.119804053  # m^2/s^2, liquid: p = p0 + a2l (rho - rhol0)
    p0: float = 70182.360745  # Pa, saturation pressure at 363.15 K
    rhol0: float = 965.3210703009725  # kg/m^3, liquid saturation density
    tau: float = 5.814252908638165e-09  # s^3/m^3, kinetic coefficient


WATER_363K = Material()


@dataclass
class Params:
    cfl: float = 0.9
    zone_half: int = 2
    theta_nb: float = 0.9
    tol_mode: int = 0  # 0: paper residual (tol_nb / tol_tiny); 1: relative update
    tol_nb: float = 1e-3
    tol_tiny: float = 1e-1
    tol_rel: float = 1e-12
    lmax: int = 100
    alpha_floor: float = 1e-6
    merge_safety: float = 1.5
    bc_left: int = 0  # 0 wall, 1 transmissive
    bc_right: int = 0
    newton_maxit: int = 50
    newton_rtol: float = 1e-10
    t_end: float = math.inf
    zone_solver: int = 0  # 0: Algorithm 2 (dual time stepping); 1: Newton on the implicit step
    zn_maxit: int = 30    # Newton zone solver: at most this many steps
    zn_rtol: float = 1e-10  # Newton zone solver: relative step tolerance

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclass
class Batch:
    """Independent 1D problems, flattened.

    Problem p has ``n_cells[p]`` background cells of width ``h[p]`` starting at
    ``x_left[p]`` and interfaces ``iface_off[p]:iface_off[p+1]``.  Interface k
    lies in background cell ``home[k]`` at offset ``hl[k]`` (0 < hl < h) and
    cuts it into two slots; so problem p owns ``n_cells + n_iface`` slots,
    laid out left to right.  ``phase_first`` is the phase of the first slot
    (0 liquid, 1 vapour); phases alternate across interfaces.
    """

    n_cells: np.ndarray
    h: np.ndarray
    x_left: np.ndarray
    phase_first: np.ndarray
    iface_off: np.ndarray
    home: np.ndarray
    hl: np.ndarray
    rho: np.ndarray
    mom: np.ndarray
    name: str = "batch"
    meta: dict = field(default_factory=dict)

    @property
    def n_problems(self) -> int:
        return int(self.n_cells.shape[0])

    @property
    def n_iface(self) -> int:
        return int(self.iface_off[-1])

    @property
    def slot_off(self) -> np.ndarray:
        ns = self.n_cells.astype(np.int64) + np.diff(self.iface_off).astype(np.int64)
        off = np.zeros(self.n_problems + 1, dtype=np.int64)
        np.cumsum(ns, out=off[1:])
        return off

    @property
    def n_slots(self) -> int:
        return int(self.slot_off[-1])

    def copy(self) -> "Batch":
        return dataclasses.replace(
            self,
            **{f.name: np.array(getattr(self, f.name), copy=True)
               for f in dataclasses.fields(self) if isinstance(getattr(self, f.name), np.ndarray)},
        )

    def subset(self, idx) -> "Batch":
        """The problems ``idx`` (in that order) as a batch of their own."""
        idx = np.asarray(idx, dtype=np.int64)
        so = self.slot_off
        io = self.iface_off.astype(np.int64)
        rho = np.concatenate([self.rho[so[p]:so[p + 1]] for p in idx])
        mom = np.concatenate([self.mom[so[p]:so[p + 1]] for p in idx])
        home = np.concatenate([self.home[io[p]:io[p + 1]] for p in idx]) if len(idx) else self.home[:0]
        hl = np.concatenate([self.hl[io[p]:io[p + 1]] for p in idx]) if len(idx) else self.hl[:0]
        nif = (io[idx + 1] - io[idx]).astype(np.int32)
        ioff = np.zeros(len(idx) + 1, dtype=np.int32)
        np.cumsum(nif, out=ioff[1:])
        return Batch(self.n_cells[idx].copy(), self.h[idx].copy(), self.x_left[idx].copy(),
                     self.phase_first[idx].copy(), ioff, home.astype(np.int32), hl, rho, mom,
                     name=f"{self.name}[subset]", meta=dict(self.meta))


def _assemble(n_cells, h, x_left, phase_first, homes, hls, cell_states, name, meta=None):
    """Builds slot arrays from per-problem lists.

    ``cell_states[p]`` is a callable ``(x_centres, phase) -> (rho, u)`` giving
    the initial state at slot centres of the given phase.
    """
    P = len(n_cells)
    iface_off = np.zeros(P + 1, dtype=np.int32)
    iface_off[1:] = np.cumsum([len(hs) for hs in homes])
    rho_all, mom_all = [], []
    for p in range(P):
        n, hp, x0 = int(n_cells[p]), float(h[p]), float(x_left[p])
        hs = np.asarray(list(homes[p]), dtype=np.int64)
        ls = np.asarray(list(hls[p]), dtype=np.float64)
        edges = x0 + np.arange(n + 1, dtype=np.float64) * hp
        xi = edges[hs] + ls
        lefts = np.insert(edges[:-1], hs + 1, xi)
        rights = np.insert(edges[1:], hs, xi)
        xc = 0.5 * (lefts + rights)
        k = len(hs)
        right_piece = hs + np.arange(k) + 1
        flips = np.searchsorted(right_piece, np.arange(n + k), side="right")
        phases = (int(phase_first[p]) + flips) & 1
        rho = np.empty_like(xc)
        u = np.empty_like(xc)
        for q in (LIQ, VAP):
            sel = phases == q
            if sel.any():
                r, v = cell_states[p](xc[sel], q)
                rho[sel] = r
                u[sel] = v
        rho_all.append(rho)
        mom_all.append(rho * u)
    home = np.asarray([c for hs in homes for c in hs], dtype=np.int32)
    hl = np.asarray([v for ls in hls for v in ls], dtype=np.float64)
    return Batch(np.asarray(n_cells, dtype=np.int32), np.asarray(h, dtype=np.float64),
                 np.asarray(x_left, dtype=np.float64), np.asarray(phase_first, dtype=np.int32),
                 iface_off, home, hl, np.concatenate(rho_all) if P else np.zeros(0),
                 np.concatenate(mom_all) if P else np.zeros(0), name=name, meta=dict(meta or {}))


def _const_states(rng, liq=(900.0, 1000.0), vap=(0.01, 0.1), uliq=(-1.0, 1.0), uvap=(-1.0, 1.0)):
    rl, ul = rng.uniform(*liq), rng.uniform(*uliq)
    rv, uv = rng.uniform(*vap), rng.uniform(*uvap)

    def states(x, q):
        if q == LIQ:
            return np.full(x.shape, rl), np.full(x.shape, ul)
        return np.full(x.shape, rv), np.full(x.shape, uv)

    return states


def loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


# ---------------------------------------------------------------------------
# paper-scale workloads
# ---------------------------------------------------------------------------

def single_cut_problem(seed=0, n=200, alpha=1e-4):
    """One liquid|vapour problem on [0,1], interface at x = 0.5 + alpha h.

    Liquid left rho ~ U[900, 1000], u ~ U[-1, 1]; vapour right
    rho ~ U[0.01, 0.1], u ~ U[-1, 1]; the cut piece [0.5, x_I] of length
    alpha h is the tiny cell.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / n
    st = _const_states(rng)
    return _assemble([n], [h], [0.0], [LIQ], [[n // 2]], [[alpha * h]], [st],
                     name=f"single_cut_n{n}_seed{seed}", meta={"alpha": alpha})


def single_cut_params():
    """Run parameters of the single 200-cell problem: CFL 0.9, zone = cut
    cell +- 2, dual time stepping to a 1e-12 relative update, walls, t = 0.1."""
    return Params(cfl=0.9, zone_half=2, tol_mode=1, tol_rel=1e-12, lmax=10000, t_end=0.1)


def _fourier(rng, x, n_modes=4, kmax=8):
    ks = rng.integers(1, kmax + 1, size=n_modes)
    amp = rng.uniform(0.2, 1.0, size=n_modes)
    ph = rng.uniform(0.0, 2 * math.pi, size=n_modes)
    s = sum(a * np.sin(2 * math.pi * k * x + f) for a, k, f in zip(amp, ks, ph))
    return s / amp.sum()


def large_smooth_problem(seed=0, n=1 << 20, alpha=None):
    """One large problem: n cells on [0,1], one interface in cell n/2 with
    cut fraction alpha ~ logU[1e-6, 1e-1]; piecewise-smooth states per phase:
    rho = lo + (hi - lo)(1/2 + s(x)/2) with s a normalised sum of 4 random
    Fourier modes, u = 0.5 * (another such sum scaled to unit RMS)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if alpha is None:
        alpha = float(loguniform(rng, 1e-6, 1e-1))
    h = 1.0 / n
    seeds = rng.integers(0, 2**62, size=4)

    def states(x, q):
        lo, hi = (900.0, 1000.0) if q == LIQ else (0.01, 0.1)
        r1 = np.random.Generator(np.random.PCG64(int(seeds[2 * q])))
        r2 = np.random.Generator(np.random.PCG64(int(seeds[2 * q + 1])))
        xs = np.linspace(0.0, 1.0, 4097)
        s = _fourier(r1, x)
        v = _fourier(r2, x)
        vs = _fourier(np.random.Generator(np.random.PCG64(int(seeds[2 * q + 1]))), xs)
        rms = float(np.sqrt(np.mean(vs * vs)))
        return lo + (hi - lo) * (0.5 + 0.5 * s), 0.5 * v / rms

    return _assemble([n], [h], [0.0], [LIQ], [[n // 2]], [[alpha * h]], [states],
                     name=f"large_smooth_n{n}_seed{seed}", meta={"alpha": alpha})


def large_smooth_params():
    """Paper's residual rule (1e-3 / 1e-1), at most 100 pseudo-steps, zone of
    5 cells, walls, CFL 0.9."""
    return Params(cfl=0.9, zone_half=2, tol_mode=0, lmax=100)


def random_batch(seed=20261202, n_problems=4096, nmin=256, nmax=16384, alpha_lo=1e-6,
                 alpha_hi=1e-1):
    """Independent liquid|vapour problems on [0,1] with uneven sizes.

    N_p = floor(exp(U[ln nmin, ln(nmax+1))))  (log-uniform integer), interface
    home cell j ~ U{ceil(N/4) .. floor(3N/4)}, cut fraction
    alpha ~ logU[alpha_lo, alpha_hi] with the tiny piece on the liquid side,
    constant states per phase drawn as for the single problem.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    P = n_problems
    N = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax + 1), size=P))).astype(np.int64)
    N = np.clip(N, nmin, nmax)
    homes, hls, states, hs = [], [], [], []
    for p in range(P):
        n = int(N[p])
        h = 1.0 / n
        j = int(rng.integers(math.ceil(n / 4), math.floor(3 * n / 4) + 1))
        a = float(loguniform(rng, alpha_lo, alpha_hi))
        homes.append([j])
        hls.append([a * h])
        hs.append(h)
        states.append(_const_states(rng))
    return _assemble(N, hs, np.zeros(P), np.zeros(P, dtype=np.int32), homes, hls, states,
                     name=f"random_batch_P{P}_seed{seed}")


def random_batch_params():
    return Params(cfl=0.9, zone_half=2, tol_mode=0, lmax=100)


def adjoint_batch(seed=20261202, n_problems=1024, nmin=256, nmax=16384):
    """Batch for the adjoint: per problem the large single problem's set-up
    (piecewise-smooth states from random Fourier modes, one interface in cell
    N/2 with cut fraction alpha ~ logU[1e-6, 1e-1]) at the uneven sizes of the
    random batch, N_p log-uniform integer in [nmin, nmax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = n_problems
    N = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax + 1), size=P))).astype(np.int64)
    N = np.clip(N, nmin, nmax)
    homes, hls, states, hs = [], [], [], []
    for p in range(P):
        n = int(N[p])
        h = 1.0 / n
        a = float(loguniform(rng, 1e-6, 1e-1))
        seeds = rng.integers(0, 2**62, size=4)

        def st(x, q, seeds=seeds):
            lo, hi = (900.0, 1000.0) if q == LIQ else (0.01, 0.1)
            s_ = _fourier(np.random.Generator(np.random.PCG64(int(seeds[2 * q]))), x)
            v = _fourier(np.random.Generator(np.random.PCG64(int(seeds[2 * q + 1]))), x)
            xs = np.linspace(0.0, 1.0, 1025)
            vs = _fourier(np.random.Generator(np.random.PCG64(int(seeds[2 * q + 1]))), xs)
            rms = float(np.sqrt(np.mean(vs * vs)))
            return lo + (hi - lo) * (0.5 + 0.5 * s_), 0.5 * v / rms

        homes.append([n // 2])
        hls.append([a * h])
        hs.append(h)
        states.append(st)
    return _assemble(N, hs, np.zeros(P), np.zeros(P, dtype=np.int32), homes, hls, states,
                     name=f"adjoint_batch_P{P}_seed{seed}")


def adjoint_batch_params():
    return Params(cfl=0.9, zone_half=2, tol_mode=0, lmax=100)


def bubble_batch(seed=20261202, n_problems=1024, n=4096, gap=16, alpha_lo=1e-6, alpha_hi=1e-2):
    """Liquid | vapour bubble | liquid problems: two interfaces around `gap`
    full vapour cells in the middle of the domain; each interface's tiny piece
    is on the vapour side with alpha ~ logU[alpha_lo, alpha_hi].  Liquid
    rho ~ U[900, 1000] pulled apart (left u = -U[0,2], right u = +U[0,2]);
    vapour rho ~ U[0.01, 0.1] at rest."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = n_problems
    h = 1.0 / n
    homes, hls, states = [], [], []
    for p in range(P):
        jA = n // 2 - gap // 2 - 1
        jB = jA + gap + 1
        aA = float(loguniform(rng, alpha_lo, alpha_hi))
        aB = float(loguniform(rng, alpha_lo, alpha_hi))
        homes.append([jA, jB])
        hls.append([h - aA * h, aB * h])
        rlL, rlR = rng.uniform(900.0, 1000.0, size=2)
        uL, uR = -rng.uniform(0.0, 2.0), rng.uniform(0.0, 2.0)
        rv = rng.uniform(0.01, 0.1)

        def st(x, q, rlL=rlL, rlR=rlR, uL=uL, uR=uR, rv=rv):
            if q == VAP:
                return np.full(x.shape, rv), np.zeros(x.shape)
            left = x < 0.5
            return np.where(left, rlL, rlR), np.where(left, uL, uR)

        states.append(st)
    return _assemble([n] * P, [h] * P, np.zeros(P), np.zeros(P, dtype=np.int32), homes, hls,
                     states, name=f"bubble_batch_P{P}_seed{seed}")


def bubble_batch_params():
    return Params(cfl=0.9, zone_half=2, tol_mode=0, lmax=100)


def riemann_problem(n, left, right, j=None, alpha=0.5, phases=(LIQ, VAP), length=1.0):
    """A single two-phase Riemann problem with constant (rho, u) states on
    [0, length]: n cells, interface at (j + alpha) h inside cell j
    (default j = n // 2)."""
    h = length / n
    if j is None:
        j = n // 2

    def st(x, q):
        s = left if q == phases[0] else right
        return np.full(x.shape, float(s[0])), np.full(x.shape, float(s[1]))

    return _assemble([n], [h], [0.0], [phases[0]], [[j]], [[alpha * h]], [st], name="riemann")


def single_phase_problem(n, rho_fn, u_fn, phase=LIQ, length=1.0):
    """A problem without interfaces: n cells of one phase with the given
    initial profiles (functions of the cell centre)."""
    h = length / n

    def st(x, q):
        return rho_fn(x), u_fn(x)

    return _assemble([n], [h], [0.0], [phase], [[]], [[]], [st], name="single_phase")


# ---------------------------------------------------------------------------
# single-phase Riemann problems for phase creation (cavitation, nucleation)
# ---------------------------------------------------------------------------

# creation thresholds at 363.15 K (Sec. 4, table of the maximum vapour
# pressure and the minimum liquid pressure)
P_MIN = 0.0
P_TILDE = 70388.660656


@dataclass
class CreationBatch:
    phase: np.ndarray  # int32 [n]: 0 liquid, 1 vapour (both states)
    rho_l: np.ndarray
    mom_l: np.ndarray
    rho_r: np.ndarray
    mom_r: np.ndarray
    name: str = "creation"

    @property
    def n(self) -> int:
        return int(self.phase.shape[0])


def _rho_of_p(material, ph, p):
    p = np.asarray(p, dtype=np.float64)
    return p / material.a2v if ph == VAP else material.rhol0 + (p - material.p0) / material.a2l


def creation_problem(material, phase, pl, ul, pr, ur):
    """One problem from pressures and velocities (the Sec. 4 tests: liquid
    60000 Pa at -/+4 m/s, vapour 70000 Pa at +/-2.7 m/s)."""
    rl, rr = _rho_of_p(material, phase, pl), _rho_of_p(material, phase, pr)
    return CreationBatch(np.array([phase], np.int32), np.array([rl]), np.array([rl * ul]),
                         np.array([rr]), np.array([rr * ur]), name="creation_problem")


def creation_batch(material, seed=20261202, n=1 << 20):
    """Single-phase Riemann problems around the paper's two creation tests:
    half liquid (p ~ U[2e4, 1e5] Pa on each side, u_l, u_r ~ U[-3, 3] m/s:
    pulled apart and cavitating, or compressed), half vapour
    (p ~ U[6.9e4, 7.035e4] Pa, u_l ~ U[-2, 8], u_r ~ U[-8, 2]: compressed,
    nucleating when hard enough, or expanding), phases interleaved."""
    rng = np.random.default_rng(seed)
    ph = (np.arange(n) & 1).astype(np.int32)
    pl = np.where(ph == LIQ, rng.uniform(2e4, 1e5, n), rng.uniform(6.9e4, 7.035e4, n))
    pr = np.where(ph == LIQ, rng.uniform(2e4, 1e5, n), rng.uniform(6.9e4, 7.035e4, n))
    ul = np.where(ph == LIQ, rng.uniform(-3.0, 3.0, n), rng.uniform(-2.0, 8.0, n))
    ur = np.where(ph == LIQ, rng.uniform(-3.0, 3.0, n), rng.uniform(-8.0, 2.0, n))
    rl = np.where(ph == LIQ, _rho_of_p(material, LIQ, pl), _rho_of_p(material, VAP, pl))
    rr = np.where(ph == LIQ, _rho_of_p(material, LIQ, pr), _rho_of_p(material, VAP, pr))
    return CreationBatch(ph, rl, rl * ul, rr, rr * ur, name=f"creation_batch_n{n}_seed{seed}")
