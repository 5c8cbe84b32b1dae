"""The creation-tube oracle (a created cell inside the mesh: appendix "Phase
Creation" step (iv), then two phase boundaries, Sec. 3 with Algorithm 2)
pinned on what the paper prints for its cavitation and nucleation tests and
on what the mathematics fixes: conservation, mirror symmetry, the plain
explicit HLL scheme where nothing is created, and the status paths."""
import numpy as np
import pytest

import oracle
from paper_2211_00705_amd import ctube_workloads as CW
from paper_2211_00705_amd.workloads import LIQ, VAP

M = CW.WATER_363K


def pres(ph, r):
    return M.a2v * r if ph == VAP else M.p0 + M.a2l * (r - M.rhol0)


def run(b, n_steps=None, log=False, threads=4):
    st = oracle.CTubeState(b)
    out = oracle.ct_run(st, n_steps, threads=threads, log=log)
    return (st, out) if log else st


def star_cells(st, b, p=0):
    """(p, u) of the cell left of the created one, the created one, the cell
    right of it."""
    o, N, f, ph = b.off[p], b.N[p], st.face[p], b.phase[p]
    res = []
    for s, phs in ((f - 1, ph), (N, 1 - ph), (f, ph)):
        r, m = st.rho[o + s], st.mom[o + s]
        res.append((pres(phs, r), m / r))
    return res


def cell_mass(st, b, p):
    o, N, h, f = b.off[p], b.N[p], b.h[p], st.face[p]
    L = np.full(N, h)
    if f >= 0:
        L[f - 1] = h + st.dl[p]
        L[f] = h - st.dr[p]
    m = float(np.sum(L * st.rho[o:o + N]))
    if f >= 0:
        m += (st.dr[p] - st.dl[p]) * st.rho[o + N]
    return m


def test_cavitation_test_reproduces_printed_rows():
    """Cavitation test (Sec. 4): liquid 60000 Pa at -/+4 m/s, h = 1e-2 m,
    C_CFL = 0.5, t_end = 5e-4 s.  The star cells at t_end carry the printed
    rows (pressure table: implicit 68483.740426 / 68477.181783 /
    68483.740588 Pa, exact 68483.741137 / 68477.181783; velocity table
    -4.005940 / ~1e-10 / 4.0059 m/s) within 1e-3 Pa (the liquid law's
    constants are recovered, not printed: the exact solution moves by
    2.6e-4 Pa), and the vapour cell has grown to (w_r - w_l) t_end =
    4.007635e-3 m."""
    b = CW.cavitation_tube()
    st = run(b)
    assert st.status[0] == 0 and st.t[0] == 5e-4 and st.face[0] == 200
    (pl, ul), (pv, uv), (pr, ur) = star_cells(st, b)
    for p, printed in ((pl, 68483.740426), (pv, 68477.181783), (pr, 68483.740588)):
        assert abs(p - printed) < 1e-3, (p, printed)
    assert abs(ul + 4.005940) < 5e-7 and abs(ur - 4.005940) < 5e-7
    assert abs(uv) < 1e-9
    assert abs((st.dr[0] - st.dl[0]) / 4.007635e-3 - 1.0) < 5e-6
    # the printed cost table counts 355 local iterations in 166 steps
    assert 200 < st.iters[0] < 500 and 140 <= st.steps[0] <= 170


def test_nucleation_test_reproduces_printed_implicit_row():
    """Nucleation test (Sec. 4): vapour 70000 Pa at +/-2.7 m/s.  The computed
    star cells sit where the printed implicit row does (70382.992468 /
    70383.072633 / 70382.992468 Pa, 0.465933 / ~1e-10 / -0.465933 m/s),
    about 0.03 Pa below the exact solution (70383.024449 / 70383.115685):
    the scheme's own error, reproduced to 5e-4 Pa in the vapour cells.  The
    created liquid cell's pressure is fixed only to within the dual time
    stop rule: with a_L^2 = 2.2e6 m^2/s^2 a density change of 5e-12
    (relative), far inside the stop tolerance, is 0.01 Pa, and changing the
    initial speeds by 1 to 7 ulp moves it between -0.01 and +0.03 Pa of the
    printed value; it is pinned to that band (0.035 Pa, still short of the
    exact value 0.043 Pa above).  The liquid cell is 2.03e-7 m at t_end."""
    b = CW.nucleation_tube()
    st = run(b)
    assert st.status[0] == 0 and st.t[0] == 5e-4 and st.face[0] == 200
    (pl, ul), (pv, uv), (pr, ur) = star_cells(st, b)
    assert abs(pl - 70382.992468) < 1e-3 and abs(pr - 70382.992468) < 1e-3
    assert abs(pv - 70383.072633) < 0.035
    assert abs(pl - 70383.024449) > 0.02  # not the exact solution
    assert abs(ul - 0.465933) < 1e-6 and abs(ur + 0.465933) < 1e-6
    assert abs(uv) < 1e-9
    assert abs((st.dr[0] - st.dl[0]) / 2.03e-7 - 1.0) < 3e-3
    # the printed cost table: 1'367'460 local iterations in 143 steps
    assert 1e6 < st.iters[0] < 5e6 and 140 <= st.steps[0] <= 150


def test_first_step_creates_the_printed_vapour_cell():
    """After the creation step the vapour cell is (w_r - w_l) dt with the
    CFL step of the initial data: 2.701184e-5 m printed."""
    b = CW.cavitation_tube()
    st = run(b, 1)
    assert st.face[0] == 200 and st.steps[0] == 1 and st.iters[0] == 0
    assert abs((st.dr[0] - st.dl[0]) / 2.701184e-5 - 1.0) < 2e-4
    assert abs(st.dl[0] + st.dr[0]) < 1e-12 * st.dr[0]  # symmetric data: w_l = -w_r
    # the created cell holds the middle star state of the five-state problem
    o = b.off[0]
    p, u = pres(VAP, st.rho[o + 400]), st.mom[o + 400] / st.rho[o + 400]
    assert abs(p - 68477.18) < 0.01 and abs(u) < 1e-9


@pytest.mark.parametrize("case", [CW.CAVITATION, CW.NUCLEATION])
def test_mass_is_conserved_between_walls(case):
    """With walls the mass sum over every cell at its current length (the
    created cell and its neighbours included) is constant to round-off:
    the boundary fluxes of the creation step and of Part 2 are the mass
    the boundaries carry."""
    b = CW.concat([CW.spec(case, 40)], "walls").with_params(bc_left=0, bc_right=0, t_end=6e-5)
    st0 = oracle.CTubeState(b)
    m0 = cell_mass(st0, b, 0)
    st = run(b)
    assert st.status[0] == 0 and st.face[0] == 20 and st.steps[0] > 10
    assert abs(cell_mass(st, b, 0) / m0 - 1.0) < 1e-14


@pytest.mark.parametrize("case", [(LIQ, (66000.0, -5.2), (60000.0, 2.8)),
                                  (VAP, (70100.0, 3.5), (70000.0, -2.0))])
def test_mirror_symmetry(case):
    """Mirrored initial data (states swapped, velocities negated) give the
    mirrored solution: cells reversed, momenta negated, dl <-> -dr."""
    ph, (pl, ul), (pr, ur) = case
    mirrored = (ph, (pr, -ur), (pl, -ul))
    b = CW.concat([CW.spec(case, 40), CW.spec(mirrored, 40)], "mirror").with_params(t_end=1e-4)
    st = run(b)
    assert np.all(st.status == 0) and np.all(st.face == 20) and st.steps[0] == st.steps[1]
    o, N = b.off, 40
    ra, rb = st.rho[o[0]:o[0] + N], st.rho[o[1]:o[1] + N][::-1]
    ma, mb = st.mom[o[0]:o[0] + N], -st.mom[o[1]:o[1] + N][::-1]
    assert np.max(np.abs(ra - rb) / ra) < 1e-12
    assert np.max(np.abs(ma - mb)) < 1e-11 * np.max(np.abs(ma))
    assert abs(st.dl[0] + st.dr[1]) < 1e-12 * abs(st.dr[1])
    # the created cell stops at the dual time tolerance, not at round-off
    assert abs(st.rho[o[0] + N] / st.rho[o[1] + N] - 1.0) < 1e-9
    assert abs(st.iters[0] / st.iters[1] - 1.0) < 0.01


def _hll_scheme(ph, r, m, h, cfl, t_end, n_steps):
    """Brute force: the explicit HLL scheme with transmissive ends, written
    out directly (Davis speeds), for tubes in which nothing is created."""
    a = np.sqrt(M.a2v if ph == VAP else M.a2l)
    t = 0.0
    for _ in range(n_steps):
        S = np.max(np.abs(m / r) + a)
        dt = min(cfl * h / S, t_end - t)
        rl, ml = np.concatenate([[r[0]], r]), np.concatenate([[m[0]], m])
        rr, mr = np.concatenate([r, [r[-1]]]), np.concatenate([m, [m[-1]]])
        ul, ur = ml / rl, mr / rr
        pl, pr = pres(ph, rl), pres(ph, rr)
        sl, sr = np.minimum(ul, ur) - a, np.maximum(ul, ur) + a
        f0l, f1l, f0r, f1r = ml, ml * ul + pl, mr, mr * ur + pr
        F0 = np.where(sl >= 0, f0l, np.where(sr <= 0, f0r,
                      (sr * f0l - sl * f0r + sl * sr * (rr - rl)) / (sr - sl)))
        F1 = np.where(sl >= 0, f1l, np.where(sr <= 0, f1r,
                      (sr * f1l - sl * f1r + sl * sr * (mr - ml)) / (sr - sl)))
        r = r - dt / h * (F0[1:] - F0[:-1])
        m = m - dt / h * (F1[1:] - F1[:-1])
        t += dt
    return r, m


@pytest.mark.parametrize("case", [(LIQ, (60000.0, 3.0), (80000.0, -3.0)),
                                  (VAP, (60000.0, -3.0), (50000.0, 2.0))])
def test_without_creation_the_scheme_is_explicit_hll(case):
    """A liquid compressed or a vapour expanded creates nothing: the tube is
    the plain explicit HLL scheme."""
    b = CW.concat([CW.spec(case, 60)], "plain").with_params(t_end=1e-3)
    st = run(b, 25)
    assert st.status[0] == 0 and st.face[0] == -1 and st.steps[0] == 25
    r, m = _hll_scheme(case[0], b.rho[:60].copy(), b.mom[:60].copy(), b.h[0], 0.5, 1e-3, 25)
    assert np.allclose(st.rho[:60], r, rtol=1e-13, atol=0)
    assert np.allclose(st.mom[:60], m, rtol=1e-11, atol=1e-9)
    assert st.rho[60] == 0.0 and st.iters[0] == 0


def test_status_paths():
    """Two creating faces in one tube (a metastable vapour above p~ on one
    side), a neighbour cell shrunk below h/2 (fast cavitation over a long
    run), and l_max reached (a flag, not a failure)."""
    specs = [dict(N=20, h=1e-2, phase=VAP, left=(71000.0, 3.0), right=(70000.0, -3.0)),
             dict(N=20, h=1e-2, phase=LIQ, left=(60000.0, -40.0), right=(60000.0, 40.0)),
             CW.spec(CW.CAVITATION, 20)]
    b = CW.concat(specs, "status").with_params(t_end=1e-3, lmax=3)
    st, (cnt, fl) = run(b, 60, log=True)
    assert st.status[0] == oracle.CT_ST_MULTI and st.steps[0] == 0
    assert st.status[1] == oracle.CT_ST_MESH and 0 < st.steps[1] < 60
    assert st.status[2] == 0 and st.face[2] == 10
    n2 = st.steps[2]
    assert fl[0, 2] == oracle.CT_FL_CREATED and cnt[0, 2] == 0
    hit = (fl[1:n2, 2] & oracle.CT_FL_LMAX) != 0
    assert hit[0] and np.all(cnt[1:n2, 2][hit] == 3) and np.all(cnt[1:n2, 2] <= 3)
    assert np.all(cnt[1:n2, 2] >= 1)
    assert np.all(fl[n2:, 2] == oracle.CT_FL_INACTIVE)


def test_batch_generator_is_deterministic_and_creates_everywhere():
    b1 = CW.ctube_batch(seed=3, n_problems=64)
    b2 = CW.ctube_batch(seed=3, n_problems=64)
    assert np.array_equal(b1.rho, b2.rho) and np.array_equal(b1.N, b2.N)
    st = run(b1.with_params(lmax=200), 2)
    assert np.all(st.status == 0) and np.all(st.face == b1.N // 2)


@pytest.mark.parametrize("case", [CW.CAVITATION, (LIQ, (66000.0, -5.2), (60000.0, 2.8))])
def test_dual_time_fixed_point_is_the_implicit_step(case):
    """Algorithm 2 run to a tight relative update (1e-15) lands on the
    implicit step of the zone: with the separately pinned interface solver
    and HLL flux evaluated at U^{n+1}, every zone cell satisfies
    h^{n+1} U^{n+1} - h^n U^n + dt (F_{i+1/2} - F_{i-1/2}) = 0 (moving
    lengths, eq. godunov_meth:nonunif; outer zone faces from U^n), and the
    boundaries moved by w(U^{n+1}) dt."""
    b = CW.concat([CW.spec(case, 40)], "fp").with_params(tol_mode=1, tol_rel=1e-15,
                                                         lmax=1_000_000, t_end=1.0)
    s0 = run(b, 3)
    s1 = run(b, 4)
    assert s1.status[0] == 0 and s1.steps[0] == 4 and s1.face[0] == 20
    ph, phn, N, j0, h = case[0], 1 - case[0], 40, 20, b.h[0]
    dt = s1.t[0] - s0.t[0]
    h0 = [h + s0.dl[0], s0.dr[0] - s0.dl[0], h - s0.dr[0]]
    h1 = [h + s1.dl[0], s1.dr[0] - s1.dl[0], h - s1.dr[0]]
    u = lambda s, c: s.mom[c] / s.rho[c]
    L = oracle.iface_solve(M, ph, s1.rho[j0 - 1], u(s1, j0 - 1), phn, s1.rho[N], u(s1, N))
    R = oracle.iface_solve(M, phn, s1.rho[N], u(s1, N), ph, s1.rho[j0], u(s1, j0))
    assert L["ok"] and R["ok"]
    FL = oracle.hll(M, ph, s0.rho[j0 - 2], s0.mom[j0 - 2], s0.rho[j0 - 1], s0.mom[j0 - 1])
    FR = oracle.hll(M, ph, s0.rho[j0], s0.mom[j0], s0.rho[j0 + 1], s0.mom[j0 + 1])
    F = [FL, (L["F0"], L["F1"]), (R["F0"], R["F1"]), FR]
    for k, c in enumerate((j0 - 1, N, j0)):
        for q, (a0, a1) in enumerate(((s0.rho, s1.rho), (s0.mom, s1.mom))):
            res = h1[k] * a1[c] - h0[k] * a0[c] + dt * (F[k + 1][q] - F[k][q])
            scale = max(abs(h1[k] * a1[c]), abs(h0[k] * a0[c]), abs(dt * F[k][q]),
                        abs(dt * F[k + 1][q]))
            assert abs(res) < 1e-11 * scale, (k, q, res / scale)
    assert abs((s1.dl[0] - s0.dl[0]) / (L["w"] * dt) - 1.0) < 1e-12
    assert abs((s1.dr[0] - s0.dr[0]) / (R["w"] * dt) - 1.0) < 1e-12


@pytest.mark.parametrize("case", [CW.CAVITATION, CW.NUCLEATION,
                                  (LIQ, (66000.0, -5.2), (60000.0, 2.8)),
                                  (VAP, (70020.0, 2.9), (69990.0, -2.6))])
def test_newton_zone_solver_lands_on_the_implicit_step(case):
    """The Newton zone solver (the paper's outlook) solves the implicit step
    of the zone to its tolerance: at U^{n+1}, with the separately pinned
    interface solver and HLL flux, every zone cell satisfies
    h^{n+1} U^{n+1} - h^n U^n + dt (F_{i+1/2} - F_{i-1/2}) = 0 and the
    boundaries moved by w(U^{n+1}) dt -- also for nucleated cells, where
    Algorithm 2's update-size rule stops early; a handful of Newton steps
    per time step."""
    b = CW.concat([CW.spec(case, 40)], "nz").with_params(t_end=1.0)
    kw = dict(solver=oracle.CT_SOLVER_NEWTON, zn_rtol=1e-10)
    s0 = oracle.CTubeState(b)
    oracle.ct_run(s0, 3, **kw)
    s1 = oracle.CTubeState(b)
    cnt, fl = oracle.ct_run(s1, 4, log=True, **kw)
    assert s1.status[0] == 0 and s1.steps[0] == 4 and s1.face[0] == 20
    assert np.all(cnt[1:, 0] <= 6) and not np.any(fl & oracle.CT_FL_LMAX)
    ph, phn, N, j0, h = case[0], 1 - case[0], 40, 20, b.h[0]
    dt = s1.t[0] - s0.t[0]
    h0 = [h + s0.dl[0], s0.dr[0] - s0.dl[0], h - s0.dr[0]]
    h1 = [h + s1.dl[0], s1.dr[0] - s1.dl[0], h - s1.dr[0]]
    u = lambda s, c: s.mom[c] / s.rho[c]
    L = oracle.iface_solve(M, ph, s1.rho[j0 - 1], u(s1, j0 - 1), phn, s1.rho[N], u(s1, N))
    R = oracle.iface_solve(M, phn, s1.rho[N], u(s1, N), ph, s1.rho[j0], u(s1, j0))
    FL = oracle.hll(M, ph, s0.rho[j0 - 2], s0.mom[j0 - 2], s0.rho[j0 - 1], s0.mom[j0 - 1])
    FR = oracle.hll(M, ph, s0.rho[j0], s0.mom[j0], s0.rho[j0 + 1], s0.mom[j0 + 1])
    F = [FL, (L["F0"], L["F1"]), (R["F0"], R["F1"]), FR]
    for k, c in enumerate((j0 - 1, N, j0)):
        for q, (a0, a1) in enumerate(((s0.rho, s1.rho), (s0.mom, s1.mom))):
            res = h1[k] * a1[c] - h0[k] * a0[c] + dt * (F[k + 1][q] - F[k][q])
            scale = max(abs(h1[k] * a1[c]), abs(h0[k] * a0[c]), abs(dt * F[k][q]),
                        abs(dt * F[k + 1][q]))
            # the check's interface solves start cold, the scheme's warm: both
            # stop once a full Newton step is below 1e-10 of the pressures,
            # and through a nucleated liquid cell (pressure law slope a_L^2)
            # that shows as up to about 1e-8 of the cell's scale (dense
            # elimination landed at 8e-9, the block solve at 1.3e-8)
            assert abs(res) < 3e-8 * scale, (k, q, res / scale)
    # a nucleated liquid layer is stiff: its boundary speed (about 2e-4 m/s)
    # moves by 1e-4 of itself when its density moves by 1e-13 of itself
    wtol = 1e-7 if ph == LIQ else 1e-3
    assert abs((s1.dl[0] - s0.dl[0]) / (L["w"] * dt) - 1.0) < wtol
    assert abs((s1.dr[0] - s0.dr[0]) / (R["w"] * dt) - 1.0) < wtol


def test_newton_zone_solver_on_the_paper_runs():
    """With the Newton zone solver the Sec. 4 runs reach t_end in the same
    large steps, the star cells within 0.02 Pa of the printed implicit rows
    (the liquid layer's pressure, p0 + a_L^2 (rho - rho0), moves 0.02 Pa per
    1e-8 kg/m^3), with about 3 Newton steps per time step instead of up to
    tens of thousands of dual time iterations."""
    for mk, rows in ((CW.cavitation_tube, (68483.740426, 68477.181783, 68483.740588)),
                     (CW.nucleation_tube, (70382.992468, 70383.072633, 70382.992468))):
        b = mk()
        sd = run(b)
        sn = oracle.CTubeState(b)
        oracle.ct_run(sn, solver=oracle.CT_SOLVER_NEWTON)
        assert sn.status[0] == 0 and sn.t[0] == 5e-4 and sn.steps[0] == sd.steps[0]
        assert sn.iters[0] < 4 * sn.steps[0]
        for (p, _), printed in zip(star_cells(sn, b), rows):
            assert abs(p - printed) < 0.02, (p, printed)
        assert abs((sn.dr[0] - sn.dl[0]) / (sd.dr[0] - sd.dl[0]) - 1.0) < 1e-6


@pytest.mark.parametrize("Z", [2, 3])
def test_newton_zone_solver_on_wider_zones(Z):
    """Zones of the created cell +- 2 and 3 cells (HLL faces inside the
    zone): the Newton zone solver creates on the same face in the same step,
    takes the same steps to t_end as Algorithm 2 (tightened to a relative
    update of 1e-12 so that it converges as far as Newton does) and ends on
    its states to 1e-8; a handful of Newton steps per time step."""
    b = CW.concat([CW.spec(CW.CAVITATION, 40)], f"nz{Z}").with_params(
        zone_half=Z, t_end=1e-4, tol_mode=1, tol_rel=1e-12, lmax=100000)
    sd = run(b)
    sn = oracle.CTubeState(b)
    oracle.ct_run(sn, solver=oracle.CT_SOLVER_NEWTON)
    assert sd.status[0] == 0 and sn.status[0] == 0
    assert sn.face[0] == sd.face[0] == 20 and sn.steps[0] == sd.steps[0]
    assert sn.iters[0] <= 6 * sn.steps[0] < sd.iters[0]
    zone = np.r_[20 - Z:20 + Z, 40]  # the zone's regular cells and the created one
    for x, y in ((sn.rho, sd.rho), (sn.mom, sd.mom)):
        assert np.max(np.abs(x[zone] - y[zone]) / np.maximum(np.abs(y[zone]), 1.0)) < 1e-8
    assert abs(sn.dr[0] - sd.dr[0]) < 1e-8 * abs(sd.dr[0] - sd.dl[0]) + 1e-15


@pytest.mark.parametrize("ph,p", [(LIQ, 60000.0), (VAP, 50000.0)])
def test_constant_state_is_preserved(ph, p):
    """A tube at rest in one uniform state creates nothing and stays exactly
    uniform (HLL fluxes of equal states cancel, walls reflect rest)."""
    b = CW.concat([dict(N=30, h=1e-2, phase=ph, left=(p, 0.0), right=(p, 0.0))],
                  "rest").with_params(bc_left=0, bc_right=0, t_end=1e-4)
    st = run(b)
    assert st.status[0] == 0 and st.face[0] == -1 and st.t[0] == 1e-4
    assert np.all(st.rho[:30] == b.rho[:30]) and np.all(st.mom[:30] == 0.0)
