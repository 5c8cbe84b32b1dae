"""Helpers for GPU-vs-oracle parity tests: run the same seeded batch through
the HIP path (via the C ABI binding) and through the CPU oracle, and compare
them element by element."""
import numpy as np

import oracle

# relative L1 tolerance per problem and component (FP64 throughout)
RTOL_L1 = 1e-10


def slot_lengths(b, home, hl):
    out = np.empty(b.n_slots)
    so = b.slot_off
    for p in range(b.n_problems):
        hp = b.h[p]
        L = np.full(int(so[p + 1] - so[p]), hp)
        for kk, k in enumerate(range(int(b.iface_off[p]), int(b.iface_off[p + 1]))):
            sL = home[k] + kk
            L[sL] = hl[k]
            L[sL + 1] = hp - hl[k]
        out[so[p]:so[p + 1]] = L
    return out


def run_oracle(batch, material, params, n_steps, threads=8):
    st = oracle.State(batch)
    lc, lf, lz = oracle.run(st, material, params, n_steps, log=True, threads=threads)
    return dict(rho=st.rho, mom=st.mom, home=st.home[:batch.n_iface], hl=st.hl[:batch.n_iface],
                t=st.t, status=st.status, steps=st.steps, count=lc, flags=lf, zlo=lz)


def run_gpu(batch, material, params, n_steps, launch=None, per_problem=False, log=True,
            lanes=None):
    """``params.zone_solver`` 1 selects the Newton zone solver; ``launch``:
    full set_launch tuple; ``lanes``: only the lanes per zone (1 or 8) with
    the other launch settings at their defaults."""
    import torch
    from paper_2211_00705_amd.imexds import IMEXDS
    s = IMEXDS(batch, material, params)
    try:
        if launch is not None:
            s.set_launch(*launch)
        elif lanes is not None:
            s.set_launch(zone_lanes=lanes)
        if getattr(params, "zone_solver", 0):
            s.set_zone_solver(params.zone_solver, params.zn_maxit, params.zn_rtol)
        s.set_state()
        if log:
            s.enable_log(n_steps)
        if per_problem:
            s.step_per_problem(n_steps)
        else:
            s.step(n_steps)
        torch.cuda.synchronize()
        rho, mom = s.state_numpy()
        home, hl, _ = s.interfaces()
        t, status, steps = s.problems()
        out = dict(rho=rho, mom=mom, home=home, hl=hl, t=t, status=status, steps=steps,
                   stats=s.stats())
        if log:
            c, f, z = s.log()
            out.update(count=c, flags=f, zlo=z)
        return out
    finally:
        s.close()


def assert_parity(batch, g, o, rtol=RTOL_L1, logs=True):
    """rel-L1 <= rtol per problem and component; identical interface cells,
    statuses, step counts and (if logged) dual-time counts, flags and zones."""
    np.testing.assert_array_equal(g["status"], o["status"])
    np.testing.assert_array_equal(g["steps"], o["steps"])
    np.testing.assert_array_equal(g["home"], o["home"])
    if logs and "count" in g and batch.n_iface > 0:
        assert g["count"].shape == o["count"].shape
        bad = np.argwhere((g["count"] != o["count"]) | (g["flags"] != o["flags"])
                          | (g["zlo"] != o["zlo"]))
        assert bad.size == 0, f"log mismatch at (step, iface) {bad[:5].tolist()}: " \
            f"gpu {[(g['count'][tuple(i)], g['flags'][tuple(i)]) for i in bad[:3]]} " \
            f"oracle {[(o['count'][tuple(i)], o['flags'][tuple(i)]) for i in bad[:3]]}"
    so = batch.slot_off
    io = batch.iface_off
    L = slot_lengths(batch, o["home"], o["hl"])
    worst = 0.0
    for p in range(batch.n_problems):
        sl = slice(int(so[p]), int(so[p + 1]))
        for key in ("rho", "mom"):
            num = np.sum(np.abs(g[key][sl] - o[key][sl]) * L[sl])
            den = np.sum(np.abs(o[key][sl]) * L[sl])
            if key == "mom":  # momentum may vanish: measure against mass x 1 m/s too
                den = max(den, np.sum(np.abs(o["rho"][sl]) * L[sl]))
            rel = num / den if den > 0 else num
            worst = max(worst, rel)
            assert rel <= rtol, f"problem {p} {key}: rel-L1 {rel:.3e}"
        hp = batch.h[p]
        for k in range(int(io[p]), int(io[p + 1])):
            assert abs(g["hl"][k] - o["hl"][k]) <= rtol * hp, (p, k, g["hl"][k], o["hl"][k])
    np.testing.assert_allclose(g["t"], o["t"], rtol=1e-13, atol=0)
    return worst


def take_problems(b, v, key, idx):
    """The entries of problems ``idx`` (in order) of a run_gpu output field."""
    so, io = b.slot_off, b.iface_off
    if key in ("rho", "mom"):
        return np.concatenate([v[so[p]:so[p + 1]] for p in idx])
    if key in ("home", "hl"):
        return np.concatenate([v[io[p]:io[p + 1]] for p in idx])
    if key in ("t", "status", "steps"):
        return v[idx]
    return v
