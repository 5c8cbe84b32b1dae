#!/usr/bin/env python3
"""Benchmark of the batched IMEX-DS step on one MI355X.

One step = one physical time step of every problem in the batch: explicit
HLL sweep of all bulk cells, dual time stepping on every implicit zone with
its interface Riemann solves, CFL reduction and bookkeeping.  Inputs are
seeded synthetic problems resident in HBM before timing starts.

Prints one JSON line with the FP64 cell-update rate of the batched launch
(HIP-graph replays), the per-problem launch form on the same state for
comparison, the HBM roofline fraction of the step as bounded by the zone
kernel (the step's 32 B per cell update over the zone kernel's own launch
duration, HIP events around each zone launch), the bulk kernel's roofline
(HIP events around each bulk launch), and the CPU oracle timed on a bounded
sample of the same problems (whose results are also compared with the
GPU's).
"""
import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 cell-updates/s (batched vs per-problem) at 1e-10 rel L1; adjoint/fwd time"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_CELL_UPDATE = 32  # rho, rho u read + write, FP64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batch", choices=["batch", "large", "bubble"])
    ap.add_argument("--problems", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the cpu_baseline leg")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--per-problem-steps", type=int, default=4)
    ap.add_argument("--roofline-steps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--newton-cpu-seconds", type=float, default=8.0,
                    help="oracle time for the Newton zone solver's CPU baseline (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration)")
    ap.add_argument("--adjoint-steps", type=int, default=500,
                    help="steps of the adjoint leg (0: skip it)")
    ap.add_argument("--adjoint-every", type=int, default=50)
    ap.add_argument("--adjoint-problems", type=int, default=1024)
    ap.add_argument("--adjoint-zone-lanes", type=int, default=8, choices=[1, 8])
    ap.add_argument("--copy-bw", type=int, default=1,
                    help="measure a plain 1 GiB device copy as the practical HBM ceiling")
    ap.add_argument("--creation-problems", type=int, default=1 << 20,
                    help="single-phase Riemann problems in the phase-creation leg (0: skip)")
    ap.add_argument("--only-creation", action="store_true",
                    help="run only the phase-creation leg (for profiling it)")
    ap.add_argument("--only-euler", action="store_true",
                    help="run only the full-Euler leg (for profiling it)")
    ap.add_argument("--per-problem-steps-euler", type=int, default=3)
    ap.add_argument("--euler-problems", type=int, default=4096,
                    help="tubes in the full-Euler Lax ensemble leg (0: skip)")
    ap.add_argument("--ctube-problems", type=int, default=4096,
                    help="creation tubes (cavitation / nucleation inside the mesh) leg (0: skip)")
    ap.add_argument("--only-ctube", action="store_true",
                    help="run only the creation-tube leg (for profiling it)")
    ap.add_argument("--ctube-steps", type=int, default=10,
                    help="creation-tube leg: steps timed (the creation step and the heaviest "
                         "dual time steps; 0: run to t_end, about 100 s)")
    ap.add_argument("--newton-steps", type=int, default=1000,
                    help="steps of the main workload with the Newton zone solver (0: skip)")
    ap.add_argument("--per-problem-steps-ctube", type=int, default=3,
                    help="steps of the creation tubes' Newton run launched tube by tube")
    ap.add_argument("--other-configs", type=int, default=1,
                    help="also time the other workloads (single cut, 2^20 cells, bubbles)")
    ap.add_argument("--adjoint-one-segment", type=int, default=1,
                    help="also time the adjoint with a single segment (no recompute)")
    return ap.parse_args()


def measured_traffic(workload, tile_cells):
    """HBM bytes per k_bulk launch from the committed rocprofv3 PMC summary,
    if it was taken on this workload and launch shape and the kernel source
    is unchanged since; else None."""
    path = os.path.join(ROOT, "profiles", "k_bulk_random_batch_4096_hbm_traffic.txt")
    if workload != "batch" or tile_cells != 1024 or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        kv[k.strip()] = v.strip()
    src = open(os.path.join(ROOT, "paper_2211_00705_amd", "csrc", "imexds_kernels.hip")).read()
    i = src.index("template <int R>\n__global__ __launch_bounds__(256) void k_bulk")
    j = src.index("// CFL over all slots of the current state")
    if hashlib.sha256(src[i:j].encode()).hexdigest() != kv.get("kernel_source_sha256"):
        return None
    return int(kv["traffic_bytes_per_launch"])


def make_workload(args):
    from paper_2211_00705_amd import workloads as W
    if args.workload == "batch":
        b = W.random_batch(n_problems=args.problems)
        P = W.random_batch_params()
        desc = (f"random_batch: {b.n_problems} independent liquid|vapour problems, "
                f"N ~ logU-int[256,16384] ({b.n_slots} slots), 1 interface each, "
                "cut fraction ~ logU[1e-6,1e-1], zone = tiny +- 2, paper stop rule, lmax 100, walls")
    elif args.workload == "bubble":
        b = W.bubble_batch(n_problems=min(args.problems, 1024))
        P = W.bubble_batch_params()
        desc = (f"bubble_batch: {b.n_problems} liquid|vapour-bubble|liquid problems x 4096 cells, "
                "2 interfaces each, vapour-side cut fraction ~ logU[1e-6,1e-2]")
    else:
        b = W.large_smooth_problem()
        P = W.large_smooth_params()
        desc = f"large_smooth: one problem of {b.n_slots} slots, piecewise-smooth states"
    return b, P, desc


def slot_lengths(b, home, hl):
    out = np.empty(b.n_slots)
    so = b.slot_off
    for p in range(b.n_problems):
        hp = b.h[p]
        L = np.full(int(so[p + 1] - so[p]), hp)
        for kk, k in enumerate(range(int(b.iface_off[p]), int(b.iface_off[p + 1]))):
            L[home[k] + kk] = hl[k]
            L[home[k] + kk + 1] = hp - hl[k]
        out[so[p]:so[p + 1]] = L
    return out


def host_info():
    """The host the oracle baseline runs on: logical CPUs, the ones this
    process may use, and the CPU model (lscpu / /proc/cpuinfo)."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    try:
        usable = len(os.sched_getaffinity(0))
    except Exception:
        usable = None
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline_leg(b, P, material, steps, gpu_rho, gpu_mom, gpu_home, gpu_hl, seconds):
    """Times the CPU oracle on chunks of the same problems for the same number
    of steps until about `seconds` of wall time, and compares its results with
    the GPU's for those problems (rel-L1 per problem and component)."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    rng = np.random.default_rng(12345)
    order = rng.permutation(b.n_problems)
    done, cu, wall, worst = [], 0, 0.0, 0.0
    so, io = b.slot_off, b.iface_off
    chunk = 32
    for c0 in range(0, b.n_problems, chunk):
        idx = sorted(order[c0:c0 + chunk].tolist())
        sub = b.subset(idx)
        st = oracle.State(sub)
        t0 = time.perf_counter()
        oracle.run(st, material, P, steps, threads=threads)
        wall += time.perf_counter() - t0
        cu += int(np.sum(st.steps * (np.diff(sub.slot_off))))
        L = slot_lengths(sub, st.home, st.hl)
        sso = sub.slot_off
        for j, p in enumerate(idx):
            g0, g1 = int(so[p]), int(so[p + 1])
            s0, s1 = int(sso[j]), int(sso[j + 1])
            for gk, ok in ((gpu_rho, st.rho), (gpu_mom, st.mom)):
                num = np.sum(np.abs(gk[g0:g1] - ok[s0:s1]) * L[s0:s1])
                den = max(np.sum(np.abs(ok[s0:s1]) * L[s0:s1]),
                          np.sum(np.abs(st.rho[s0:s1]) * L[s0:s1]))
                worst = max(worst, num / den)
            ks = range(int(io[p]), int(io[p + 1]))
            if list(gpu_home[list(ks)]) != list(st.home[int(sub.iface_off[j]):int(sub.iface_off[j + 1])]):
                worst = max(worst, 1.0)
        done += idx
        if wall >= seconds:
            break
    return {"value": cu / wall, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(done)} of {b.n_problems} problems ({int(np.sum(np.diff(b.slot_off)[done]))} slots) "
                      f"x {steps} steps, OpenMP over problems, {wall:.1f} s",
            "host": host_info(),
            "parity_max_rel_l1": worst}


def adjoint_leg(args, material):
    """Adjoint workload: plain forward of n steps (HIP graphs) vs the
    checkpointed forward and the reverse sweep, all timed with HIP events on
    the library's stream; gradient of the window objective."""
    import torch
    from paper_2211_00705_amd import workloads as W
    from paper_2211_00705_amd.imexds import IMEXDS
    from paper_2211_00705_amd.autograd import window_objective
    b = W.adjoint_batch(n_problems=args.adjoint_problems)
    P = W.adjoint_batch_params()
    n, C = args.adjoint_steps, args.adjoint_every
    s = IMEXDS(b, material, P)
    try:
        s.set_launch(1024, 64, 0, 10, args.adjoint_zone_lanes)
        s.set_state()
        s.step(2)
        torch.cuda.synchronize()
        s.set_state()
        s.step(n)
        torch.cuda.synchronize()
        fwd_ms, _ = s.last_timing()
        s.set_state()
        s.forward_ckpt(n, C)
        torch.cuda.synchronize()
        ck_ms, _ = s.last_timing()
        rho, mom = s.state()
        home, hl, _ = s.interfaces()
        hl_t = torch.tensor(hl, dtype=torch.float64, device="cuda", requires_grad=True)
        rho_t = rho.clone().requires_grad_(True)
        window_objective(b, home, hl_t, rho_t).sum().backward()
        g = (rho_t.grad.contiguous(), torch.zeros_like(rho), hl_t.grad.contiguous())
        t0 = time.perf_counter()
        s.adjoint(*g)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        adj_ms, _ = s.last_timing()
        # one segment (checkpoint interval = n): the forward records the tape
        # of all n steps (HBM permitting) and the reverse sweep re-runs nothing
        one = None
        if args.adjoint_one_segment:
            s.set_state()
            s.forward_ckpt(n, n)
            torch.cuda.synchronize()
            ck1_ms, _ = s.last_timing()
            s.adjoint(*g)
            torch.cuda.synchronize()
            adj1_ms, _ = s.last_timing()
            one = {"forward_ckpt_ms": ck1_ms, "adjoint_ms": adj1_ms,
                   "adjoint_over_forward": adj1_ms / fwd_ms,
                   "total_over_forward": (ck1_ms + adj1_ms) / fwd_ms}
    finally:
        s.close()
    return {"workload": f"adjoint_batch: {b.n_problems} problems, N ~ logU-int[256,16384] "
                        f"({b.n_slots} slots), piecewise-smooth states, 1 interface each, "
                        f"{n} steps, checkpoint every {C}",
            "objective": "sum of interface positions + mass in [0.4, 0.6]",
            "forward_ms": fwd_ms, "forward_ckpt_ms": ck_ms, "adjoint_ms": adj_ms,
            "adjoint_wall_ms": wall * 1e3,
            "adjoint_over_forward": adj_ms / fwd_ms,
            "total_over_forward": (ck_ms + adj_ms) / fwd_ms,
            "one_segment": one}


def other_configs_leg(material, cpu):
    """The other configured workloads at their full size, fewer steps: GPU
    batched (graph replay) and per-problem launches, and (cpu) the oracle on
    one host thread and on all of them, on bounded samples."""
    import torch
    from paper_2211_00705_amd import workloads as W
    from paper_2211_00705_amd.imexds import IMEXDS
    out = {}
    cases = [
        ("single_cut: 1 problem, 200 cells, cut 1e-4 h, relative-update DTS to 1e-12",
         W.single_cut_problem(seed=0), W.single_cut_params().replace(t_end=math.inf), 2000, 0, 2000),
        ("large_smooth: 1 problem, 2^20 cells, paper stop rule, lmax 100",
         W.large_smooth_problem(), W.large_smooth_params(), 200, 0, 10),
        ("bubble_batch: 1024 problems x 4096 cells, 2 interfaces each",
         W.bubble_batch(), W.bubble_batch_params(), 200, 4, 200),
    ]
    for desc, b, P, n, npp, ncpu in cases:
        s = IMEXDS(b, material, P)
        try:
            s.set_launch(1024, 8, 0, 10, 8)
            s.set_state()
            s.step(4)
            torch.cuda.synchronize()
            s.set_state()
            st0 = s.stats()
            s.step(n)
            torch.cuda.synchronize()
            ms, _ = s.last_timing()
            cu = s.stats()["cell_updates"] - st0["cell_updates"]
            rec = {"steps": n, "ms_per_step": ms / n, "value": cu / (ms * 1e-3),
                   "hbm_roofline_frac": cu / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9 / BYTES_PER_CELL_UPDATE)}
            if npp:
                s.set_state()
                st0 = s.stats()
                s.step_per_problem(npp)
                torch.cuda.synchronize()
                pms, _ = s.last_timing()
                pcu = s.stats()["cell_updates"] - st0["cell_updates"]
                rec["per_problem"] = {"steps": npp, "value": pcu / (pms * 1e-3),
                                      "batched_speedup": rec["value"] / (pcu / (pms * 1e-3))}
        finally:
            s.close()
        if cpu:
            import oracle
            sub = b if b.n_problems <= 8 else b.subset(list(range(0, b.n_problems, b.n_problems // 8)))
            for threads in (1, max(1, min(16, os.cpu_count() or 1))):
                stc = oracle.State(sub)
                t0 = time.perf_counter()
                oracle.run(stc, material, P, ncpu, threads=threads)
                wall = time.perf_counter() - t0
                key = "cpu_1_thread" if threads == 1 else "cpu_all_threads"
                rec[key] = {"value": float(np.sum(stc.steps * np.diff(sub.slot_off))) / wall,
                            "threads": threads, "sample": f"{sub.n_problems} problems x {ncpu} steps"}
        out[desc] = rec
    return out


# FP64 lane operations executed per unit of work (rocprofv3 SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64,
# FMA counted twice, x 64 lanes, so lanes idled by divergence count too), per run of the
# profiled workloads divided by the units of that run (profiles/ and DESIGN)
EU_ZONE_FLOP_PER_TUBE_ITER = 8989.0  # k_eu_zone: per tube and dual time iteration
EU_BULK_FLOP_PER_FACE = 1343.0       # k_eu_bulk: per face of a tube still running
CR_FLOP_PER_PROBLEM = 2460.0         # k_cr_detect + k_cr_solve per problem of creation_batch
# k_ct_zone: FP64 operations of the busy lanes per tube and dual time
# iteration, from the rocprofv3 PMC counts of the leg's 10 steps of
# ctube_batch: 47456 executed lane operations (64 per wave instruction), of
# which the 8 lanes a wave keeps busy (2 tubes of 4 lanes) do 8/64
CT_ZONE_FLOP_PER_TUBE_ITER = 47456.0 * 8.0 / 64.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def euler_leg(args, cpu):
    """Full-Euler Lax-tube ensemble (Sec. 4 first test, batched): 4096 tubes
    run to t_end = 1 on the GPU with per-launch HIP events, and (cpu) the
    oracle on a bounded sample of the same tubes on 1 and on all threads."""
    import torch
    from paper_2211_00705_amd import euler_workloads as EW
    from paper_2211_00705_amd.euler import EulerIMEXDS
    b = EW.lax_batch(n_problems=args.euler_problems)
    cells = (b.N.astype(np.int64) + 1)
    s = EulerIMEXDS(b)
    try:
        best = None
        for tile, lanes, ppw in ((1024, 2, 32), (256, 2, 32), (1024, 2, 16)):
            s.set_launch(tile, lanes, ppw)
            s.set_state()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = s.run(1 << 20, 64)
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            if best is None or w < best[0]:
                best = (w, tile, lanes, ppw)
        _, tile, lanes, ppw = best
        s.set_launch(tile, lanes, ppw)
        s.set_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = s.run(1 << 20, 64)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t, st, steps, iters = s.problems()
        cu = float(np.sum(cells * steps))
        # the unbatched form on the first steps: every problem's kernels in turn
        s.set_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step_per_problem(args.per_problem_steps_euler)
        torch.cuda.synchronize()
        pp_wall = time.perf_counter() - t0
        _, _, steps_pp, _ = s.problems()
        pp_value = float(np.sum(cells * steps_pp)) / pp_wall
        s.set_state()
        s.time_kernels(True)
        n_timed = s.run(1 << 20, 64)
        bulk_ms, zone_ms, step_ms = s.last_timing()
        s.time_kernels(False)
        _, _, steps_t, iters_t = s.problems()
    finally:
        s.close()
    # dominant kernel: the dual time kernel, one dependent chain per tube
    tube_iters_per_launch = float(np.sum(iters_t)) / max(1, n_timed)
    zone_tflops = EU_ZONE_FLOP_PER_TUBE_ITER * tube_iters_per_launch / (zone_ms * 1e-3) / 1e12
    faces_per_launch = float(np.sum((cells + 1) * steps_t)) / max(1, n_timed)
    bulk_tflops = EU_BULK_FLOP_PER_FACE * faces_per_launch / (bulk_ms * 1e-3) / 1e12
    rec = {"workload": f"lax_batch: {b.n_problems} Lax-type tubes, N in {{100,200,400}} "
                       f"({b.n_cells} cells), alpha logU[1e-6,1e-2], theta_nb in {{0.9,0.1}}, "
                       "states scaled by up to 25%, run to t_end = 1",
           "unit": "cell-updates/s", "value": cu / wall, "wall_s": wall, "launch_steps": n,
           "launch": {"tile_cells": tile, "zone_lanes": lanes, "zone_problems_per_wave": ppw,
                      "check_every": 64},
           "failed_problems": int(np.sum(st != 0)),
           "mean_dual_time_iterations": float(np.sum(iters) / max(1, np.sum(steps))),
           "bulk_ms_per_launch": bulk_ms, "zone_ms_per_launch": zone_ms,
           "step_ms": step_ms,
           "per_problem": {"value": pp_value, "unit": "cell-updates/s",
                           "steps": args.per_problem_steps_euler,
                           "batched_speedup": (cu / wall) / pp_value},
           "roofline": {"bound": "alu", "kernel": "k_eu_zone", "achieved": zone_tflops,
                        "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": zone_tflops / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                        "per_unit": f"{EU_ZONE_FLOP_PER_TUBE_ITER:.0f} FP64 ops per tube and "
                                    "dual time iteration",
                        "units_per_launch": tube_iters_per_launch,
                        "note": "one dependent FP64 chain per tube: latency, not the ALU "
                                "peak, bounds it"},
           "bulk_roofline": {"bound": "alu", "kernel": "k_eu_bulk", "achieved": bulk_tflops,
                             "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": bulk_tflops / FP64_VECTOR_PEAK_TFLOPS,
                             "per_unit": f"{EU_BULK_FLOP_PER_FACE:.0f} FP64 ops per face"}}
    if cpu:
        import oracle
        sub = b.subset(list(range(0, b.n_problems, max(1, b.n_problems // 64))))
        for threads in (1, max(1, min(16, os.cpu_count() or 1))):
            stc = oracle.EulerState(sub)
            t0 = time.perf_counter()
            oracle.euler_run(stc, threads=threads)
            w = time.perf_counter() - t0
            key = "cpu_1_thread" if threads == 1 else "cpu_all_threads"
            rec[key] = {"value": float(np.sum((sub.N + 1) * stc.steps)) / w, "threads": threads,
                        "kind": "oracle", "sample": f"{sub.n_problems} of the tubes to t_end"}
    return rec


def creation_leg(args, cpu):
    """Batched phase creation (cavitation / nucleation detection and the
    five-state solve) on 2^20 single-phase Riemann problems, timed with HIP
    events on the launching stream; the oracle on a sample on the host."""
    import torch
    from paper_2211_00705_amd import workloads as W
    from paper_2211_00705_amd.creation import imexds_creation_rp
    M = W.WATER_363K
    b = W.creation_batch(M, n=args.creation_problems)
    dev = lambda a, t=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
    args_d = (dev(b.phase, torch.int32), dev(b.rho_l), dev(b.mom_l), dev(b.rho_r), dev(b.mom_r))
    st, out = imexds_creation_rp(M, *args_d, W.P_MIN, W.P_TILDE)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        imexds_creation_rp(M, *args_d, W.P_MIN, W.P_TILDE, status=st, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    s = st.cpu().numpy()
    rec = {"workload": f"creation_batch: {b.n} single-phase Riemann problems (half liquid "
                       "pulled apart or compressed, half vapour compressed or expanded)",
           "unit": "problems/s", "value": b.n / (ms * 1e-3), "ms_per_launch": ms,
           "created": int(np.sum(s == 1)), "failed": int(np.sum(s < 0))}
    tf = CR_FLOP_PER_PROBLEM * b.n / (ms * 1e-3) / 1e12
    rec["roofline"] = {"bound": "alu", "kernel": "k_cr_detect + k_cr_solve (one call)",
                       "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                       "per_unit": f"{CR_FLOP_PER_PROBLEM:.0f} FP64 ops per problem"}
    if cpu:
        import oracle
        k = min(b.n, 1 << 18)
        for threads in (1, max(1, min(16, os.cpu_count() or 1))):
            t0 = time.perf_counter()
            oracle.creation_batch(M, b.phase[:k], b.rho_l[:k], b.mom_l[:k], b.rho_r[:k],
                                  b.mom_r[:k], W.P_MIN, W.P_TILDE, threads=threads)
            w = time.perf_counter() - t0
            key = "cpu_1_thread" if threads == 1 else "cpu_all_threads"
            rec[key] = {"value": k / w, "threads": threads, "kind": "oracle",
                        "sample": f"first {k} problems"}
    return rec


def ctube_leg(args, cpu):
    """Creation tubes (Sec. 4 cavitation and nucleation runs, batched): 4096
    tubes, half cavitating liquid, half nucleating vapour, from the creation
    step to t_end = 5e-4 s with the paper's stop rule; HIP events around every
    launch; the oracle on a bounded sample of the same tubes."""
    import torch
    from paper_2211_00705_amd import ctube_workloads as CW
    from paper_2211_00705_amd.ctube import CreationTubes
    b = CW.ctube_batch(n_problems=args.ctube_problems)
    slots = b.N.astype(np.int64) + 1
    lanes, ppw = 4, 2
    s = CreationTubes(b)
    try:
        s.set_launch(lanes, ppw)
        s.set_state()
        s.time_kernels(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if args.ctube_steps > 0:
            s.step(args.ctube_steps)
            n = args.ctube_steps
        else:
            n = s.run(1 << 20, 64)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        bulk_ms, zone_ms, step_ms = s.last_timing()
        s.time_kernels(False)
        t, st, steps, iters, face, _, _ = s.problems()
    finally:
        s.close()
    cu = float(np.sum(slots * steps))
    tube_iters = float(np.sum(iters))
    rec = {"workload": f"ctube_batch: {b.n_problems} creation tubes (half liquid pulled apart "
                       "at 1-6 m/s, cavitating; half vapour compressed at 2.6-3 m/s, "
                       f"nucleating), N in {{200,400,800}}, h = 1e-2 m ({b.n_slots} slots), "
                       "C_CFL 0.5, zone +-1, paper stop rule, l_max 1e5, "
                       + (f"first {args.ctube_steps} steps (creation step and the heaviest "
                          "dual time steps)" if args.ctube_steps > 0 else "to t_end = 5e-4 s"),
           "unit": "cell-updates/s", "value": cu / wall, "wall_s": wall, "launch_steps": n,
           "launch": {"zone_lanes": lanes, "zone_problems_per_wave": ppw, "check_every": 64},
           "failed_problems": int(np.sum(st != 0)),
           "created": int(np.sum(face >= 0)),
           "tube_steps_per_s": float(np.sum(steps)) / wall,
           "tubes_to_t_end_per_s": float(b.n_problems) / wall if args.ctube_steps == 0 else None,
           "dual_time_iterations": tube_iters,
           "dual_time_iterations_per_s": tube_iters / wall,
           "max_iterations_per_tube": int(np.max(iters)) if len(iters) else 0,
           "bulk_ms_per_launch": bulk_ms, "zone_ms_per_launch": zone_ms, "step_ms": step_ms}
    if CT_ZONE_FLOP_PER_TUBE_ITER:
        tf = CT_ZONE_FLOP_PER_TUBE_ITER * (tube_iters / max(1, n)) / (zone_ms * 1e-3) / 1e12
        rec["roofline"] = {"bound": "alu", "kernel": "k_ct_zone", "achieved": tf,
                           "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                           "per_unit": f"{CT_ZONE_FLOP_PER_TUBE_ITER:.0f} FP64 ops per tube and "
                                       "dual time iteration",
                           "units_per_launch": tube_iters / max(1, n),
                           "note": "operations of the busy lanes only (8 of a wave's 64); "
                                   "the nucleating tubes' dependent chains (tens of thousands "
                                   "of dual time iterations per step) bound it: latency"}
    # the Newton zone solver (zone +- 1) on the whole run to t_end
    s = CreationTubes(b)
    nlanes, nppw = 2, 4  # the Newton kernel's fastest shape (7 groups of 2 lanes, 4 tubes a wave)
    try:
        s.set_launch(nlanes, nppw)
        s.set_solver(1)
        s.set_state()
        s.time_kernels(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nn = s.run(1 << 20, 64)
        torch.cuda.synchronize()
        nwall = time.perf_counter() - t0
        nb_ms, nz_ms, ns_ms = s.last_timing()
        s.time_kernels(False)
        _, nst, nsteps, niters, nface, _, _ = s.problems()
        # the unbatched form on the first steps: every tube's kernels in turn
        npp = None
        if args.per_problem_steps_ctube > 0:
            s.set_state()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step_per_problem(args.per_problem_steps_ctube)
            torch.cuda.synchronize()
            ppw_s = time.perf_counter() - t0
            _, _, pp_steps, _, _, _, _ = s.problems()
            pp_value = float(np.sum(slots * pp_steps)) / ppw_s
            npp = {"value": pp_value, "unit": "cell-updates/s",
                   "steps": args.per_problem_steps_ctube,
                   "batched_speedup": (float(np.sum(slots * nsteps)) / nwall) / pp_value}
    finally:
        s.close()
    rec["newton_zone_solver"] = {
        "what": "the zone's implicit step by Newton (forward-difference Jacobian, block "
                "tridiagonal solve, tolerance 1e-10) instead of dual time stepping, the whole "
                "run to t_end = 5e-4 s",
        "unit": "cell-updates/s", "value": float(np.sum(slots * nsteps)) / nwall,
        "wall_s": nwall, "launch_steps": nn, "failed_problems": int(np.sum(nst != 0)),
        "launch": {"zone_lanes": nlanes, "zone_problems_per_wave": nppw},
        "tubes_to_t_end_per_s": float(b.n_problems) / nwall,
        "newton_steps": int(np.sum(niters)), "max_newton_steps_per_tube": int(np.max(niters)),
        "per_problem": npp,
        "bulk_ms_per_launch": nb_ms, "zone_ms_per_launch": nz_ms, "step_ms": ns_ms}
    if cpu:
        import oracle
        sub = b.subset(list(range(0, b.n_problems, 16)))
        for threads in (1, max(1, min(16, os.cpu_count() or 1))):
            stc = oracle.CTubeState(sub)
            t0 = time.perf_counter()
            oracle.ct_run(stc, threads=threads, solver=oracle.CT_SOLVER_NEWTON)
            w = time.perf_counter() - t0
            key = "cpu_1_thread" if threads == 1 else "cpu_all_threads"
            rec["newton_zone_solver"][key] = {
                "value": float(np.sum((sub.N + 1) * stc.steps)) / w, "threads": threads,
                "kind": "oracle", "sample": f"every 16th tube ({sub.n_problems}) to t_end",
                "wall_s": w}
    if cpu:
        import oracle
        idx = [0, 1, 2, 3]
        sub = b.subset(idx)
        for threads in (1, 4):
            stc = oracle.CTubeState(sub)
            t0 = time.perf_counter()
            oracle.ct_run(stc, args.ctube_steps if args.ctube_steps > 0 else None,
                          threads=threads)
            w = time.perf_counter() - t0
            key = "cpu_1_thread" if threads == 1 else "cpu_4_threads"
            rec[key] = {"value": float(np.sum((sub.N + 1) * stc.steps)) / w, "threads": threads,
                        "kind": "oracle", "sample": "tubes 0-3 of the ensemble (2 cavitating, "
                                                    "2 nucleating), the same steps",
                        "wall_s": w}
    return rec


def measure_copy_bandwidth(mib=1024, reps=20):
    """Read+write bandwidth of a plain device-to-device copy (torch copy_) of
    `mib` MiB: the practical HBM ceiling the sweep's roofline is read against."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (ms * 1e-3) / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU only: the problems are independent and a multi-GPU "
                                   "run would split the batch by problem, which is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2211_00705_amd import imexds as I
    from paper_2211_00705_amd.workloads import WATER_363K as material

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        xa = torch.ones(n, dtype=torch.float64, device="cuda")
        xb = torch.empty_like(xa)
        xb.copy_(xa)
        torch.cuda.synchronize()
        del xa, xb

    if args.only_euler:
        print(json.dumps({"euler_lax": euler_leg(args, not args.no_cpu)}))
        return
    if args.only_creation:
        print(json.dumps({"phase_creation": creation_leg(args, not args.no_cpu)}))
        return
    if args.only_ctube:
        print(json.dumps({"creation_tubes": ctube_leg(args, not args.no_cpu)}))
        return

    b, P, desc = make_workload(args)
    s = I.IMEXDS(b, material, P)
    rho0 = torch.from_numpy(np.ascontiguousarray(b.rho)).cuda()
    mom0 = torch.from_numpy(np.ascontiguousarray(b.mom)).cuda()
    s.set_state(rho0, mom0)
    tune = {"tile_cells": 1024, "zones_per_group": 64, "zone_groups": 0, "zone_lanes": 8}
    if not args.no_autotune:
        tc, zp, zg, zn, ms = s.autotune(10)
        tune = {"tile_cells": tc, "zones_per_group": zp, "zone_groups": zg, "zone_lanes": zn,
                "ms_per_step": ms}
    graph_steps = 10
    s.set_launch(tune["tile_cells"], tune["zones_per_group"], tune["zone_groups"], graph_steps,
                 tune["zone_lanes"])

    # warm-up on the initial state, then reload it so the timed steps are the first K steps
    s.step(args.warmup)
    torch.cuda.synchronize()
    s.set_state(rho0, mom0)
    torch.cuda.synchronize()
    st0 = s.stats()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms, _ = s.last_timing()
    st1 = s.stats()
    cell_updates = st1["cell_updates"] - st0["cell_updates"]
    ms = ev_ms
    value = cell_updates / (ms * 1e-3)

    g_rho, g_mom = s.state_numpy()
    g_home, g_hl, _ = s.interfaces()
    _, g_status, g_steps = s.problems()

    # kernel rooflines: the same K steps from the initial state again, each
    # bulk launch and each zone launch alone between two HIP events on the
    # main stream (the zones follow the sweep instead of overlapping it)
    NIF = b.n_iface
    zone_slots = int(round(NIF * (2 * P.zone_half + 1)))
    bulk_bytes = BYTES_PER_CELL_UPDATE * (b.n_slots - zone_slots)
    step_bytes = cell_updates / args.steps * BYTES_PER_CELL_UPDATE
    bulk_ms = achieved = zone_ms = zone_achieved = None
    zone_kernel = "k_zone8" if tune["zone_lanes"] == 8 else "k_zone"
    if args.roofline_steps > 0:
        s.set_state(rho0, mom0)
        s.time_bulk(True)
        s.step(args.steps)
        torch.cuda.synchronize()
        _, zone_ms, n_timed = s.kernel_timing()
        s.time_bulk(False)
        zone_achieved = step_bytes / (zone_ms * 1e-3) / 1e9
    # a plain copy moving the same bytes per launch (read + write), the
    # practical ceiling at this transfer size
    copy_mib_same = max(1, int(round(bulk_bytes / 2 / (1 << 20))))
    roof_tile = 1024  # the bulk sweep's own best tile class (the step's may differ)
    if args.roofline_steps > 0:
        s.set_launch(roof_tile, tune["zones_per_group"], tune["zone_groups"], graph_steps,
                     tune["zone_lanes"])
        s.time_bulk(True)
        s.step(args.roofline_steps)
        torch.cuda.synchronize()
        _, bulk_ms = s.last_timing()
        s.time_bulk(False)
        achieved = bulk_bytes / (bulk_ms * 1e-3) / 1e9

    # per-problem launch form on the same state
    pp = None
    if args.per_problem_steps > 0:
        s.step_per_problem(args.per_problem_steps)
        torch.cuda.synchronize()
        pp_ms, _ = s.last_timing()
        pp_value = args.per_problem_steps * b.n_slots / (pp_ms * 1e-3)
        pp = {"value": pp_value, "unit": "cell-updates/s", "ms_per_step": pp_ms / args.per_problem_steps,
              "steps": args.per_problem_steps, "batched_speedup": value / pp_value}
    # the same steps with the zones solved by Newton on their implicit step
    # instead of Algorithm 2 (the paper's outlook): same workload, same
    # launch, from the initial state
    nz = None
    if args.newton_steps > 0:
        # one-lane groups at tile class 1024: the fastest measured shape
        s.set_launch(1024, tune["zones_per_group"], tune["zone_groups"], 10, 1)
        s.set_zone_solver(1)
        s.set_state(rho0, mom0)
        s.step(args.warmup)
        torch.cuda.synchronize()
        s.set_state(rho0, mom0)
        torch.cuda.synchronize()
        n0 = s.stats()
        s.step(args.newton_steps)
        torch.cuda.synchronize()
        nz_ms, _ = s.last_timing()
        n1 = s.stats()
        ncu = n1["cell_updates"] - n0["cell_updates"]
        nval = ncu / (nz_ms * 1e-3)
        _, nz_status, _ = s.problems()
        nz_rho, nz_mom = s.state_numpy()
        nz_home, nz_hl, _ = s.interfaces()
        nz = {"what": "the zones' implicit steps solved by Newton (forward-difference Jacobian, "
                      "block tridiagonal solve, tolerance 1e-10) instead of dual time stepping; same workload, tile class "
                      "1024, one-lane groups (1 + 4 zone_half + 2 per zone)",
              "value": nval, "unit": "cell-updates/s", "steps": args.newton_steps,
              "ms_per_step": nz_ms / args.newton_steps,
              "newton_steps_per_zone_step": (n1["pseudo_iters"] - n0["pseudo_iters"])
              / max(1, NIF * args.newton_steps),
              "failed_problems": int(np.sum(nz_status != 0)),
              "step_roofline_frac": nval / (HBM_PEAK_GBS * 1e9 / BYTES_PER_CELL_UPDATE),
              "over_dual_time": nval / value}
        s.set_zone_solver(0)
        if not args.no_cpu and args.newton_cpu_seconds > 0:
            nz["cpu_baseline"] = cpu_baseline_leg(b, dataclasses.replace(P, zone_solver=1),
                                                  material, args.newton_steps, nz_rho, nz_mom,
                                                  nz_home, nz_hl, args.newton_cpu_seconds)
    s.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded), inputs resident in HBM",
        "config": {"workload": desc, "problems": b.n_problems, "slots": b.n_slots,
                   "interfaces": b.n_iface,
                   "launch": f"hipGraph replay, {graph_steps} steps per graph",
                   "launch_tuning": tune},
        "wall_s": wall,
        "failed_problems": int(np.sum(g_status != 0)),
        "pseudo_iters_per_zone_step": (st1["pseudo_iters"] - st0["pseudo_iters"]) / max(1, NIF * args.steps),
        "interface_solves": {
            "per_zone_step": (st1["iface_solves"] - st0["iface_solves"]) / max(1, NIF * args.steps),
            "evaluations_of_G_per_solve": (st1["newton_iters"] - st0["newton_iters"])
            / max(1, st1["iface_solves"] - st0["iface_solves"]),
            "lmax_hits_per_step": (st1["lmax_hits"] - st0["lmax_hits"]) / max(1, args.steps)},
        "per_problem": pp,
        "roofline": {"bound": "hbm", "kernel": zone_kernel, "achieved": zone_achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (zone_achieved / HBM_PEAK_GBS) if zone_achieved else None,
                     "traffic": None,
                     "zone_ms_per_launch": zone_ms,
                     "zone_launches_timed": args.steps if zone_ms else 0,
                     "algorithmic_bytes_per_launch": step_bytes,
                     "note": "the step's algorithmic bytes (32 B per cell update: rho, rho u "
                             "read and written, every slot) over the duration of the zone "
                             "kernel, the step's longest kernel (launched alone, HIP events on "
                             "its stream, same steps as the headline).  The zone kernel itself "
                             "moves about 0.2 KB per zone: it is bound by its dependent FP64 "
                             "chain (dual time iterations of the slowest zone), not by HBM; "
                             "traffic is not reported for it"},
        "bulk_roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": measured_traffic(args.workload, roof_tile),
                     "tile_cells": roof_tile,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_bulk", "bulk_ms_per_launch": bulk_ms,
                     "bulk_launches_timed": args.roofline_steps,
                     "algorithmic_bytes_per_launch": bulk_bytes,
                     "copy_GBs_measured": None, "frac_of_copy": None,
                     "copy_same_bytes_GBs": None, "frac_of_same_bytes_copy": None},
        "step_roofline_frac": value / (HBM_PEAK_GBS * 1e9 / BYTES_PER_CELL_UPDATE),
        "newton_zone_solver": nz,
    }
    if args.adjoint_steps > 0:
        adj = adjoint_leg(args, material)
        out["adjoint"] = adj
        out["adjoint_over_forward"] = adj["adjoint_over_forward"]
    if args.other_configs:
        out["other_configs"] = other_configs_leg(material, not args.no_cpu)
    if args.euler_problems > 0:
        out["euler_lax"] = euler_leg(args, not args.no_cpu)
    if args.creation_problems > 0:
        out["phase_creation"] = creation_leg(args, not args.no_cpu)
    if args.ctube_problems > 0:
        out["creation_tubes"] = ctube_leg(args, not args.no_cpu)
    if args.copy_bw:
        # the plain-copy ceilings, after every GPU leg: measured before them,
        # these copies made the adjoint leg's two-stream overlap slower
        br = out["bulk_roofline"]
        copy_gbs = measure_copy_bandwidth()
        copy_same_gbs = measure_copy_bandwidth(mib=copy_mib_same)
        br["copy_GBs_measured"] = copy_gbs
        br["frac_of_copy"] = (achieved / copy_gbs) if (achieved and copy_gbs) else None
        br["copy_same_bytes_GBs"] = copy_same_gbs
        br["frac_of_same_bytes_copy"] = (achieved / copy_same_gbs) if (achieved and copy_same_gbs) else None
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_leg(b, P, material, args.steps, g_rho, g_mom, g_home,
                                               g_hl, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
