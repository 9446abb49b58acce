"""Benchmark: fine cell-steps per second of FAS-MGRIT V-cycles on one MI355X.

Workload (the largest single-problem configuration, which fits one GPU):
inviscid Burgers, WENO5-JS (eps = 1e-6) + Lax-Friedrichs flux + SSPRK3 at
CFL 0.8, N_x = 65536, N_T = 16384, m = 16, 4-level FCF V-cycle, FP64,
u0 = 0.5 + 16 seeded Fourier modes with wave numbers in 1..64 (synthetic,
seed 210409404 + 2).  Every line is split over 16 workgroups that meet once
per Runge-Kutta stage.

One "step" is one MGRIT iteration: the level-0 F-relaxation that yields the
residual, the C-relaxation and second F-sweep fused with the FAS restriction,
FCF relaxation and restriction on levels 1 and 2, the serial coarsest solve
and the ideal interpolations.  The timed region runs K such iterations
inside one mgrit_cycle call on data resident in HBM (tol < 0, so no early
exit; the coarse CFL of this problem makes MGRIT diverge, so the cycle count
is fixed), i.e. K cycles plus the residual sweep of the final iterate.

value = (cell steps executed by all kernels of the region) / (wall time of
the region), where a cell step is one application of Phi to one cell.  HIP
events on the launch stream bracket the dominant kernel's launches only (the
level-0 F + C sweep); its average duration gives the roofline figure.

Extra fields: the same measurement on the 1024-cell problem, the 512-problem
batch, the adjoint/forward ratio against a serial and an MGRIT forward, MGRIT
wall time to a residual of 1e-10 where MGRIT converges (with GPU serial
stepping beside it), and the scheme-variant and system sweeps.  Beside the
CPU baseline's Phi rate: the oracle's MGRIT on the host (one iteration of
the 1024-cell problem, the 64-cell first-order problem to 1e-10, and one
iteration of the benchmark problem extrapolated from the Phi rate).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WENO5-SSPRK3 fine cell-steps/s in MGRIT relax; adjoint/forward time ratio"
# algorithmic FP64 flops per cell step of WENO5-JS + LF + SSPRK3 (three stages of
# two reconstructions per interface, LF flux, flux difference, RK combination);
# divisions count as one flop
FLOPS_PER_CELL_STEP = 440.0
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12
# first order (k = 0) LF + forward Euler: two flux evaluations, the LF flux
# and the difference, the update; one line read and one written per step when
# every node is stored
K0_FE_FLOPS_PER_CELL_STEP = 10.0
K0_FE_BYTES_PER_CELL_STEP = 8.0
ONE_WG_FC = "relax_fc_kernel<4, 4, 2, 3, false, false>"


def _record(name):
    """The JSON record profiles/<name>, or None when it is missing."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            rec = json.load(f)
        return rec
    except (OSError, ValueError):
        return None


def _fresh(rec):
    """True while the sources a counter record lists still hash to the value
    recorded with it (the counters were taken on this code)."""
    import hashlib

    try:
        h = hashlib.sha256()
        for name in rec["sources"]:
            with open(os.path.join(ROOT, name), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, TypeError):
        return False
    return h.hexdigest() == rec.get("sources_sha256")


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the FETCH_SIZE / WRITE_SIZE counter
    record in profiles/traffic.json (counters scaled by a plain copy of known
    size), or None when the record is missing or the kernel's sources changed
    since the counters were taken."""
    rec = _record("traffic.json")
    if rec is None or kernel not in rec or not _fresh(rec[kernel]):
        return None
    return rec[kernel]["hbm_bytes_per_launch"]


def measured_variant_flops():
    """Executed FP64 flops per cell-step of each scheme variant's level-0
    F-sweep, from the SQ_INSTS_VALU_*_F64 counter record in
    profiles/variant_flops.json (FMA = 2 flops, x 64 lanes), or None when the
    record is missing or the kernel sources changed since it was taken."""
    rec = _record("variant_flops.json")
    return rec["flops_per_cell_step"] if rec is not None and _fresh(rec) else None


def measured_system_flops():
    """Executed FP64 flops per cell-step of the system sweeps from
    profiles/system_flops.json, or None when missing or stale (as for the
    scheme variants)."""
    rec = _record("system_flops.json")
    return rec["flops_per_cell_step"] if rec is not None and _fresh(rec) else None


def variant_rates():
    """Row f3 measured: the level-0 F-sweep of the 1024-cell problem's shape for
    every reconstruction degree with the LF and the Roe flux."""
    from paper_2104_09404_amd import profiling

    rates = profiling.variants(reps=5, quiet=True)
    flops = measured_variant_flops()
    for name, r in rates.items():
        f = flops.get(name) if flops else None
        r["executed_flops_per_cell_step"] = f
        r["tflops"] = f * r["cell_steps_per_s"] / 1e12 if f else None
        r["frac_fp64_peak"] = f * r["cell_steps_per_s"] / PEAK_FP64 if f else None
    return {"workload": "level-0 F-sweep of burgers_weno5_nx1024: 512 chunks x 7 SSPRK3 steps x 1024 cells",
            "kernel": "relax_f_kernel<4, 4, k, 3, false, roe>", "variants": rates}


def system_rates():
    """Row f4 measured: F-sweeps of 512 chunks x 7 SSPRK3 steps on 512-cell
    lines of shallow water and Euler."""
    from paper_2104_09404_amd import profiling

    rates = profiling.systems(reps=5, quiet=True)
    flops = measured_system_flops()
    for name, r in rates.items():
        f = flops.get(name) if flops else None
        r["executed_flops_per_cell_step"] = f
        r["tflops"] = f * r["cell_steps_per_s"] / 1e12 if f else None
        r["frac_fp64_peak"] = f * r["cell_steps_per_s"] / PEAK_FP64 if f else None
    return {"workload": "F-sweep of 512 chunks x 7 SSPRK3 steps on 512-cell lines (shallow water g = 9.81, "
                        "Euler gamma = 5/3), CFL 0.4",
            "kernel": "sys_relax_f_kernel<D, k, 3, roe>", "systems": rates}


def gpu_serial_ms(mgrit, s, pb, u0, reps=3):
    """Serial time stepping of the same problem on the GPU (N_T steps of Phi on
    one line), the comparison point for the MGRIT solve."""
    import torch

    out = torch.empty((pb.nt + 1, mgrit.line_len(s)), dtype=torch.float64, device=u0.device)
    mgrit.serial(s, pb.dt, pb.nt, u0, out)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        mgrit.serial(s, pb.dt, pb.nt, u0, out)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    del out
    return best * 1e3


def time_to_tolerance(mgrit):
    """MGRIT wall time to a residual of 1e-10 where MGRIT converges, from the
    first launch to the converged readback (one untimed solve first), with GPU
    serial stepping of the same problem beside it:
      * the first-order 64-cell problem (2 levels, m = 4);
      * the paper's high-order experiment with WENO5 + LF (64 cells, 400 steps);
      * the paper's fine-matching experiment at its largest grid (1024 cells,
        8192 steps, 5 levels, m = 2, first-order matching), moving shock, V-
        and F-cycle;
      * the 1024-cell WENO5 problem with a step that puts the coarsest level at
        CFL 0.8 (m = 4, 3 levels, 4096 steps);
      * the 4096-cell adjoint problem likewise (m = 4, 3 levels, 2048 steps,
        coarsest CFL 0.8);
      * the 65536-cell problem with the benchmark's N_T = 16384 and m = 16, 3
        levels and a step that puts the coarsest level at CFL 0.8.
    The 1024- and 65536-cell benchmark problems themselves have coarse CFL
    51 and 3277 and diverge, as sec 4 finds for large coarse CFL."""
    import torch

    from paper_2104_09404_amd import workloads as W

    out = {}
    probs = [W.w0_burgers_k0(), W.e4_high_order(2, 0), W.e1_fine_matching(cycle=0), W.e1_fine_matching(cycle=1),
             W.w1_stable_coarse(), W.w4_stable_coarse(), W.w2_stable_coarse()]
    for pb in probs:
        s = mgrit.scheme_from_problem(pb)
        u0 = torch.from_numpy(pb.u0).cuda()
        u = torch.zeros((pb.nt + 1, pb.nx), dtype=torch.float64, device="cuda")
        p = mgrit.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, cycle=pb.cycle,
                         max_iter=max(pb.max_iter, 100), tol=1e-10, sync_every=1,
                         coarse_integrator=pb.coarse_integrator)
        ws = mgrit.alloc_workspace(s, p)
        mgrit.cycle(s, p, u0, u, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, hist, n = mgrit.cycle(s, p, u0, u, ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        ser = gpu_serial_ms(mgrit, s, pb, u0)
        name = pb.name + ("_fcycle" if pb.cycle == 1 else "")
        out[name] = {"ms": ms, "cycles": n, "converged": rc == 0, "residual": hist[-1], "gpu_serial_ms": ser,
                     "mgrit_over_serial": ms / ser, "nx": pb.nx, "nt": pb.nt, "m": pb.m, "levels": pb.levels,
                     "coarsest_cfl": pb.cfl * pb.m ** (pb.levels - 1),
                     "cfl_per_level": [pb.cfl * pb.m ** lv for lv in range(pb.levels)]}
        del u, ws
    out["verdict"] = ("MGRIT faster than GPU serial stepping on: " +
                      ", ".join(k for k, v in out.items() if v["converged"] and v["ms"] < v["gpu_serial_ms"])
                      if any(v["converged"] and v["ms"] < v["gpu_serial_ms"] for v in out.values())
                      else "MGRIT is slower than GPU serial stepping on every converging problem measured")
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the reference-oracle CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the scheme-variant and system sweeps")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratios")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the 1024-cell problem, the batch, the adjoint, the time to "
                         "tolerance and the variant sweeps")
    return ap.parse_args()


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_baseline(pb, budget_s):
    """The reference oracle (plain serial C, the same source as the parity
    checks, built with -O3 -march=native on this host) applying Phi to 2 lines
    of the benchmark problem, repeatedly, for about ``budget_s`` seconds on one
    thread."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import numpy as np
    import oracle

    so = oracle.scheme(pb.nx, flux=pb.flux, k=pb.k, stepper=pb.stepper, a=pb.a, eps=pb.eps, L=pb.L)
    lines = np.ascontiguousarray(np.tile(pb.u0, (2, 1)))
    reps, el, flags = oracle.timing_phi(so, pb.dt, lines, budget_s)
    cells = reps * lines.shape[0] * pb.nx
    model, ncpu, usable = host_cpu()
    return {"value": cells / el, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d Phi steps (WENO5 + LF + SSPRK3) of 2 lines x %d cells of the benchmark problem, "
                      "%.1f s on 1 thread" % (reps, pb.nx, el),
            "build": flags, "host_cpu": model, "host_nproc": ncpu, "host_cpus_usable": usable}


def cpu_mgrit(phi_rate, gpu):
    """The oracle's FAS-MGRIT on the host in the same speed build as
    cpu_baseline: one iteration (V-cycle plus the residual of its result) of
    the 1024-cell problem, and the first-order 64-cell problem to a residual
    of 1e-10.  A CPU iteration of the 65536-cell benchmark problem (about
    five minutes) is not run: it is extrapolated from the measured Phi rate and
    the cell steps of one GPU iteration, and labelled so.  ``gpu`` holds the
    GPU figures of the same problems where the run measured them."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_2104_09404_amd import workloads as W

    def run(pb, max_iter, tol):
        so = oracle.scheme(pb.nx, flux=pb.flux, k=pb.k, stepper=pb.stepper, a=pb.a, eps=pb.eps, L=pb.L)
        po = oracle.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, max_iter=max_iter, tol=tol)
        return oracle.timing_mgrit(so, po, pb.u0)

    out = {}
    pb = W.w1_burgers_weno5()
    el, n, res, _ = run(pb, 1, -1.0)
    rec = {"workload": pb.name, "s_per_iteration": el, "iterations": n, "threads": 1}
    if gpu.get("nx1024_ms_per_step"):
        rec["gpu_ms_per_iteration"] = gpu["nx1024_ms_per_step"]
        rec["cpu_over_gpu"] = el * 1e3 / gpu["nx1024_ms_per_step"]
    out["burgers_weno5_nx1024_one_iteration"] = rec
    pb = W.w0_burgers_k0()
    el, n, res, _ = run(pb, pb.max_iter, 1e-10)
    rec = {"workload": pb.name, "s": el, "cycles": n, "residual": res, "threads": 1}
    if gpu.get("k0_ms_to_tol"):
        rec["gpu_ms"] = gpu["k0_ms_to_tol"]
    out["burgers_k0_fe_nx64_to_1e-10"] = rec
    if gpu.get("cell_steps_per_step"):
        out["burgers_weno5_nx65536_one_iteration"] = {
            "s_per_iteration_extrapolated": gpu["cell_steps_per_step"] / phi_rate,
            "basis": "extrapolated, not run: cell steps of one GPU iteration (%.4g) / the oracle's measured "
                     "Phi rate on this problem's lines" % gpu["cell_steps_per_step"],
            "gpu_ms_per_iteration": gpu.get("ms_per_step"),
        }
    return out


def run_cycles(mgrit, pb, steps, warmup, dominant="relax_fc_l0", storage=0):
    """K fixed V-cycles of problem pb inside one mgrit_cycle call, events on
    the dominant kernel class only; then the same K cycles again with events
    on every class (outside the timed region) for the per-kernel breakdown."""
    import torch

    s = mgrit.scheme_from_problem(pb)
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(pb.u0).to(dev)
    nlines = pb.nt + 1 if storage == 0 else pb.nt // pb.m + 1
    u = torch.zeros((nlines, pb.nx), dtype=torch.float64, device=dev)

    def params(iters):
        return mgrit.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, cycle=0, max_iter=iters,
                            tol=-1.0, storage=storage, sync_every=max(iters, 1))

    ws = mgrit.alloc_workspace(s, params(max(steps, warmup, 1)))
    if warmup > 0:
        mgrit.cycle(s, params(warmup), u0, u, ws)
    torch.cuda.synchronize()
    mgrit.set_profiling(True, classes=[dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, hist, n = mgrit.cycle(s, params(steps), u0, u, ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = mgrit.get_profile()
    mgrit.set_profiling(False)
    mgrit.set_profiling(True)
    mgrit.cycle(s, params(steps), u0, u, ws)
    torch.cuda.synchronize()
    breakdown = mgrit.get_profile()
    mgrit.set_profiling(False)
    del u, ws
    torch.cuda.empty_cache()
    import math

    cells = sum(v["cell_steps"] for v in prof.values())
    dom = prof[dominant]
    dom_ms = dom["ms"] / max(dom["launches"], 1)
    dom_cells = dom["cell_steps"] / max(dom["launches"], 1)
    relax_classes = ["relax_fc_l0", "relax_fr_l0", "relax_fc_coarse", "relax_fr_coarse", "interp"]
    relax_cells = sum(breakdown[c]["cell_steps"] for c in relax_classes)
    relax_ms = sum(breakdown[c]["ms"] for c in relax_classes)
    l0 = breakdown["relax_fc_l0"], breakdown["relax_fr_l0"]
    return {
        "value": cells / wall,
        "wall_s": wall,
        "ms_per_step": wall * 1e3 / steps,
        "cell_steps": cells,
        "dominant_avg_launch_ms": dom_ms,
        "dominant_cell_steps_per_launch": dom_cells,
        "dominant_launches": dom["launches"],
        "relax_cell_steps_per_s": relax_cells / (relax_ms * 1e-3) if relax_ms > 0 else None,
        "level0_relax_cell_steps_per_s": (l0[0]["cell_steps"] + l0[1]["cell_steps"])
        / ((l0[0]["ms"] + l0[1]["ms"]) * 1e-3),
        "kernel_ms_per_step": {k: v["ms"] / steps for k, v in breakdown.items() if v["launches"]},
        "mgrit_converges": bool(math.isfinite(hist[-1]) and hist[-1] < 1e-10),
    }


def measured_executed_flops(kernel):
    """Executed FP64 flops per cell-step of ``kernel`` from the
    SQ_INSTS_VALU_*_F64 counter record profiles/executed_flops.json (FMA = 2,
    x 64 lanes), or None when missing or the sources changed since."""
    rec = _record("executed_flops.json")
    if rec is None or kernel not in rec or not _fresh(rec[kernel]):
        return None
    return rec[kernel]["flops_per_cell_step"]


def roofline(kernel, desc, r):
    achieved = FLOPS_PER_CELL_STEP * r["dominant_cell_steps_per_launch"] / (r["dominant_avg_launch_ms"] * 1e-3)
    executed = measured_executed_flops(kernel)
    rate = r["dominant_cell_steps_per_launch"] / (r["dominant_avg_launch_ms"] * 1e-3)
    return {
        "bound": "alu",
        "kernel": kernel + ": " + desc,
        "achieved": achieved / 1e12,
        "peak": PEAK_FP64 / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64,
        "traffic": measured_traffic(kernel),
        "traffic_unit": "HBM bytes per launch",
        "flops_per_cell_step": FLOPS_PER_CELL_STEP,
        "cell_steps_per_launch": r["dominant_cell_steps_per_launch"],
        "avg_launch_ms": r["dominant_avg_launch_ms"],
        # the counter view: FP64 flops the kernel actually executes (fewer
        # than the algorithmic count: smoothness indicators serve both faces)
        "executed_flops_per_cell_step": executed,
        "executed_frac": None if executed is None else executed * rate / PEAK_FP64,
    }


def batched(mgrit):
    """The 512-problem batch (half Burgers, half advection, N_x log-uniform in
    [256, 8192], N_T = 4 N_x, 2-level FCF, m = 8, C-point storage): one
    mgrit_cycle_batched call of 2 cycles plus the final residual sweep, after
    an untimed warm-up call of 1 cycle; cell-steps/s of the whole call and of
    the level-0 sweeps."""
    import torch

    from paper_2104_09404_amd import workloads as W

    pbs = W.w3_batched()
    table = []
    for pb in pbs:
        u = torch.zeros((pb.nt // pb.m + 1, pb.nx), dtype=torch.float64, device="cuda")
        table.append((mgrit.scheme_from_problem(pb), pb.nt, pb.dt, torch.from_numpy(pb.u0).cuda(), u))
    arr = mgrit.problem_table(table)

    def params(it):
        return mgrit.params(0, 0.0, 8, 2, relax=1, max_iter=it, tol=-1.0, storage=1, sync_every=it)

    ws = torch.empty(mgrit.batched_workspace_bytes(arr, params(2)) // 8 + 64, dtype=torch.float64, device="cuda")
    mgrit.cycle_batched(arr, params(1), workspace=ws)
    torch.cuda.synchronize()
    mgrit.set_profiling(True, classes=[])
    t0 = time.perf_counter()
    mgrit.cycle_batched(arr, params(2), workspace=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = mgrit.get_profile()
    mgrit.set_profiling(False)
    mgrit.set_profiling(True)
    mgrit.cycle_batched(arr, params(2), workspace=ws)
    torch.cuda.synchronize()
    br = mgrit.get_profile()
    mgrit.set_profiling(False)
    cells = sum(v["cell_steps"] for v in prof.values())
    l0 = br["relax_fc_l0"], br["relax_fr_l0"]
    l0_rate = (l0[0]["cell_steps"] + l0[1]["cell_steps"]) / ((l0[0]["ms"] + l0[1]["ms"]) * 1e-3)
    out = {"workload": "batched_512: 512 problems, half Burgers half advection, N_x log-uniform in [256, 8192], "
                       "N_T = 4 N_x, WENO5 + SSPRK3 at CFL U(0.3, 0.9), 2-level FCF, m = 8, C-point storage; "
                       "2 cycles + the final residual sweep",
           "value": cells / wall, "unit": "cell-steps/s", "wall_s": wall,
           "level0_relax_cell_steps_per_s": l0_rate,
           "level0_tflops": FLOPS_PER_CELL_STEP * l0_rate / 1e12,
           "level0_frac_fp64_peak": FLOPS_PER_CELL_STEP * l0_rate / PEAK_FP64,
           "kernel_ms": {k: v["ms"] for k, v in br.items() if v["launches"]}}
    del table, ws
    torch.cuda.empty_cache()
    return out


def adjoint_ratio(mgrit, reps=3):
    """Adjoint/forward time ratio.  (a) The adjoint workload (Burgers WENO5 +
    SSPRK3, N_x = 4096, N_T = 2048, CFL 0.8, checkpoints every 32 steps): the
    reverse sweep including the recomputation of every segment (all segments
    in one launch) over the serial forward that keeps the checkpoints.  Its
    3-level MGRIT forward does not converge (coarse CFL 6.4 / 51).  (b) The
    same problem with m = 4, 3 levels and the coarsest level at CFL 0.8: the
    reverse sweep from the level-0 C-points of an MGRIT forward converged to
    1e-10 (checkpoints every m = 4 steps) over that MGRIT forward, with the
    serial forward of the same problem beside it."""
    import torch

    from paper_2104_09404_amd import workloads as W

    def best(f):
        f()
        torch.cuda.synchronize()
        b = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            b = min(b, time.perf_counter() - t0)
        return b * 1e3

    pb = W.w4_adjoint()
    nx, nt, every = pb.nx, pb.nt, pb.extra["checkpoint_every"]
    s = mgrit.scheme_from_problem(pb)
    u0 = torch.from_numpy(pb.u0).cuda()
    tgt = torch.from_numpy(pb.extra["u_target"]).cuda()
    ck = torch.zeros((nt // every + 1, nx), dtype=torch.float64, device="cuda")
    lam0 = torch.zeros(nx, dtype=torch.float64, device="cuda")
    P = nt // every
    ws = torch.empty(mgrit.adjoint_workspace_bytes(s, nt, every, P) // 8 + 64, dtype=torch.float64, device="cuda")
    t_fwd = best(lambda: mgrit.checkpoints(s, pb.dt, nt, every, u0, ck))
    lamT = (ck[-1] - tgt).contiguous()
    t_rev = best(lambda: mgrit.adjoint(s, pb.dt, nt, every, ck, lamT, lam0, parallel_segments=P, workspace=ws))
    out = {"value": t_rev / t_fwd, "adjoint_ms": t_rev, "forward_ms": t_fwd,
           "workload": "adjoint_nx4096: Burgers WENO5 + SSPRK3, N_x=4096, N_T=2048, CFL 0.8, "
                       "checkpoints every 32 steps, J = 1/2 ||u(T) - u_target||^2",
           "forward": "serial stepping keeping the checkpoints (the 3-level MGRIT forward of this problem "
                      "diverges: coarse CFL 6.4 / 51)"}
    del ws, ck

    q = W.w4_stable_coarse()
    s2 = mgrit.scheme_from_problem(q)
    u02 = torch.from_numpy(q.u0).cuda()
    tgt2 = torch.from_numpy(q.extra["u_target"]).cuda()
    p2 = mgrit.params(q.nt, q.dt, q.m, q.levels, relax=1, max_iter=q.max_iter, tol=1e-10, storage=1, sync_every=1)
    ckm = torch.zeros((q.nt // q.m + 1, q.nx), dtype=torch.float64, device="cuda")
    wsm = mgrit.alloc_workspace(s2, p2)
    res = {}

    def fwd_mgrit():
        res["r"] = mgrit.cycle(s2, p2, u02, ckm, wsm)

    t_mg = best(fwd_mgrit)
    rc, hist, iters = res["r"]
    every2 = q.m
    P2 = q.nt // every2
    wsa = torch.empty(mgrit.adjoint_workspace_bytes(s2, q.nt, every2, P2) // 8 + 64, dtype=torch.float64,
                      device="cuda")
    lamT2 = (ckm[-1] - tgt2).contiguous()
    lam02 = torch.zeros(q.nx, dtype=torch.float64, device="cuda")
    t_rev2 = best(lambda: mgrit.adjoint(s2, q.dt, q.nt, every2, ckm, lamT2, lam02, parallel_segments=P2,
                                        workspace=wsa))
    ck2 = torch.zeros((q.nt // every2 + 1, q.nx), dtype=torch.float64, device="cuda")
    t_ser2 = best(lambda: mgrit.checkpoints(s2, q.dt, q.nt, every2, u02, ck2))
    out["mgrit_forward"] = {
        "workload": q.name + ": N_x=4096, N_T=2048, m=4, 3-level FCF, coarsest CFL 0.8, checkpoints = the "
                             "level-0 C-points (every 4 steps)",
        "converged": rc == 0, "cycles": iters, "residual": hist[-1],
        "mgrit_forward_ms": t_mg, "adjoint_ms": t_rev2, "value": t_rev2 / t_mg,
        "serial_forward_ms": t_ser2, "adjoint_over_serial_forward": t_rev2 / t_ser2}
    del wsm, wsa, ckm, ck2
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the MGRIT sweeps would shard in time across "
              "GPUs, but no multi-GPU path is implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2104_09404_amd import mgrit
    from paper_2104_09404_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mgrit.load()
    pb = W.w2_burgers_weno5_large()
    cpt, nw, tiles = mgrit.tiled_config(pb.nx)
    pair = mgrit.tiled_intervals(pb.nx) == 2
    rag = not (pb.nx % tiles == 0 and (pb.nx // tiles) % cpt == 0)
    # template arguments: cells per thread, waves, WENO degree, stages, ragged, Roe, two chunks per workgroup
    kernel = "tiled_relax_fc_kernel<%d, %d, 2, 3, %s, false, %s>" % (cpt, nw, "true" if rag else "false",
                                                                     "true" if pair else "false")
    r = run_cycles(mgrit, pb, args.steps, args.warmup)
    nch = pb.nt // pb.m
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "burgers_weno5_nx65536: Burgers, WENO5-JS + LF + SSPRK3, CFL 0.8, N_x=65536, "
                        "N_T=16384, m=16, 4-level FCF V-cycle, fixed cycle count, FP64",
            "nx": pb.nx, "nt": pb.nt, "m": pb.m, "levels": pb.levels, "relax": "FCF", "cycle": "V",
            "split_line": {"tiles": tiles, "cells_per_thread": cpt, "waves": nw},
        },
        "roofline": roofline(kernel, "level-0 F-sweep + C-step + residual, %d chunks x %d Phi steps x %d cells "
                                     "(%d tiles per line)" % (nch, pb.m, pb.nx, tiles), r),
        "relax_cell_steps_per_s": r["relax_cell_steps_per_s"],
        "level0_relax_cell_steps_per_s": r["level0_relax_cell_steps_per_s"],
        "kernel_ms_per_step": r["kernel_ms_per_step"],
        "breakdown_note": "relax_*_per_s and kernel_ms_per_step come from a second run of the same K cycles "
                          "with events on every kernel, outside the timed region",
        "mgrit_converges": r["mgrit_converges"],
    }
    if not args.no_extras:
        w1 = W.w1_burgers_weno5()
        r1 = run_cycles(mgrit, w1, 20, 3)
        s1 = mgrit.scheme_from_problem(w1)
        out["burgers_weno5_nx1024"] = {
            "workload": "Burgers, WENO5-JS + LF + SSPRK3, CFL 0.8, N_x=1024, N_T=4096, m=8, 3-level FCF V-cycle, "
                        "20 fixed cycles",
            "value": r1["value"], "unit": "cell-steps/s", "ms_per_step": r1["ms_per_step"],
            "roofline": roofline(ONE_WG_FC, "level-0 F-sweep + C-step + residual, 512 chunks x 8 Phi steps x "
                                            "1024 cells", r1),
            "relax_cell_steps_per_s": r1["relax_cell_steps_per_s"],
            "level0_relax_cell_steps_per_s": r1["level0_relax_cell_steps_per_s"],
            "kernel_ms_per_step": r1["kernel_ms_per_step"],
            "mgrit_converges": r1["mgrit_converges"],
            "gpu_serial_ms": gpu_serial_ms(mgrit, s1, w1, torch.from_numpy(w1.u0).cuda()),
        }
        w0 = W.w0_burgers_k0()
        r0 = run_cycles(mgrit, w0, 50, 3, dominant="relax_fr_l0")
        rate0 = r0["level0_relax_cell_steps_per_s"]
        out["burgers_k0_fe_nx64"] = {
            "workload": "Burgers, first-order LF + forward Euler, N_x=64, N_T=256, m=4, 2-level F-relaxation V-cycle, "
                        "50 fixed cycles (a correctness configuration)",
            "value": r0["value"], "unit": "cell-steps/s", "ms_per_step": r0["ms_per_step"],
            "level0_relax_cell_steps_per_s": rate0,
            "frac_fp64_peak": K0_FE_FLOPS_PER_CELL_STEP * rate0 / PEAK_FP64,
            "frac_hbm_peak": K0_FE_BYTES_PER_CELL_STEP * rate0 / PEAK_HBM,
            "note": "64 chunks of 64-cell lines fill 64 wavefronts of a 256-CU GPU: the sweeps are latency bound "
                    "and neither the FP64 roofline (%g flops per cell-step) nor the HBM roofline (%g B per "
                    "materialised cell-step) is reachable" % (K0_FE_FLOPS_PER_CELL_STEP, K0_FE_BYTES_PER_CELL_STEP),
            "kernel_ms_per_step": r0["kernel_ms_per_step"],
        }
        out["batched_512"] = batched(mgrit)
        out["adjoint_forward_ratio"] = None if args.no_adjoint else adjoint_ratio(mgrit)
        out["time_to_tolerance"] = time_to_tolerance(mgrit)
        out["gpu_serial_ms"] = gpu_serial_ms(mgrit, mgrit.scheme_from_problem(pb), pb,
                                             torch.from_numpy(pb.u0).cuda(), reps=1)
        out["scheme_variants"] = None if args.no_variants else variant_rates()
        out["systems"] = None if args.no_variants else system_rates()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb, args.cpu_seconds)
        gpu = {"cell_steps_per_step": r["cell_steps"] / args.steps, "ms_per_step": r["ms_per_step"]}
        if isinstance(out.get("burgers_weno5_nx1024"), dict):
            gpu["nx1024_ms_per_step"] = out["burgers_weno5_nx1024"]["ms_per_step"]
        ttt = out.get("time_to_tolerance")
        if isinstance(ttt, dict) and isinstance(ttt.get("burgers_k0_fe_nx64"), dict):
            gpu["k0_ms_to_tol"] = ttt["burgers_k0_fe_nx64"]["ms"]
        out["cpu_baseline"]["mgrit"] = cpu_mgrit(out["cpu_baseline"]["value"], gpu)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
