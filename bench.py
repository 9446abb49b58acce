"""Benchmark: fine cell-steps per second of FAS-MGRIT V-cycles on one MI355X.

Workload (the configuration the metric is quoted on): inviscid Burgers,
WENO5-JS (eps = 1e-6) + Lax-Friedrichs flux + SSPRK3 at CFL 0.8, N_x = 1024,
N_T = 4096, m = 8, 3-level FCF V-cycle, FP64, u0 = 0.5 + 4 seeded Fourier
modes (synthetic, seed 210409404 + 1).

One "step" is one MGRIT iteration: the level-0 F-relaxation that yields the
residual, the C-relaxation and second F-sweep fused with the FAS restriction,
the level-1 FCF relaxation and restriction, the serial coarsest solve, and the
ideal interpolation.  The timed region runs K such iterations inside one
mgrit_cycle call on data resident in HBM (tol < 0, so no early exit), i.e.
K cycles plus the residual sweep of the final iterate.

value = (cell steps executed by all kernels of the region) / (wall time of
the region), where a cell step is one application of Phi to one cell.  The
library's HIP events around every kernel (on the launch stream) give the
per-kernel durations used for the roofline of the dominant kernel, the fused
level-0 F + C sweep.
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
DOMINANT = "relax_fc_kernel<4, 4, 2, 3, false, false>"


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the FETCH_SIZE / WRITE_SIZE counter
    record in profiles/traffic.json (counters scaled by a plain copy of known
    size), or None when the record is missing or the kernel's sources changed
    since the counters were taken."""
    import hashlib

    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            rec = json.load(f)[kernel]
        h = hashlib.sha256()
        for name in rec["sources"]:
            with open(os.path.join(ROOT, name), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def measured_variant_flops():
    """Executed FP64 flops per cell-step of each scheme variant's level-0
    F-sweep, from the SQ_INSTS_VALU_*_F64 counter record in
    profiles/variant_flops.json (FMA = 2 flops, x 64 lanes), or None when the
    record is missing or the kernel sources changed since it was taken."""
    import hashlib

    try:
        with open(os.path.join(ROOT, "profiles", "variant_flops.json")) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for name in rec["sources"]:
            with open(os.path.join(ROOT, name), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    return rec["flops_per_cell_step"] if h.hexdigest() == rec["sources_sha256"] else None


def variant_rates():
    """Row f3 measured: the level-0 F-sweep of the benchmark shape for every
    reconstruction degree with the LF and the Roe flux."""
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


def measured_system_flops():
    """Executed FP64 flops per cell-step of the system sweeps from
    profiles/system_flops.json, or None when missing or stale (as for the
    scheme variants)."""
    import hashlib

    try:
        with open(os.path.join(ROOT, "profiles", "system_flops.json")) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for name in rec["sources"]:
            with open(os.path.join(ROOT, name), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    return rec["flops_per_cell_step"] if h.hexdigest() == rec["sources_sha256"] else None


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


def time_to_tolerance(mgrit):
    """MGRIT wall time to a residual of 1e-10 where MGRIT converges (the
    benchmark workload's coarse CFL of 51 makes it diverge, as the paper
    finds for large coarse CFL): the first-order workload and the paper's
    high-order experiment with WENO5 + LF."""
    import torch

    from paper_2104_09404_amd import workloads as W

    out = {}
    for pb in (W.w0_burgers_k0(), W.e4_high_order(2, 0)):
        s = mgrit.scheme_from_problem(pb)
        u0 = torch.from_numpy(pb.u0).cuda()
        u = torch.zeros((pb.nt + 1, pb.nx), dtype=torch.float64, device="cuda")
        p = mgrit.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, max_iter=max(pb.max_iter, 100),
                         tol=1e-10, sync_every=1)
        ws = mgrit.alloc_workspace(s, p)
        mgrit.cycle(s, p, u0, u, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, hist, n = mgrit.cycle(s, p, u0, u, ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[pb.name] = {"ms": ms, "cycles": n, "converged": rc == 0, "residual": hist[-1],
                        "gpu_serial_ms": gpu_serial_ms(mgrit, s, pb, u0)}
    return out


def gpu_serial_ms(mgrit, s, pb, u0, reps=3):
    """Serial time stepping of the same problem on the GPU (N_T steps of Phi on
    one line, one workgroup), the comparison point for the MGRIT solve."""
    import torch

    out = torch.empty((pb.nt + 1, pb.nx), dtype=torch.float64, device=u0.device)
    mgrit.serial(s, pb.dt, pb.nt, u0, out)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        mgrit.serial(s, pb.dt, pb.nt, u0, out)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best * 1e3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the reference-oracle CPU baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the scheme-variant and system sweeps")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward ratio (its split-line launches are cooperative)")
    return ap.parse_args()


def cpu_baseline(pb, budget_s):
    """The reference oracle (plain serial C) applying Phi to W1 lines on the host:
    one Phi step of all 512 level-0 chunk lines per repetition, repeated for about
    ``budget_s`` seconds.  Single thread."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import numpy as np
    import oracle

    so = oracle.scheme(pb.nx, flux=pb.flux, k=pb.k, stepper=pb.stepper, a=pb.a, eps=pb.eps, L=pb.L)
    lines = np.ascontiguousarray(np.tile(pb.u0, (64, 1)))
    reps = 0
    t0 = time.perf_counter()
    while True:
        lines = oracle.phi(so, pb.dt, lines)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    cells = reps * lines.shape[0] * pb.nx
    return {"value": cells / el, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d Phi steps of 64 lines x %d cells of the benchmark workload (%.1f s, 1 thread)"
                      % (reps, pb.nx, el)}


def adjoint_ratio(mgrit, reps=3):
    """Adjoint workload (Burgers WENO5 + SSPRK3, N_x = 4096, N_T = 2048, CFL 0.8,
    checkpoints every 32 steps): time of the reverse sweep including the
    recomputation of every segment (all 64 segments recomputed in one launch)
    over the time of the forward it differentiates (serial stepping keeping the
    checkpoints).  The 3-level MGRIT forward of this workload does not converge
    (coarse CFL 6.4 / 51), so the serial forward is the denominator."""
    import torch

    from paper_2104_09404_amd import workloads as W

    pb = W.w4_adjoint()
    nx, nt, every = pb.nx, pb.nt, pb.extra["checkpoint_every"]
    s = mgrit.scheme_from_problem(pb)
    u0 = torch.from_numpy(pb.u0).cuda()
    tgt = torch.from_numpy(pb.extra["u_target"]).cuda()
    ck = torch.zeros((nt // every + 1, nx), dtype=torch.float64, device="cuda")
    lam0 = torch.zeros(nx, dtype=torch.float64, device="cuda")
    P = nt // every
    ws = torch.empty(mgrit.adjoint_workspace_bytes(s, nt, every, P) // 8 + 64, dtype=torch.float64, device="cuda")

    def fwd():
        mgrit.checkpoints(s, pb.dt, nt, every, u0, ck)

    def rev():
        mgrit.adjoint(s, pb.dt, nt, every, ck, lamT, lam0, parallel_segments=P, workspace=ws)

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

    t_fwd = best(fwd)
    lamT = (ck[-1] - tgt).contiguous()
    t_rev = best(rev)
    return {"value": t_rev / t_fwd, "adjoint_ms": t_rev, "forward_ms": t_fwd,
            "workload": "adjoint_nx4096: Burgers WENO5 + SSPRK3, N_x=4096, N_T=2048, CFL 0.8, "
                        "checkpoints every 32 steps, J = 1/2 ||u(T) - u_target||^2",
            "forward": "serial stepping keeping the checkpoints (the MGRIT forward does not converge here)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the MGRIT sweeps would shard in time across "
              "GPUs, but no multi-GPU path is implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2104_09404_amd import mgrit
    from paper_2104_09404_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mgrit.load()
    pb = W.w1_burgers_weno5()
    s = mgrit.scheme_from_problem(pb)
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(pb.u0).to(dev)
    u = torch.zeros((pb.nt + 1, pb.nx), dtype=torch.float64, device=dev)

    def params(iters):
        return mgrit.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, cycle=0, max_iter=iters,
                            tol=-1.0, storage=0, sync_every=max(iters, 1))

    ws = mgrit.alloc_workspace(s, params(max(args.steps, args.warmup)))
    if args.warmup > 0:
        mgrit.cycle(s, params(args.warmup), u0, u, ws)
    torch.cuda.synchronize()

    # timed region: K iterations; HIP events bracket the dominant kernel only
    # (every event pair costs stream time), the other kernels are counted
    mgrit.set_profiling(True, classes=["relax_fc_l0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, hist, n = mgrit.cycle(s, params(args.steps), u0, u, ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = mgrit.get_profile()
    mgrit.set_profiling(False)
    # per-kernel breakdown: the same K iterations again, outside the timed
    # region, with events on every kernel
    mgrit.set_profiling(True)
    mgrit.cycle(s, params(args.steps), u0, u, ws)
    torch.cuda.synchronize()
    breakdown = mgrit.get_profile()
    mgrit.set_profiling(False)

    cells = sum(v["cell_steps"] for v in prof.values())
    value = cells / wall
    dom = prof["relax_fc_l0"]
    dom_ms = dom["ms"] / max(dom["launches"], 1)
    dom_flops = FLOPS_PER_CELL_STEP * dom["cell_steps"] / max(dom["launches"], 1)
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    relax_classes = ["relax_fc_l0", "relax_fr_l0", "relax_fc_coarse", "relax_fr_coarse", "interp"]
    relax_cells = sum(breakdown[c]["cell_steps"] for c in relax_classes)
    relax_ms = sum(breakdown[c]["ms"] for c in relax_classes)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "burgers_weno5_nx1024: Burgers, WENO5-JS + LF + SSPRK3, CFL 0.8, N_x=1024, "
                        "N_T=4096, m=8, 3-level FCF V-cycle, FP64",
            "nx": pb.nx, "nt": pb.nt, "m": pb.m, "levels": pb.levels, "relax": "FCF", "cycle": "V",
        },
        "roofline": {
            "bound": "alu",
            "kernel": DOMINANT + ": level-0 F-sweep + C-step + residual, 512 chunks x 8 Phi steps x 1024 cells",
            "achieved": achieved,
            "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved * 1e12 / PEAK_FP64,
            "traffic": measured_traffic(DOMINANT),
            "traffic_unit": "HBM bytes per launch",
            "flops_per_cell_step": FLOPS_PER_CELL_STEP,
            "avg_launch_ms": dom_ms,
        },
        "relax_cell_steps_per_s": relax_cells / (relax_ms * 1e-3) if relax_ms > 0 else None,
        "level0_relax_cell_steps_per_s": (breakdown["relax_fc_l0"]["cell_steps"]
                                          + breakdown["relax_fr_l0"]["cell_steps"])
        / ((breakdown["relax_fc_l0"]["ms"] + breakdown["relax_fr_l0"]["ms"]) * 1e-3),
        "kernel_ms_per_step": {k: v["ms"] / args.steps for k, v in breakdown.items() if v["launches"]},
        "breakdown_note": "relax_*_per_s and kernel_ms_per_step come from a second run of the same K cycles "
                          "with events on every kernel, outside the timed region",
        "adjoint_forward_ratio": None if args.no_adjoint else adjoint_ratio(mgrit),
        "mgrit_converges": bool(np.isfinite(hist[-1]) and hist[-1] < 1e-10),
        "gpu_serial_ms": gpu_serial_ms(mgrit, s, pb, u0),
        "time_to_tolerance": time_to_tolerance(mgrit),
        "scheme_variants": None if args.no_variants else variant_rates(),
        "systems": None if args.no_variants else system_rates(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
