"""Small drivers for hardware-counter runs (rocprofv3 --pmc ...).

    python -m paper_2104_09404_amd.profiling copy [MiB]
        a plain device-to-device copy of a known size (default 256 MiB, five
        times): the reference that converts the FETCH_SIZE / WRITE_SIZE
        counters of other kernels into bytes.
    python -m paper_2104_09404_amd.profiling sweep [steps]
        only the level-0 relaxation sweeps of the N_x = 1024 benchmark workload
        (mgrit_relax F-sweeps on the full level-0 array), for counter runs
        that should not include the rest of the cycle.
    python -m paper_2104_09404_amd.profiling variants [reps]
        the same level-0 F-sweep (512 chunks x 7 steps x 1024 cells, SSPRK3)
        for every reconstruction degree k = 0..3 with the Lax-Friedrichs and
        the Roe flux, each `reps` times in the order of VARIANTS, with its
        time per sweep from HIP events on the launch stream.
    python -m paper_2104_09404_amd.profiling systems [reps]
        the same shape of F-sweep (512 chunks x 7 SSPRK3 steps) for shallow
        water and Euler on 512-cell lines, WENO degrees 0, 2 and 3, LF and Roe,
        in the order of SYSTEMS.
    python -m paper_2104_09404_amd.profiling cycle1024 [cycles]
        only `cycles` V-cycles (default 3) of the N_x = 1024 workload
        (N_T = 4096, m = 8, 3-level FCF, fixed count), for counter runs on its
        level-0 sweep kernel without the rest of the benchmark.
    python -m paper_2104_09404_amd.profiling shortlines [reps]
        F-sweeps of 4096 chunks of 15 WENO5 + SSPRK3 steps on 256-cell lines
        (mgrit_relax on 65537 nodes, m = 16) under every compiled
        one-workgroup shape that covers 256 cells (SHORT_SHAPES), with
        HIP-event times per sweep.
    python -m paper_2104_09404_amd.profiling serial [reps]
        serial time stepping of the 65536-cell workload (workloads.
        w2_burgers_weno5_large: N_T = 16384 steps of Phi on one line,
        mgrit_serial), `reps` times after one warm-up, each timed with HIP
        events on the launch stream; the launch's tile shape is printed.
    python -m paper_2104_09404_amd.profiling batch [cycles]
        the 512-problem batch (workloads.w3_batched, 2-level FCF, m = 8,
        C-point storage): one warm-up call of one cycle, then one
        mgrit_cycle_batched call of `cycles` cycles (default 2) plus the final
        residual sweep, timed on the host around a synchronised call.
"""
from __future__ import annotations

import sys


def copy(mib: int = 256, reps: int = 5):
    import torch

    n = mib * 1024 * 1024 // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d MiB x %d" % (mib, reps))


def sweep(reps: int = 3):
    import numpy as np
    import torch

    from . import mgrit
    from . import workloads as W

    pb = W.w1_burgers_weno5()
    s = mgrit.scheme_from_problem(pb)
    lvl = torch.from_numpy(np.tile(pb.u0, (pb.nt + 1, 1))).cuda()
    for _ in range(reps):
        mgrit.relax(s, pb.dt, pb.m, 0, lvl, None, pb.nt)
    torch.cuda.synchronize()
    print("ran %d F-sweeps of %d chunks" % (reps, pb.nt // pb.m))


# (k, numflux) in the order the variant sweeps run
VARIANTS = [(0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (1, 1), (2, 1), (3, 1)]


def variant_name(k: int, numflux: int) -> str:
    return "weno%d_%s" % (2 * k + 1, "roe" if numflux else "lf")


def variants(reps: int = 5, quiet: bool = False) -> dict:
    """Level-0 F-sweeps of the benchmark shape per scheme variant; returns
    {name: {"ms_per_sweep", "cell_steps", "cell_steps_per_s"}} (median of
    ``reps`` sweeps, each bracketed by HIP events on the current stream)."""
    import numpy as np
    import torch

    from . import mgrit
    from . import workloads as W

    pb = W.w1_burgers_weno5()
    base = np.tile(pb.u0, (pb.nt + 1, 1))
    lvl = torch.from_numpy(base).cuda()
    nchunks = pb.nt // pb.m
    cell_steps = float(nchunks * (pb.m - 1) * pb.nx)
    st = torch.cuda.current_stream()
    out = {}
    for k, numflux in VARIANTS:
        s = mgrit.scheme(pb.nx, k=k, stepper=3, numflux=numflux)
        mgrit.relax(s, pb.dt, pb.m, 0, lvl, None, pb.nt)  # warm-up
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            mgrit.relax(s, pb.dt, pb.m, 0, lvl, None, pb.nt)
            e1.record(st)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        out[variant_name(k, numflux)] = {"ms_per_sweep": med, "cell_steps": cell_steps,
                                         "cell_steps_per_s": cell_steps / (med * 1e-3)}
        if not quiet:
            print("%s %.4f ms per sweep" % (variant_name(k, numflux), med), flush=True)
    return out


# (system, k, numflux) in the order the system sweeps run
SYSTEMS = [(sysname, k, numflux) for sysname in ("sw", "euler") for k in (0, 2, 3) for numflux in (0, 1)]


def system_name(sysname: str, k: int, numflux: int) -> str:
    return "%s_weno%d_%s" % (sysname, 2 * k + 1, "roe" if numflux else "lf")


def systems(reps: int = 5, quiet: bool = False) -> dict:
    """Level-0 F-sweeps of 512 chunks x 7 steps on 512-cell lines of shallow
    water (h = 1 + sin(2 pi x)/4, hu = 0) and Euler (rho = 1, rho u = 0,
    E = 1 + sin(2 pi x)/4) at CFL 0.4; returns {name: {"ms_per_sweep",
    "cell_steps", "cell_steps_per_s"}} (median of ``reps``, HIP events)."""
    import math

    import numpy as np
    import torch

    from . import mgrit
    from . import workloads as W

    nx, m, nt = 512, 8, 4096
    sn = W.cell_average_sin(nx, 1, 0.0)
    init = {"sw": (np.concatenate([1.0 + 0.25 * sn, np.zeros(nx)]), math.sqrt(9.81 * 1.25)),
            "euler": (np.concatenate([np.ones(nx), np.zeros(nx), 1.0 + 0.25 * sn]),
                      math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * 1.25))}
    cell_steps = float((nt // m) * (m - 1) * nx)
    st = torch.cuda.current_stream()
    out = {}
    for sysname, k, numflux in SYSTEMS:
        u0, speed = init[sysname]
        lvl = torch.from_numpy(np.tile(u0, (nt + 1, 1))).cuda()
        s = (mgrit.shallow_water_scheme(nx, k=k, numflux=numflux) if sysname == "sw"
             else mgrit.euler_scheme(nx, k=k, numflux=numflux))
        dt = 0.4 / nx / speed
        mgrit.relax(s, dt, m, 0, lvl, None, nt)  # warm-up
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            mgrit.relax(s, dt, m, 0, lvl, None, nt)
            e1.record(st)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        name = system_name(sysname, k, numflux)
        out[name] = {"ms_per_sweep": med, "cell_steps": cell_steps, "cell_steps_per_s": cell_steps / (med * 1e-3)}
        if not quiet:
            print("%s %.4f ms per sweep" % (name, med), flush=True)
        del lvl
    return out


def cycle1024(cycles: int = 3):
    import torch

    from . import mgrit
    from . import workloads as W

    pb = W.w1_burgers_weno5()
    s = mgrit.scheme_from_problem(pb)
    p = mgrit.params(pb.nt, pb.dt, pb.m, pb.levels, relax=1, max_iter=cycles, tol=-1.0, sync_every=cycles)
    u = torch.zeros((pb.nt + 1, pb.nx), dtype=torch.float64, device="cuda")
    mgrit.cycle(s, p, torch.from_numpy(pb.u0).cuda(), u)
    torch.cuda.synchronize()
    print("ran %d cycles of the %d-cell problem" % (cycles, pb.nx))


SHORT_SHAPES = [(4, 1), (2, 2), (1, 4), (2, 4), (1, 8)]


def shortlines(reps: int = 5, quiet: bool = False) -> dict:
    import numpy as np
    import torch

    from . import mgrit
    from . import workloads as W

    nx, m, n = 256, 16, 65536
    s = mgrit.scheme(nx)
    u = torch.from_numpy(W.random_lines(7, 1, nx)).cuda().repeat(n + 1, 1)
    dt = 0.5 / nx / float(u.abs().max())
    out = {}
    for cpt, nw in SHORT_SHAPES:
        mgrit.clear_kernel_config()
        mgrit.set_kernel_config(nx, nx, cpt, nw, latency=False)
        mgrit.relax(s, dt, m, 0, u, None, n)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mgrit.relax(s, dt, m, 0, u, None, n)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        med = float(np.median(ts))
        cells = (n // m) * (m - 1) * nx
        out["%dx%d" % (cpt, nw)] = {"ms": med, "cell_steps_per_s": cells / (med * 1e-3)}
        if not quiet:
            print("(%d, %d): %.4f ms per sweep, %.3e cell-steps/s" % (cpt, nw, med, cells / (med * 1e-3)), flush=True)
    mgrit.clear_kernel_config()
    return out


def serial(reps: int = 2):
    import torch

    from . import mgrit
    from . import workloads as W

    pb = W.w2_burgers_weno5_large()
    s = mgrit.scheme_from_problem(pb)
    u0 = torch.from_numpy(pb.u0).cuda()
    out = torch.empty((pb.nt + 1, pb.nx), dtype=torch.float64, device="cuda")
    print("serial stepping, N_x = %d, N_T = %d: tiles (cells per thread, waves, tiles) = %s"
          % (pb.nx, pb.nt, mgrit.tiled_launch_config(pb.nx, 1)), flush=True)
    mgrit.serial(s, pb.dt, pb.nt, u0, out)
    torch.cuda.synchronize()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mgrit.serial(s, pb.dt, pb.nt, u0, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        print("  %.2f ms, %.3f us per Runge-Kutta stage" % (ms, 1e3 * ms / (3 * pb.nt)), flush=True)


def batch(cycles: int = 2):
    import time

    import torch

    from . import mgrit
    from . import workloads as W

    pbs = W.w3_batched()
    table = []
    for pb in pbs:
        u = torch.zeros((pb.nt // pb.m + 1, pb.nx), dtype=torch.float64, device="cuda")
        table.append((mgrit.scheme_from_problem(pb), pb.nt, pb.dt, torch.from_numpy(pb.u0).cuda(), u))
    arr = mgrit.problem_table(table)

    def params(it):
        return mgrit.params(0, 0.0, 8, 2, relax=1, max_iter=it, tol=-1.0, storage=1, sync_every=it)

    ws = torch.empty(mgrit.batched_workspace_bytes(arr, params(cycles)) // 8 + 64, dtype=torch.float64,
                     device="cuda")
    mgrit.cycle_batched(arr, params(1), workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mgrit.cycle_batched(arr, params(cycles), workspace=ws)
    torch.cuda.synchronize()
    print("batch of %d problems, %d cycles: %.3f s" % (len(pbs), cycles, time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "copy"
    if what == "copy":
        copy(int(sys.argv[2]) if len(sys.argv) > 2 else 256)
    elif what == "sweep":
        sweep(int(sys.argv[2]) if len(sys.argv) > 2 else 3)
    elif what == "variants":
        variants(int(sys.argv[2]) if len(sys.argv) > 2 else 5)
    elif what == "systems":
        systems(int(sys.argv[2]) if len(sys.argv) > 2 else 5)
    elif what == "cycle1024":
        cycle1024(int(sys.argv[2]) if len(sys.argv) > 2 else 3)
    elif what == "shortlines":
        shortlines(int(sys.argv[2]) if len(sys.argv) > 2 else 5)
    elif what == "serial":
        serial(int(sys.argv[2]) if len(sys.argv) > 2 else 2)
    elif what == "batch":
        batch(int(sys.argv[2]) if len(sys.argv) > 2 else 2)
    else:
        raise SystemExit("usage: python -m paper_2104_09404_amd.profiling "
                         "copy|sweep|variants|systems|cycle1024|shortlines|batch [n]")
