"""Small drivers for hardware-counter runs (rocprofv3 --pmc ...).

    python -m paper_2104_09404_amd.profiling copy [MiB]
        a plain device-to-device copy of a known size (default 256 MiB, five
        times): the reference that converts the FETCH_SIZE / WRITE_SIZE
        counters of other kernels into bytes.
    python -m paper_2104_09404_amd.profiling sweep [steps]
        only the level-0 relaxation sweeps of the N_x = 1024 benchmark workload
        (mgrit_relax F-sweeps on the full level-0 array), for counter runs
        that should not include the rest of the cycle.
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


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "copy"
    if what == "copy":
        copy(int(sys.argv[2]) if len(sys.argv) > 2 else 256)
    elif what == "sweep":
        sweep(int(sys.argv[2]) if len(sys.argv) > 2 else 3)
    else:
        raise SystemExit("usage: python -m paper_2104_09404_amd.profiling copy|sweep [n]")
