"""The allocation-free cycle (mgrit_cycle_noalloc, static device workspace)
against mgrit_cycle with a caller workspace, through the C ABI: identical
iterates and residual histories on consecutive calls of decreasing size (the
static workspace keeps the previous call's contents), on a split line and a
split system line, and refusal of a problem larger than the static
workspace."""
import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_09404_amd import mgrit

    mgrit.load()
    return mgrit


def solve_both(gpu, pb, iters, relax):
    import torch

    s = gpu.scheme_from_problem(pb)
    p = gpu.params(pb.nt, pb.dt, pb.m, pb.levels, relax=relax, max_iter=iters, tol=-1.0)
    assert gpu.workspace_bytes(s, p) <= gpu.NOALLOC_SCRATCH_BYTES
    u0 = torch.from_numpy(pb.u0).cuda()
    ref = torch.zeros((pb.nt + 1, pb.nx), dtype=torch.float64, device="cuda")
    rc_r, h_r, n_r = gpu.cycle(s, p, u0, ref)
    got = torch.full((pb.nt + 1, pb.nx), float("nan"), dtype=torch.float64, device="cuda")
    rc_g, h_g, n_g = gpu.cycle_noalloc(s, p, u0, got)
    torch.cuda.synchronize()
    assert (rc_g, n_g) == (rc_r, n_r) == (gpu.MGRIT_NOT_CONVERGED, iters)
    assert np.all(np.isfinite(h_r)) and h_r[-1] < 0.5 * h_r[0]
    assert np.array_equal(np.array(h_g).view(np.int64), np.array(h_r).view(np.int64))
    assert torch.equal(got.view(torch.int64), ref.view(torch.int64))
    return got


def test_noalloc_matches_cycle_on_consecutive_calls(gpu):
    """1024 cells x 4096 steps of WENO5 (3-level FCF, m = 4, coarsest CFL 0.8;
    26 MB of workspace), then 64 cells x 256 steps of the first-order scheme
    (2-level F, m = 4): the second call runs on the first one's leftovers.
    Iterates and residual histories are compared bit for bit."""
    big = W.w1_stable_coarse()
    solve_both(gpu, big, 3, 1)
    small = W.w0_burgers_k0()
    solve_both(gpu, small, 4, 0)


def test_noalloc_split_line(gpu):
    """An 8192-cell line (two tiles that meet once per stage through the
    synchronisation scratch, here inside the static workspace)."""
    pb = W.w1_stable_coarse(nx=8192, nt=64, m=4, levels=2)
    assert gpu.tiled_config(pb.nx)[2] > 1
    solve_both(gpu, pb, 2, 1)


def test_noalloc_refuses_oversized_problem(gpu):
    import ctypes as C

    import torch

    pb = W.w2_burgers_weno5_large()
    s = gpu.scheme_from_problem(pb)
    p = gpu.params(pb.nt, pb.dt, pb.m, pb.levels, relax=1, max_iter=2, tol=-1.0)
    assert gpu.workspace_bytes(s, p) > gpu.NOALLOC_SCRATCH_BYTES
    L = gpu.load()
    hist = (C.c_double * 3)()
    it = C.c_int32(0)
    u0 = torch.zeros(pb.nx, dtype=torch.float64, device="cuda")
    u1 = torch.zeros((1, pb.nx), dtype=torch.float64, device="cuda")
    rc = L.mgrit_cycle_noalloc(C.byref(s), C.byref(p), u0.data_ptr(), u1.data_ptr(), hist, C.byref(it), None)
    assert rc == gpu.MGRIT_EINVAL
    assert b"static workspace" in L.mgrit_last_error()


def test_noalloc_split_system_line(gpu):
    """Euler on a 1000-cell line (two tiles of a split system line, their
    synchronisation scratch inside the static workspace), 2-level FCF with a
    stable coarse step: bit for bit as mgrit_cycle."""
    import torch

    nx, nt, m, gam = 1000, 64, 4, 5.0 / 3.0
    sn = W.cell_average_sin(nx, 1, 0.0)
    rho, p = 1.0 + 0.2 * sn, 1.0 + 0.2 * np.roll(sn, nx // 3)
    u0 = np.concatenate([rho, np.zeros(nx), p / (gam - 1.0)])
    smax = float(np.max(np.sqrt(gam * p / rho)))
    dt = 0.8 / m / nx / smax
    s = gpu.euler_scheme(nx, gamma=gam)
    assert gpu.sys_tiles(s) == 2
    pr = gpu.params(nt, dt, m, 2, relax=1, max_iter=2, tol=-1.0)
    assert gpu.workspace_bytes(s, pr) <= gpu.NOALLOC_SCRATCH_BYTES
    u0d = torch.from_numpy(u0).cuda()
    ref = torch.zeros((nt + 1, 3 * nx), dtype=torch.float64, device="cuda")
    rc_r, h_r, n_r = gpu.cycle(s, pr, u0d, ref)
    got = torch.full((nt + 1, 3 * nx), float("nan"), dtype=torch.float64, device="cuda")
    rc_g, h_g, n_g = gpu.cycle_noalloc(s, pr, u0d, got)
    torch.cuda.synchronize()
    assert (rc_g, n_g) == (rc_r, n_r)
    assert np.all(np.isfinite(h_r)) and h_r[-1] < 0.5 * h_r[0]
    assert np.array_equal(np.array(h_g).view(np.int64), np.array(h_r).view(np.int64))
    assert torch.equal(got.view(torch.int64), ref.view(torch.int64))
