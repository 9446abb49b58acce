"""GPU parity of batches of independent problems (mgrit_cycle_batched): every
problem's iterate and residual history bitwise equal to mgrit_cycle on that
problem alone (mixed line lengths, ragged and split lines, both fluxes),
per-problem retirement at convergence, and the 512-problem workload (N_x
log-uniform in [256, 8192], N_T = 4 N_x, m = 8, 2-level FCF) at full size
against the oracle on its 16 smallest and 2 largest problems."""
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


def T(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def H(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_lines(x, ref):
    x = np.atleast_2d(x)
    ref = np.atleast_2d(ref)
    return np.linalg.norm(x - ref, axis=-1) / np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)


def mixed_problems(gpu, nxs, cfl, m, seed):
    g = np.random.default_rng(seed)
    out = []
    for i, nx in enumerate(nxs):
        flux = i % 2
        a = float(g.uniform(0.5, 1.5)) if flux == 1 else 1.0
        u0 = W.random_lines(seed * 100 + i, 1, nx)[0]
        speed = np.max(np.abs(u0)) if flux == 0 else a
        dt = cfl / nx / speed
        nt = 4 * m * max(1, nx // (4 * m))
        nt -= nt % m
        out.append((gpu.scheme(nx, flux=flux, a=a), nt, dt, u0))
    return out


def run_batch(gpu, probs, p):
    us = []
    table = []
    for sch, nt, dt, u0 in probs:
        nl = nt + 1 if p.storage == 0 else nt // p.m + 1
        u = T(np.zeros((nl, sch.nx)))
        us.append(u)
        table.append((sch, nt, dt, T(u0), u))
    hs, its, sts = gpu.cycle_batched(table, p)
    return [H(u) for u in us], hs, its, sts


def run_single(gpu, prob, p):
    sch, nt, dt, u0 = prob
    q = gpu.params(nt, dt, p.m, p.levels, relax=p.relax, cycle=p.cycle, max_iter=p.max_iter, tol=p.tol,
                   storage=p.storage, coarse_guess=p.coarse_guess, sync_every=p.sync_every)
    nl = nt + 1 if p.storage == 0 else nt // p.m + 1
    u = T(np.zeros((nl, sch.nx)))
    rc, hist, n = gpu.cycle(sch, q, T(u0), u)
    return H(u), hist, n, rc


def same(a, b):
    with np.errstate(invalid="ignore"):
        return bool(np.all((a == b) | (np.isnan(a) & np.isnan(b))))


def close_hist(a, b):
    """Residual norms: the batch may run a problem's sweeps in another launch
    configuration than its own solve (the batch has more lines), which groups
    the per-chunk partial sums differently; iterates are bitwise equal."""
    a, b = np.asarray(a), np.asarray(b)
    if a.shape != b.shape:
        return False
    with np.errstate(invalid="ignore"):
        ok = (np.abs(a - b) <= 1e-13 * np.abs(b)) | (np.isnan(a) & np.isnan(b)) | (a == b)
    return bool(np.all(ok))


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("levels,relax,cycle", [(2, 1, 0), (3, 1, 0), (3, 0, 1)])
def test_batch_equals_single_problems(gpu, storage, levels, relax, cycle):
    nxs = [64, 100, 256, 300, 514, 1000, 1024, 2050, 4096, 4098, 6002, 130]
    m = 4
    probs = mixed_problems(gpu, nxs, 0.6, m, 3 + levels)
    p = gpu.params(0, 0.0, m, levels, relax=relax, cycle=cycle, max_iter=3, tol=-1.0, storage=storage,
                   sync_every=3)
    ub, hb, ib, sb = run_batch(gpu, probs, p)
    for i, prob in enumerate(probs):
        us, hs, n, rc = run_single(gpu, prob, p)
        assert same(ub[i], us), (i, prob[0].nx)
        assert ib[i] == n == 3
        assert close_hist(hb[i], hs), (i, hb[i], hs)


def test_batch_retirement(gpu):
    """Stable coarse CFL, tolerance 1e-10: problems converge after different
    numbers of cycles; each one's iterate, history and count equal its own
    solve, and converged problems stop changing."""
    nxs = [64, 128, 200, 256, 512, 300]
    m = 4
    probs = mixed_problems(gpu, nxs, 0.8 / m, m, 11)
    p = gpu.params(0, 0.0, m, 2, relax=1, max_iter=40, tol=1e-10, storage=0, sync_every=1)
    ub, hb, ib, sb = run_batch(gpu, probs, p)
    assert all(st == gpu.MGRIT_OK for st in sb)
    assert len(set(ib)) > 1
    for i, prob in enumerate(probs):
        us, hs, n, rc = run_single(gpu, prob, p)
        assert rc == gpu.MGRIT_OK and ib[i] == n
        assert np.array_equal(ub[i], us)
        assert close_hist(hb[i], hs), (i, hb[i], hs)


def test_w3_full_size(orc, gpu):
    """All 512 problems, one cycle (C-point storage).  Against the oracle, on
    the 16 smallest and the 2 largest problems: r_0, and the C-points that one
    FCF cycle makes exact (nodes m and 2m equal serial stepping).  Beyond them
    the coarse CFL (8 x 0.3..0.9) amplifies round-off by about an order of
    magnitude per chunk in any implementation, so the rest of the iterate is
    compared bitwise against each problem's own solve instead (every 64th
    problem and the 2 largest)."""
    import torch

    pbs = W.w3_batched()
    p = gpu.params(0, 0.0, 8, 2, relax=1, max_iter=1, tol=-1.0, storage=1, sync_every=1)
    table, us = [], []
    for pb in pbs:
        u = torch.zeros((pb.nt // 8 + 1, pb.nx), dtype=torch.float64, device="cuda")
        us.append(u)
        table.append((gpu.scheme_from_problem(pb), pb.nt, pb.dt, T(pb.u0), u))
    hs, its, sts = gpu.cycle_batched(table, p)
    assert all(n == 1 for n in its)
    order = np.argsort([pb.nx for pb in pbs], kind="stable")
    for idx in list(order[:16]) + list(order[-2:]):
        pb = pbs[idx]
        so = orc.scheme(pb.nx, flux=pb.flux, a=pb.a)
        x = pb.u0[None, :]
        for _ in range(7):
            x = orc.phi(so, pb.dt, x)
        t = orc.phi(so, pb.dt, x)[0]
        r0 = np.sqrt(pb.nt // 8) * np.linalg.norm(t - pb.u0)
        assert abs(hs[idx][0] - r0) < 1e-12 * r0, (idx, pb.nx)
        ref = orc.serial(so, pb.dt, 16, pb.u0)
        u = H(us[idx][:3])
        assert np.all(rel_lines(u, ref[::8]) < 1e-12), (idx, pb.nx)
    for idx in list(range(0, len(pbs), 64)) + list(order[-2:]):
        pb = pbs[idx]
        prob = (gpu.scheme_from_problem(pb), pb.nt, pb.dt, pb.u0)
        u1, h1, n1, rc1 = run_single(gpu, prob, p)
        assert same(H(us[idx]), u1), (idx, pb.nx)
        assert close_hist(hs[idx], h1), (idx, hs[idx], h1)
    del us
    torch.cuda.empty_cache()


@pytest.mark.parametrize("levels,relax", [(2, 1), (3, 0)])
def test_batch_weno7_split_lines(gpu, levels, relax):
    """WENO7 (four ghost cells per tile side) in batches with split lines of
    both fluxes: every problem bitwise equal to its own solve."""
    nxs = [300, 4098, 6002, 8192, 1000]
    m = 4
    g = np.random.default_rng(40 + levels)
    probs = []
    for i, nx in enumerate(nxs):
        flux = i % 2
        a = float(g.uniform(0.5, 1.5)) if flux == 1 else 1.0
        u0 = W.random_lines(500 + i, 1, nx)[0]
        speed = np.max(np.abs(u0)) if flux == 0 else a
        nt = 8 * m
        probs.append((gpu.scheme(nx, flux=flux, a=a, k=3), nt, 0.5 / nx / speed, u0))
    p = gpu.params(0, 0.0, m, levels, relax=relax, max_iter=2, tol=-1.0, storage=0, sync_every=2)
    ub, hb, ib, sb = run_batch(gpu, probs, p)
    for i, prob in enumerate(probs):
        us, hs, n, rc = run_single(gpu, prob, p)
        assert same(ub[i], us), (i, prob[0].nx)
        assert close_hist(hb[i], hs), (i, hb[i], hs)


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("levels,relax,cycle", [(2, 1, 0), (3, 1, 0), (3, 0, 1)])
def test_batch_wide_lines(gpu, storage, levels, relax, cycle):
    """Lines of 4097..8192 cells that are multiples of 4 run the batch's
    many-chunk phases on one workgroup per line (several cell blocks per
    thread), their own solves on split lines: every iterate bitwise equal,
    residual histories to round-off (partials grouped per line instead of
    per tile); mixed with split and one-workgroup lines, both fluxes."""
    nxs = [5000, 8192, 4100, 6002, 1000, 7996]
    m = 4
    probs = mixed_problems(gpu, nxs, 0.6, m, 30 + levels + storage)
    p = gpu.params(0, 0.0, m, levels, relax=relax, cycle=cycle, max_iter=3, tol=-1.0, storage=storage,
                   sync_every=3)
    ub, hb, ib, sb = run_batch(gpu, probs, p)
    for i, prob in enumerate(probs):
        us, hs, n, rc = run_single(gpu, prob, p)
        assert same(ub[i], us), (i, prob[0].nx)
        assert ib[i] == n == 3
        assert close_hist(hb[i], hs), (i, hb[i], hs)


def test_batch_scheduled_serial_solves(gpu):
    """72 problems of 4098..4240 cells (split lines) with uneven step counts:
    their serial coarse solves share one persistent launch of 4 tiles per
    problem, one 1024-thread workgroup per compute unit, so 256 compute units
    hold 64 line groups and the 72 solves go to the groups by the greedy
    longest-first schedule.  Every iterate bitwise equal to the problem's
    own solve."""
    import torch

    m, n = 8, 72
    assert torch.cuda.get_device_properties(0).multi_processor_count // 4 < n
    g = np.random.default_rng(91)
    probs = []
    for i in range(n):
        nx = 4098 + 2 * i
        flux = i % 2
        a = float(g.uniform(0.5, 1.5)) if flux == 1 else 1.0
        u0 = W.random_lines(9100 + i, 1, nx)[0]
        speed = np.max(np.abs(u0)) if flux == 0 else a
        nt = m * (4 + (7 * i) % 13)
        probs.append((gpu.scheme(nx, flux=flux, a=a), nt, 0.6 / nx / speed, u0))
    p = gpu.params(0, 0.0, m, 2, relax=1, max_iter=2, tol=-1.0, storage=0, sync_every=2)
    ub, hb, ib, sb = run_batch(gpu, probs, p)
    for i, prob in enumerate(probs):
        us, hs, k, rc = run_single(gpu, prob, p)
        assert same(ub[i], us), (i, prob[0].nx)
        assert ib[i] == k == 2
        assert close_hist(hb[i], hs), (i, hb[i], hs)
