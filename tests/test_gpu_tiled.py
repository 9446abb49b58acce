"""GPU parity of split lines (one line over several workgroups, one global
synchronisation per Runge-Kutta stage): bitwise equal to one workgroup per
line for every entry point, oracle parity for lines longer than one
workgroup holds, and the 65536-cell workload (N_T = 16384, m = 16, 4 levels)
at full size, sampled."""
import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
TILED = [(1, 4), (2, 4), (2, 8), (4, 4), (4, 8), (16, 8)]


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_09404_amd import mgrit

    mgrit.load()
    return mgrit


@pytest.fixture
def tiled(gpu):
    yield gpu
    gpu.clear_tiled_config()


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


def lines_for(nx, nlines, seed):
    return np.concatenate([W.random_lines(seed, nlines // 2, nx), W.shock_lines(seed, nlines - nlines // 2, nx)])


def expected_tiles(nx, cfg):
    t = 64 * cfg[0] * cfg[1]
    return (nx + t - 1) // t


def phi_both(gpu, s, dt, u, nx, cfg):
    out1 = T(np.zeros_like(u))
    gpu.phi(s, dt, T(u), out1)
    gpu.set_tiled_config(nx, nx, *cfg)
    assert gpu.tiled_config(nx) == (cfg[0], cfg[1], expected_tiles(nx, cfg))
    out2 = T(np.zeros_like(u))
    gpu.phi(s, dt, T(u), out2)
    gpu.clear_tiled_config()
    return H(out1), H(out2)


@pytest.mark.parametrize("cfg", TILED)
@pytest.mark.parametrize("nx", [300, 1000, 1024, 4096])
@pytest.mark.parametrize("k,stepper,flux", [(2, 3, 0), (0, 1, 0), (2, 2, 1), (2, 1, 1)])
def test_phi_split_is_bitwise(tiled, nx, cfg, k, stepper, flux):
    """Tiles of 256..2048 cells, balanced and ragged, including one tile
    (its own neighbour on both sides)."""
    u = lines_for(nx, 6, nx + 3 * k + stepper)
    a = 0.9
    s = tiled.scheme(nx, flux=flux, k=k, stepper=stepper, a=a)
    dt = 0.6 / nx / (np.max(np.abs(u)) if flux == 0 else a)
    one, split = phi_both(tiled, s, dt, u, nx, cfg)
    assert np.array_equal(one, split)


def test_serial_split_is_bitwise(tiled):
    nx, nt = 1000, 120
    u0 = W.random_lines(31, 1, nx)[0]
    s = tiled.scheme(nx)
    dt = 0.8 / nx / np.max(np.abs(u0))
    a = T(np.zeros((nt + 1, nx)))
    tiled.serial(s, dt, nt, T(u0), a)
    tiled.set_tiled_config(nx, nx, 1, 4)
    b = T(np.zeros((nt + 1, nx)))
    tiled.serial(s, dt, nt, T(u0), b)
    assert np.array_equal(H(a), H(b))


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("with_g", [False, True])
def test_relax_split_is_bitwise(tiled, kind, with_g):
    nx, m, n = 1000, 8, 64
    g0 = np.random.default_rng(5)
    u = np.concatenate([W.random_lines(40 + kind, n + 1, nx)])
    g = 1e-3 * g0.standard_normal((n + 1, nx)) if with_g else None
    s = tiled.scheme(nx)
    dt = 0.5 / nx / np.max(np.abs(u))
    a = T(u)
    tiled.relax(s, dt, m, kind, a, T(g) if g is not None else None, n)
    tiled.set_tiled_config(nx, nx, 2, 4)
    b = T(u)
    tiled.relax(s, dt, m, kind, b, T(g) if g is not None else None, n)
    assert np.array_equal(H(a), H(b))


@pytest.mark.parametrize("coarse_guess", [0, 1])
def test_residual_split_is_bitwise(tiled, coarse_guess):
    nx, m, n = 1000, 8, 64
    u = W.random_lines(50, n + 1, nx)
    g = 1e-3 * np.random.default_rng(6).standard_normal((n + 1, nx))
    s = tiled.scheme(nx)
    dt = 0.5 / nx / np.max(np.abs(u))
    nc = n // m

    def run():
        r, uc, gc, nrm = (T(np.zeros((nc, nx))), T(np.zeros((nc + 1, nx))), T(np.zeros((nc + 1, nx))),
                          T(np.zeros(1)))
        tiled.residual(s, dt, m, T(u), T(g), n, coarse_guess=coarse_guess, r=r, u_coarse=uc, g_coarse=gc,
                       norm=nrm)
        return [H(x) for x in (r, uc, gc, nrm)]

    a = run()
    tiled.set_tiled_config(nx, nx, 4, 4)
    b = run()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("relax,cycle", [(1, 0), (0, 0), (1, 1)])
def test_cycle_split_is_bitwise(orc, tiled, relax, cycle):
    """Fixed number of cycles (3 levels), split vs one workgroup per line:
    iterates bitwise equal and equal to the oracle; the residual norms sum
    per-tile partials, a different order, so they agree to round-off."""
    nx, nt, m, levels = 1000, 64, 4, 3
    u0 = W.random_lines(61, 1, nx)[0]
    dt = 0.8 / m ** (levels - 1) / nx / np.max(np.abs(u0))
    s = tiled.scheme(nx)
    p = tiled.params(nt, dt, m, levels, relax=relax, cycle=cycle, max_iter=3, tol=-1.0)

    def run():
        ug = T(np.zeros((nt + 1, nx)))
        rc, hist, n = tiled.cycle(s, p, T(u0), ug)
        return H(ug), np.array(hist)

    ua, ha = run()
    tiled.set_tiled_config(nx, nx, 1, 4)
    ub, hb = run()
    assert np.array_equal(ua, ub)
    np.testing.assert_allclose(hb, ha, rtol=1e-13, atol=0)
    so = orc.scheme(nx)
    po = orc.params(nt, dt, m, levels, relax=relax, cycle=cycle, max_iter=3, tol=-1.0)
    uo, ho, no, sto = orc.mgrit(so, po, u0)
    assert np.all(rel_lines(ub, uo) < TOL)


@pytest.mark.parametrize("cfg", [(1, 4), (2, 8)])
def test_cycle_weno7_split_is_bitwise(orc, tiled, cfg):
    """WENO7 (four ghost cells per tile side): two FCF V-cycles on 3 levels,
    split vs one workgroup per line bitwise, and equal to the oracle."""
    nx, nt, m, levels = 1000, 64, 4, 3
    u0 = W.shock_lines(62, 1, nx)[0]
    dt = 0.8 / m ** (levels - 1) / nx / np.max(np.abs(u0))
    s = tiled.scheme(nx, k=3)
    p = tiled.params(nt, dt, m, levels, relax=1, max_iter=2, tol=-1.0)

    def run():
        ug = T(np.zeros((nt + 1, nx)))
        tiled.cycle(s, p, T(u0), ug)
        return H(ug)

    ua = run()
    tiled.set_tiled_config(nx, nx, *cfg)
    ub = run()
    assert np.array_equal(ua, ub)
    uo, ho, no, sto = orc.mgrit(orc.scheme(nx, k=3), orc.params(nt, dt, m, levels, relax=1, max_iter=2, tol=-1.0),
                                u0)
    assert np.all(rel_lines(ub, uo) < TOL)


def test_cycle_weno7_long_line_vs_oracle(orc, gpu):
    """A 6002-cell WENO7 line on its default split: one FCF V-cycle against
    the oracle."""
    nx, nt, m, levels = 6002, 32, 4, 2
    assert gpu.tiled_config(nx)[2] >= 2
    u0 = W.random_lines(63, 1, nx)[0]
    dt = 0.8 / m / nx / np.max(np.abs(u0))
    p = gpu.params(nt, dt, m, levels, relax=1, max_iter=1, tol=-1.0)
    ug = T(np.zeros((nt + 1, nx)))
    gpu.cycle(gpu.scheme(nx, k=3), p, T(u0), ug)
    uo, ho, no, sto = orc.mgrit(orc.scheme(nx, k=3), orc.params(nt, dt, m, levels, relax=1, max_iter=1, tol=-1.0),
                                u0)
    assert np.all(rel_lines(H(ug), uo) < TOL)


@pytest.mark.parametrize("k,numflux", [(2, 0), (2, 1), (3, 0), (0, 0)])
def test_wide_tiles_bitwise(tiled, k, numflux):
    """A 32768-cell line on its default 4 tiles of 8192 cells (16 per thread)
    against 8 tiles of 4096 (4 per thread): Phi and relaxation bitwise equal."""
    nx, m, n = 32768, 4, 16
    assert tiled.tiled_config(nx) == (16, 8, 4)
    u = W.random_lines(80 + k, n + 1, nx)
    s = tiled.scheme(nx, k=k, numflux=numflux)
    dt = 0.6 / nx / np.max(np.abs(u))

    def run():
        a = T(u)
        tiled.relax(s, dt, m, 2, a, None, n)
        out = T(np.zeros((2, nx)))
        tiled.phi(s, dt, T(u[:2]), out)
        return H(a), H(out)

    ra = run()
    tiled.set_tiled_config(nx, nx, 4, 16)
    assert tiled.tiled_config(nx) == (4, 16, 8)
    rb = run()
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("k", [2, 3])
def test_latency_tiles_bitwise(tiled, k):
    """Launches of few chunks that form no residual take 1024-cell tiles
    (16 per 16384-cell line instead of 4): serial stepping, Phi, relaxation
    and a two-level cycle (whose residual sweeps keep the default tiles)
    bitwise equal to every launch on the default tiles."""
    nx, m, n, nt = 16384, 4, 16, 64
    assert tiled.tiled_launch_config(nx, 1) == (2, 8, 16)
    assert tiled.tiled_launch_config(nx, 16, residual=True) == (4, 16, 4)
    u = W.random_lines(90 + k, n + 1, nx)
    s = tiled.scheme(nx, k=k)
    dt = 0.6 / nx / np.max(np.abs(u))
    p = tiled.params(nt, dt, m, 2, relax=1, max_iter=3, tol=-1.0)

    def run():
        traj = T(np.zeros((nt + 1, nx)))
        tiled.serial(s, dt, nt, T(u[0]), traj)
        a = T(u)
        tiled.relax(s, dt, m, 2, a, None, n)
        out = T(np.zeros((2, nx)))
        tiled.phi(s, dt, T(u[:2]), out)
        ug = T(np.zeros((nt + 1, nx)))
        _, hist, _ = tiled.cycle(s, p, T(u[0]), ug)
        return H(traj), H(a), H(out), H(ug), np.array(hist)

    ra = run()
    tiled.set_tiled_config(nx, nx, 4, 16)
    assert tiled.tiled_launch_config(nx, 1) == (4, 16, 4)
    rb = run()
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y, equal_nan=True)


def test_many_line_groups_twice(tiled):
    """512 chunks of 1024 cells on 2 tiles each, so that hundreds of line
    groups are resident at once, launched twice in a row (every group's
    counter must start from zero at every launch): F- and FCF-relaxation
    bitwise equal to one workgroup per line."""
    nx, m, n = 1024, 8, 4096
    u = W.random_lines(70, n + 1, nx)
    s = tiled.scheme(nx)
    dt = 0.8 / nx / np.max(np.abs(u))
    for kind in (0, 2):
        ref = T(u)
        tiled.relax(s, dt, m, kind, ref, None, n)
        ref = H(ref)
        tiled.set_tiled_config(nx, nx, 2, 4)
        for _ in range(2):
            got = T(u)
            tiled.relax(s, dt, m, kind, got, None, n)
            assert np.array_equal(H(got), ref)
        tiled.clear_tiled_config()


def test_benchmark_cycle_split_is_bitwise(tiled):
    """Two V-cycles of the 1024-cell benchmark workload with every sweep on
    split lines equal the one-workgroup cycles bitwise."""
    pb = W.w1_burgers_weno5()
    s = tiled.scheme_from_problem(pb)
    p = tiled.params(pb.nt, pb.dt, pb.m, pb.levels, relax=1, max_iter=2, tol=-1.0)

    def run():
        ug = T(np.zeros((pb.nt + 1, pb.nx)))
        tiled.cycle(s, p, T(pb.u0), ug)
        return H(ug)

    a = run()
    tiled.set_tiled_config(pb.nx, pb.nx, 4, 4)
    b = run()
    with np.errstate(invalid="ignore"):
        same = (a == b) | (np.isnan(a) & np.isnan(b))
    assert np.all(same)


# ---------------------------------------------------------------------------
# lines longer than one workgroup holds (default split)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nx", [4098, 6002, 8192, 65536])
@pytest.mark.parametrize("k,stepper,flux", [(2, 3, 0), (2, 3, 1), (0, 1, 0), (3, 3, 0), (3, 2, 1)])
def test_phi_long_lines_vs_oracle(orc, gpu, nx, k, stepper, flux):
    cpt, waves, tiles = gpu.tiled_config(nx)
    assert tiles >= 2
    u = lines_for(nx, 4, nx + k + flux)
    a = 1.1
    so = orc.scheme(nx, flux=flux, k=k, stepper=stepper, a=a)
    sg = gpu.scheme(nx, flux=flux, k=k, stepper=stepper, a=a)
    dt = 0.6 / nx / (np.max(np.abs(u)) if flux == 0 else a)
    out = T(np.zeros_like(u))
    gpu.phi(sg, dt, T(u), out)
    assert np.all(rel_lines(H(out), orc.phi(so, dt, u)) < TOL)


def test_serial_long_line_vs_oracle(orc, gpu):
    nx, nt = 65536, 24
    u0 = W.fourier_data(W.rng(2), nx, 16, 64)
    dt = 0.8 / nx / np.max(np.abs(u0))
    traj = T(np.zeros((nt + 1, nx)))
    gpu.serial(gpu.scheme(nx), dt, nt, T(u0), traj)
    ref = orc.serial(orc.scheme(nx), dt, nt, u0)
    assert np.all(rel_lines(H(traj), ref) < TOL)


def test_w2_full_size_sampled(orc, gpu):
    """The 65536-cell workload (N_T = 16384, m = 16, 4-level FCF V-cycle), one
    cycle at full size on split lines: r_0 equals the oracle's, the first two
    chunks of the iterate equal serial stepping, sampled chunks conserve mass."""
    import torch

    pb = W.w2_burgers_weno5_large()
    m = pb.m
    so = orc.scheme(pb.nx)
    sg = gpu.scheme_from_problem(pb)
    p = gpu.params(pb.nt, pb.dt, m, pb.levels, relax=1, max_iter=1, tol=-1.0)
    ug = torch.zeros((pb.nt + 1, pb.nx), dtype=torch.float64, device="cuda")
    rc, hist, n = gpu.cycle(sg, p, T(pb.u0), ug)
    x = pb.u0[None, :]
    for _ in range(m - 1):
        x = orc.phi(so, pb.dt, x)
    t = orc.phi(so, pb.dt, x)[0]
    r0 = np.sqrt(pb.nt // m) * np.linalg.norm(t - pb.u0)
    assert abs(hist[0] - r0) < 1e-12 * r0
    us = orc.serial(so, pb.dt, 2 * m, pb.u0)
    head = H(ug[: 2 * m + 1])
    assert np.all(rel_lines(head, us) < TOL)
    # every chunk that stayed bounded (coarse CFLs 12.8 / 205 / 3277 make most
    # of the iterate blow up, as the paper finds) conserves mass across its F-points
    sums = H(ug.sum(dim=1))
    amax = H(torch.nan_to_num(ug.abs(), nan=np.inf).amax(dim=1))
    checked = 0
    for c in range(pb.nt // m):
        blk = slice(c * m, (c + 1) * m)
        if np.all(amax[blk] < 10.0):
            assert np.max(np.abs(sums[blk] - sums[c * m])) < 1e-9 * max(1.0, abs(sums[c * m]))
            checked += 1
    assert checked >= 2
    del ug
    torch.cuda.empty_cache()


def test_w2_stable_coarse_converges_to_serial(orc, gpu):
    """The 65536-cell problem with the benchmark's N_T = 16384 and m = 16, on
    3 levels with a step that puts the coarsest level at CFL 0.8: FCF
    V-cycles reach a residual of 1e-10 within 4 cycles, and the iterate equals
    serial stepping of the same problem (MGRIT's fixed point) to round-off;
    the first steps of both equal the oracle's serial stepping."""
    import torch

    pb = W.w2_stable_coarse()
    sg = gpu.scheme_from_problem(pb)
    p = gpu.params(pb.nt, pb.dt, pb.m, pb.levels, relax=1, max_iter=8, tol=1e-10)
    ug = torch.zeros((pb.nt + 1, pb.nx), dtype=torch.float64, device="cuda")
    rc, hist, n = gpu.cycle(sg, p, T(pb.u0), ug)
    assert rc == 0 and n <= 4 and hist[-1] <= 1e-10, (rc, n, hist)
    traj = torch.empty_like(ug)
    gpu.serial(sg, pb.dt, pb.nt, T(pb.u0), traj)
    diff = float((ug - traj).abs().max())
    assert diff < 1e-11 * float(traj.abs().max()), diff
    us = orc.serial(orc.scheme(pb.nx), pb.dt, 2 * pb.m, pb.u0)
    assert np.all(rel_lines(H(ug[: 2 * pb.m + 1]), us) < TOL)
    del ug, traj
    torch.cuda.empty_cache()
