"""GPU parity of systems (shallow water, Euler) on split lines: a line cut
into tiles of one workgroup each, with k + 1 ghost cells per side and one
exchange of alpha_LF and edge-face flux parts per Runge-Kutta stage.  Bitwise
equal to one workgroup per line wherever both run (every degree k = 0..3,
LF and Roe, every stepper, relaxation, residual and restriction, MGRIT
cycles), and within 1e-12 (relative L2 per line) of the oracle on lines
longer than one workgroup holds (513 to 4099 cells)."""
import numpy as np
import pytest

from test_gpu_systems import H, T, rel_lines, schemes, state_lines

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_09404_amd import mgrit

    mgrit.load()
    return mgrit


@pytest.fixture
def split(gpu):
    yield gpu
    gpu.clear_sys_tiles()


def same(a, b):
    with np.errstate(invalid="ignore"):
        return bool(np.all((a == b) | (np.isnan(a) & np.isnan(b))))


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("nx,tiles", [(64, 2), (300, 3), (500, 7), (37, 9)])
@pytest.mark.parametrize("k,numflux,stepper", [(0, 0, 1), (1, 0, 3), (2, 0, 3), (3, 0, 2), (2, 1, 3), (3, 1, 1)])
def test_split_phi_is_bitwise(split, sysname, nx, tiles, k, numflux, stepper):
    u, smax = state_lines(sysname, 4, nx, nx + 3 * k + numflux)
    s = schemes(split, split, sysname, nx, k=k, numflux=numflux, stepper=stepper)[1]
    dt = 0.5 / nx / smax
    one = T(np.zeros_like(u))
    split.phi(s, dt, T(u), one)
    split.set_sys_tiles(nx, nx, tiles)
    assert split.sys_tiles(s) == tiles
    two = T(np.zeros_like(u))
    split.phi(s, dt, T(u), two)
    assert same(H(one), H(two))


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("nx", [513, 1000, 2048, 4099])
@pytest.mark.parametrize("k,numflux", [(2, 0), (3, 0), (2, 1), (0, 1)])
def test_long_lines_vs_oracle(orc, gpu, sysname, nx, k, numflux):
    so, sg = schemes(orc, gpu, sysname, nx, k=k, numflux=numflux)
    assert gpu.sys_tiles(sg) >= 2
    u, smax = state_lines(sysname, 2, nx, nx + k)
    dt = 0.5 / nx / smax
    out = T(np.zeros_like(u))
    gpu.phi(sg, dt, T(u), out)
    assert np.all(rel_lines(H(out), orc.phi(so, dt, u)) < TOL)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_serial_long_line_and_conservation(orc, gpu, sysname):
    nx, nt = 2000, 24
    u, smax = state_lines(sysname, 2, nx, 31)
    u0 = u[1]
    so, sg = schemes(orc, gpu, sysname, nx, k=2)
    assert gpu.sys_tiles(sg) == 4
    dt = 0.5 / nx / smax
    traj = T(np.zeros((nt + 1, u0.size)))
    gpu.serial(sg, dt, nt, T(u0), traj)
    tg = H(traj)
    assert np.all(rel_lines(tg, orc.serial(so, dt, nt, u0)) < TOL)
    D = u0.size // nx
    for d in range(D):
        sums = tg[:, d * nx:(d + 1) * nx].sum(axis=1)
        assert np.max(np.abs(sums - sums[0])) < 1e-12 * nx * max(1.0, abs(sums[0]) / nx)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_relax_split_is_bitwise(split, sysname, kind):
    nx, m, n = 300, 4, 32
    u, smax = state_lines(sysname, n + 1, nx, 40 + kind)
    g = 1e-4 * np.random.default_rng(kind).standard_normal(u.shape)
    s = schemes(split, split, sysname, nx, k=3)[1]
    dt = 0.5 / nx / smax
    a = T(u)
    split.relax(s, dt, m, kind, a, T(g), n)
    split.set_sys_tiles(nx, nx, 4)
    b = T(u)
    split.relax(s, dt, m, kind, b, T(g), n)
    assert same(H(a), H(b))


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("coarse_guess", [0, 1])
def test_residual_split_is_bitwise(split, sysname, coarse_guess):
    nx, m, n = 300, 4, 32
    u, smax = state_lines(sysname, n + 1, nx, 50 + coarse_guess)
    g = 1e-4 * np.random.default_rng(6).standard_normal(u.shape)
    s = schemes(split, split, sysname, nx, k=2, numflux=1)[1]
    dt = 0.5 / nx / smax
    nc, L = n // m, u.shape[1]

    def run():
        r, uc, gc, nrm = (T(np.zeros((nc, L))), T(np.zeros((nc + 1, L))), T(np.zeros((nc + 1, L))), T(np.zeros(1)))
        split.residual(s, dt, m, T(u), T(g), n, coarse_guess=coarse_guess, r=r, u_coarse=uc, g_coarse=gc, norm=nrm)
        return [H(x) for x in (r, uc, gc, nrm)]

    a = run()
    split.set_sys_tiles(nx, nx, 3)
    b = run()
    for x, y in zip(a, b):
        assert same(x, y)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("relax,cycle", [(1, 0), (0, 1)])
def test_cycle_split_is_bitwise(orc, split, sysname, relax, cycle):
    """Two cycles on 3 levels, split (3 tiles) vs one workgroup per line:
    iterates bitwise equal and equal to the oracle; the residual norms sum
    per-tile partials, another order, so they agree to round-off."""
    nx, nt, m, levels = 240, 64, 4, 3
    u, smax = state_lines(sysname, 1, nx, 61)
    u0 = u[0]
    so, sg = schemes(orc, split, sysname, nx, k=2)
    dt = 0.5 / m ** (levels - 1) / nx / smax
    p = split.params(nt, dt, m, levels, relax=relax, cycle=cycle, max_iter=2, tol=-1.0)

    def run():
        ug = T(np.zeros((nt + 1, u0.size)))
        rc, hist, n = split.cycle(sg, p, T(u0), ug)
        return H(ug), np.array(hist)

    ua, ha = run()
    split.set_sys_tiles(nx, nx, 3)
    ub, hb = run()
    assert same(ua, ub)
    np.testing.assert_allclose(hb, ha, rtol=1e-13, atol=0)
    po = orc.params(nt, dt, m, levels, relax=relax, cycle=cycle, max_iter=2, tol=-1.0)
    uo, ho, _, _ = orc.mgrit(so, po, u0)
    assert np.all(rel_lines(ub, uo) < TOL)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_cycle_long_line_vs_oracle(orc, gpu, sysname):
    nx, nt, m, levels = 1500, 16, 4, 2
    u, smax = state_lines(sysname, 1, nx, 71)
    u0 = u[0]
    so, sg = schemes(orc, gpu, sysname, nx, k=3, numflux=1)
    assert gpu.sys_tiles(sg) == 3
    dt = 0.5 / m / nx / smax
    p = gpu.params(nt, dt, m, levels, relax=1, max_iter=1, tol=-1.0)
    ug = T(np.zeros((nt + 1, u0.size)))
    gpu.cycle(sg, p, T(u0), ug)
    po = orc.params(nt, dt, m, levels, relax=1, max_iter=1, tol=-1.0)
    uo, _, _, _ = orc.mgrit(so, po, u0)
    assert np.all(rel_lines(H(ug), uo) < TOL)


def test_split_system_rejections(split):
    """A scheme per level stays on one workgroup per line; tile settings that
    cannot split are refused."""
    nx = 600
    s1, s2 = split.euler_scheme(nx, k=2), split.euler_scheme(nx, k=1)
    p = split.params(32, 1e-5, 4, 2, relax=0, max_iter=1, tol=-1.0)
    u = T(np.zeros((33, 3 * nx)))
    with pytest.raises(split.MgritError):
        split.cycle_levels([s1, s2], p, T(np.ones(3 * nx)), u)
    with pytest.raises(split.MgritError):
        split.set_sys_tiles(100, 2000, 2)  # 1000-cell tiles
    with pytest.raises(split.MgritError):
        split.set_sys_tiles(8, 64, 4)  # 2-cell tiles at nx = 8
