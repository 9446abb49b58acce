"""GPU parity of split lines with two chunks per workgroup (the chunks run
half a Runge-Kutta stage apart, so that one chunk's exchange with the other
tiles overlaps the other chunk's reconstruction): bitwise equal to one
workgroup per line for every entry point and role, with more chunks than
line groups (pairs plus a lone last chunk), whole-thread and ragged tiles,
every reconstruction degree of split lines, every Runge-Kutta scheme and
both fluxes."""
import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

pytestmark = pytest.mark.gpu

PAIRED = [(4, 8)]


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


def lines_for(nx, nlines, seed):
    return np.concatenate([W.random_lines(seed, nlines // 2, nx), W.shock_lines(seed, nlines - nlines // 2, nx)])


def split_paired(gpu, nx, cfg):
    gpu.set_tiled_intervals(nx, nx, cfg[0], cfg[1], 2)
    t = 64 * cfg[0] * cfg[1]
    assert gpu.tiled_config(nx) == (cfg[0], cfg[1], (nx + t - 1) // t)
    assert gpu.tiled_intervals(nx) == 2


@pytest.mark.parametrize("cfg", PAIRED)
@pytest.mark.parametrize("nx", [4096, 4100])
@pytest.mark.parametrize("k,stepper,flux,numflux", [(2, 3, 0, 0), (0, 1, 0, 0), (1, 2, 1, 0), (2, 3, 0, 1),
                                                    (2, 1, 1, 0)])
def test_phi_paired_is_bitwise(tiled, cfg, nx, k, stepper, flux, numflux):
    """301 lines: more chunks than the line groups that fit at once, so most
    groups run pairs and some end with one chunk alone."""
    u = lines_for(nx, 301, nx + 3 * k + stepper + 7 * numflux)
    a = 0.9
    s = tiled.scheme(nx, flux=flux, k=k, stepper=stepper, a=a, numflux=numflux)
    dt = 0.6 / nx / (np.max(np.abs(u)) if flux == 0 else a)
    ref = T(np.zeros_like(u))
    tiled.phi(s, dt, T(u), ref)
    split_paired(tiled, nx, cfg)
    got = T(np.zeros_like(u))
    tiled.phi(s, dt, T(u), got)
    assert np.array_equal(H(ref), H(got))


@pytest.mark.parametrize("cfg", PAIRED)
@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("with_g", [False, True])
def test_relax_paired_is_bitwise(tiled, cfg, kind, with_g):
    nx, m, n = 4096, 8, 8 * 301
    u = W.random_lines(80 + kind, n + 1, nx)
    g = 1e-3 * np.random.default_rng(7).standard_normal((n + 1, nx)) if with_g else None
    s = tiled.scheme(nx)
    dt = 0.5 / nx / np.max(np.abs(u))
    a = T(u)
    tiled.relax(s, dt, m, kind, a, T(g) if g is not None else None, n)
    split_paired(tiled, nx, cfg)
    b = T(u)
    tiled.relax(s, dt, m, kind, b, T(g) if g is not None else None, n)
    assert np.array_equal(H(a), H(b))


@pytest.mark.parametrize("cfg", PAIRED)
@pytest.mark.parametrize("coarse_guess", [0, 1])
def test_residual_paired_is_bitwise(tiled, cfg, coarse_guess):
    """C-point residual fused with the FAS restriction (the role whose last
    job steps the chunk-start line with the coarse step)."""
    nx, m, n = 4096, 8, 8 * 301
    u = W.random_lines(90, n + 1, nx)
    g = 1e-3 * np.random.default_rng(8).standard_normal((n + 1, nx))
    s = tiled.scheme(nx)
    dt = 0.5 / nx / np.max(np.abs(u))
    nc = n // m

    def run():
        r, uc, gc, nrm = (T(np.zeros((nc, nx))), T(np.zeros((nc + 1, nx))), T(np.zeros((nc + 1, nx))),
                          T(np.zeros(1)))
        tiled.residual(s, dt, m, T(u), T(g), n, coarse_guess=coarse_guess, r=r, u_coarse=uc, g_coarse=gc,
                       norm=nrm)
        return [H(x) for x in (r, uc, gc)], H(nrm)

    a, na = run()
    split_paired(tiled, nx, cfg)
    b, nb = run()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # the norm sums per-tile partials, a different order
    np.testing.assert_allclose(nb, na, rtol=1e-13)


@pytest.mark.parametrize("relax,cycle", [(1, 0), (0, 1)])
def test_cycle_paired_is_bitwise(tiled, relax, cycle):
    """Three MGRIT cycles (3 levels, m = 4) of a 4096-cell problem whose
    coarsest level runs at CFL 0.8: iterates bitwise equal to one workgroup
    per line."""
    nx, nt, m, levels = 4096, 2048, 4, 3
    u0 = W.random_lines(95, 1, nx)[0]
    dt = 0.8 / m ** (levels - 1) / nx / np.max(np.abs(u0))
    s = tiled.scheme(nx)
    p = tiled.params(nt, dt, m, levels, relax=relax, cycle=cycle, max_iter=3, tol=-1.0)

    def run():
        ug = T(np.zeros((nt + 1, nx)))
        rc, hist, n = tiled.cycle(s, p, T(u0), ug)
        return H(ug), np.array(hist)

    ua, ha = run()
    split_paired(tiled, nx, (4, 8))
    ub, hb = run()
    assert np.array_equal(ua, ub)
    np.testing.assert_allclose(hb, ha, rtol=1e-13, atol=0)
    assert hb[-1] < hb[0]


def test_paired_configuration_checks(gpu):
    """Only compiled shapes take two intervals; one or two intervals only."""
    assert gpu.load().mgrit_set_tiled_intervals(8000, 9000, 4, 8, 3) == gpu.MGRIT_EINVAL
    assert gpu.load().mgrit_set_tiled_intervals(8000, 9000, 1, 4, 2) == gpu.MGRIT_EINVAL
    assert gpu.load().mgrit_set_tiled_intervals(8000, 9000, 4, 16, 2) == gpu.MGRIT_EINVAL
    assert gpu.load().mgrit_set_tiled_intervals(8000, 9000, 1, 4, 1) == gpu.MGRIT_OK
    assert gpu.tiled_intervals(8192) == 1
    gpu.clear_tiled_config()
