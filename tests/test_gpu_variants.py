"""GPU parity of the scheme variants against the oracle: WENO of degree
k = 1, 3 (s = 3, 7; tables from eq C, B, D), the Roe flux with the
Harten-Hyman fix (sec 2.1.3, eq roeflux), on one workgroup per line, on
split lines and in batches; MGRIT with a scheme per level (Fig.
MGRITweno_diffOrd); the paper's high-order experiments (Fig. MGRITweno,
MGRITcfl) at their own sizes.  Bar: 1e-12 relative L2 per line; bitwise
where the same kernels run in another arrangement."""
import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
K_OF_S = {1: 0, 3: 1, 5: 2, 7: 3}


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


def schemes(orc, gpu, nx, **kw):
    return orc.scheme(nx, **kw), gpu.scheme(nx, **kw)


def same(a, b):
    with np.errstate(invalid="ignore"):
        return bool(np.all((a == b) | (np.isnan(a) & np.isnan(b))))


# ---------------------------------------------------------------------------
# Phi on independent lines
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nx", [8, 13, 64, 257, 1000, 2050, 4096])
@pytest.mark.parametrize("k,numflux", [(1, 0), (3, 0), (0, 1), (1, 1), (2, 1), (3, 1)])
@pytest.mark.parametrize("flux", [0, 1])
def test_phi_parity(orc, gpu, nx, k, numflux, flux):
    """Every one-workgroup configuration from one wave to 8 cells x 8 waves,
    ragged and not, SSPRK3."""
    u = lines_for(nx, 6, nx + 7 * k + numflux)
    a = -0.8
    so, sg = schemes(orc, gpu, nx, flux=flux, k=k, stepper=3, a=a, numflux=numflux)
    dt = 0.6 / nx / (np.max(np.abs(u)) if flux == 0 else abs(a))
    out = T(np.zeros_like(u))
    gpu.phi(sg, dt, T(u), out)
    assert np.all(rel_lines(H(out), orc.phi(so, dt, u)) < TOL)


@pytest.mark.parametrize("k,numflux", [(1, 0), (3, 1), (2, 1)])
@pytest.mark.parametrize("stepper", [1, 2])
def test_phi_parity_steppers(orc, gpu, k, numflux, stepper):
    nx = 300
    u = lines_for(nx, 4, 11 + stepper)
    so, sg = schemes(orc, gpu, nx, k=k, stepper=stepper, numflux=numflux)
    dt = 0.3 / nx / np.max(np.abs(u))
    out = T(np.zeros_like(u))
    gpu.phi(sg, dt, T(u), out)
    assert np.all(rel_lines(H(out), orc.phi(so, dt, u)) < TOL)


def test_roe_opens_transonic_rarefaction(gpu):
    """-1 | +1: the cells beside the jump move by dt/(2 dx) after one
    first-order step (the flux through a transonic rarefaction is 0)."""
    nx = 64
    u = np.where(np.arange(nx) < nx // 2, -1.0, 1.0)[None, :]
    dt = 0.2 / nx
    out = T(np.zeros_like(u))
    gpu.phi(gpu.scheme(nx, k=0, stepper=1, numflux=1), dt, T(u), out)
    o = H(out)[0]
    j = nx // 2
    assert abs(o[j - 1] - (-1.0 + 0.5 * dt * nx)) < 1e-15
    assert abs(o[j] - (1.0 - 0.5 * dt * nx)) < 1e-15


@pytest.mark.parametrize("k,numflux", [(3, 0), (1, 1), (3, 1)])
def test_serial_parity(orc, gpu, k, numflux):
    nx, nt = 1000, 80
    u0 = W.shock_lines(21, 1, nx)[0]
    so, sg = schemes(orc, gpu, nx, k=k, numflux=numflux)
    dt = 0.7 / nx / np.max(np.abs(u0))
    traj = T(np.zeros((nt + 1, nx)))
    gpu.serial(sg, dt, nt, T(u0), traj)
    assert np.all(rel_lines(H(traj), orc.serial(so, dt, nt, u0)) < TOL)


# ---------------------------------------------------------------------------
# split lines
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfg", [(1, 4), (2, 4), (4, 8)])
@pytest.mark.parametrize("nx", [300, 1000, 4096])
@pytest.mark.parametrize(
    "k,numflux,flux", [(1, 0, 0), (1, 1, 0), (2, 1, 0), (0, 1, 1), (2, 1, 1), (3, 0, 0), (3, 1, 0), (3, 0, 1)]
)
def test_split_phi_is_bitwise(tiled, nx, cfg, k, numflux, flux):
    u = lines_for(nx, 4, nx + k + 3 * numflux)
    a = 0.9
    s = tiled.scheme(nx, flux=flux, k=k, a=a, numflux=numflux)
    dt = 0.6 / nx / (np.max(np.abs(u)) if flux == 0 else a)
    one = T(np.zeros_like(u))
    tiled.phi(s, dt, T(u), one)
    tiled.set_tiled_config(nx, nx, *cfg)
    two = T(np.zeros_like(u))
    tiled.phi(s, dt, T(u), two)
    assert np.array_equal(H(one), H(two))


@pytest.mark.parametrize("nx", [4098, 6002])
@pytest.mark.parametrize("k,numflux", [(1, 0), (1, 1), (2, 1), (3, 0), (3, 1)])
def test_long_lines_vs_oracle(orc, gpu, nx, k, numflux):
    assert gpu.tiled_config(nx)[2] >= 2
    u = lines_for(nx, 2, 5 + k)
    so, sg = schemes(orc, gpu, nx, k=k, numflux=numflux)
    dt = 0.6 / nx / np.max(np.abs(u))
    out = T(np.zeros_like(u))
    gpu.phi(sg, dt, T(u), out)
    assert np.all(rel_lines(H(out), orc.phi(so, dt, u)) < TOL)


def test_unsupported_combinations(tiled):
    """Any of the new schemes in the adjoint, Roe with a fixed LF coefficient:
    rejected on the host before any launch."""
    w = T(np.zeros((1, 256)))
    for s in (tiled.scheme(256, k=1), tiled.scheme(256, numflux=1), tiled.scheme(256, k=3)):
        with pytest.raises(tiled.MgritError):
            tiled.phi_vjp(s, 1e-4, w, w, w)
    with pytest.raises(tiled.MgritError):
        tiled.phi(tiled.scheme(256, numflux=1, alpha_fixed=1.0), 1e-4, w, w)


# ---------------------------------------------------------------------------
# MGRIT: the paper's high-order experiments
# ---------------------------------------------------------------------------
def gpu_iterates(gpu, schemes_g, pb, iters, levels=None):
    levels = levels or pb.levels
    p = gpu.params(pb.nt, pb.dt, pb.m, levels, relax=pb.relax, max_iter=iters, tol=-1.0)
    u = T(np.zeros((pb.nt + 1, pb.nx)))
    if len(set(id(s) for s in schemes_g)) == 1:
        rc, hist, n = gpu.cycle(schemes_g[0], p, T(pb.u0), u)
    else:
        rc, hist, n = gpu.cycle_levels(schemes_g, p, T(pb.u0), u)
    return H(u), np.array(hist)


@pytest.mark.parametrize("s_", [1, 3, 5, 7])
@pytest.mark.parametrize("numflux", [0, 1])
def test_high_order_experiment_parity(orc, gpu, s_, numflux):
    """Fig. MGRITweno (Burgers, N_x = 64, N_T = 400, 3-level V-cycle, m = 2,
    F-relaxation): 4 cycles on the GPU equal the oracle's iterates and
    residual history."""
    k = K_OF_S[s_]
    pb = W.e4_high_order(k, numflux)
    so, sg = schemes(orc, gpu, pb.nx, k=k, stepper=3, numflux=numflux)
    ug, hg = gpu_iterates(gpu, [sg] * 3, pb, 4)
    po = orc.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, max_iter=4, tol=-1.0)
    uo, ho, no, _ = orc.mgrit(so, po, pb.u0)
    assert np.all(rel_lines(ug, uo) < TOL)
    np.testing.assert_allclose(hg, ho, rtol=1e-10, atol=1e-13 * np.linalg.norm(pb.u0) * np.sqrt(pb.nt))


LEVEL_CASES = [
    ("decreasing s", [5, 3, 1], [3, 3, 3]),
    ("decreasing s and d", [5, 3, 1], [3, 2, 1]),
    ("increasing s", [1, 3, 5], [3, 3, 3]),
    ("s = 7 on the fine level", [7, 5, 3], [3, 3, 2]),
]


@pytest.mark.parametrize("name,ss,ds", LEVEL_CASES, ids=[c[0] for c in LEVEL_CASES])
@pytest.mark.parametrize("numflux", [0, 1])
def test_scheme_per_level_parity(orc, gpu, name, ss, ds, numflux):
    """Fig. MGRITweno_diffOrd: s (and the RK order d) changing across levels;
    3 cycles of mgrit_cycle_levels equal the oracle's."""
    pb = W.e4_high_order(K_OF_S[ss[0]], numflux)
    so = [orc.scheme(pb.nx, k=K_OF_S[a], stepper=d, numflux=numflux) for a, d in zip(ss, ds)]
    sg = [gpu.scheme(pb.nx, k=K_OF_S[a], stepper=d, numflux=numflux) for a, d in zip(ss, ds)]
    ug, hg = gpu_iterates(gpu, sg, pb, 3)
    po = orc.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, max_iter=3, tol=-1.0)
    uo, ho, _, _ = orc.mgrit_levels(so, po, pb.u0)
    assert np.all(rel_lines(ug, uo) < TOL)
    np.testing.assert_allclose(hg, ho, rtol=1e-10)


@pytest.mark.parametrize("relax,cycle", [(0, 0), (1, 0), (1, 1)])
def test_scheme_per_level_same_scheme_is_mgrit_cycle(gpu, relax, cycle):
    """One scheme on every level, passed as separate entries: bitwise the
    solve of mgrit_cycle (the restriction then stays fused)."""
    pb = W.e4_high_order(2, 1)
    s = gpu.scheme(pb.nx, k=2, stepper=3, numflux=1)
    p = gpu.params(pb.nt, pb.dt, pb.m, 4, relax=relax, cycle=cycle, max_iter=3, tol=-1.0)
    a = T(np.zeros((pb.nt + 1, pb.nx)))
    b = T(np.zeros((pb.nt + 1, pb.nx)))
    ra, ha, na = gpu.cycle(s, p, T(pb.u0), a)
    copies = [gpu.scheme(pb.nx, k=2, stepper=3, numflux=1) for _ in range(4)]
    rb, hb, nb = gpu.cycle_levels(copies, p, T(pb.u0), b)
    assert same(H(a), H(b)) and ha == hb and na == nb


def test_scheme_per_level_fcf_fcycle_parity(orc, gpu):
    """FCF-relaxation and the F-cycle with a scheme per level (4 levels)."""
    pb = W.e4_high_order(2, 0)
    ks, ds = [2, 1, 1, 0], [3, 3, 2, 1]
    so = [orc.scheme(pb.nx, k=k, stepper=d) for k, d in zip(ks, ds)]
    sg = [gpu.scheme(pb.nx, k=k, stepper=d) for k, d in zip(ks, ds)]
    for relax, cycle in ((1, 0), (1, 1), (0, 1)):
        p = gpu.params(pb.nt, pb.dt, pb.m, 4, relax=relax, cycle=cycle, max_iter=2, tol=-1.0)
        u = T(np.zeros((pb.nt + 1, pb.nx)))
        gpu.cycle_levels(sg, p, T(pb.u0), u)
        po = orc.params(pb.nt, pb.dt, pb.m, 4, relax=relax, cycle=cycle, max_iter=2, tol=-1.0)
        uo, _, _, _ = orc.mgrit_levels(so, po, pb.u0)
        assert np.all(rel_lines(H(u), uo) < TOL), (relax, cycle)


def test_scheme_per_level_rejects_split_lines_and_mismatch(gpu):
    nx = 8192
    p = gpu.params(256, 1e-5, 4, 2, max_iter=1, tol=-1.0)
    u = T(np.zeros((257, nx)))
    with pytest.raises(gpu.MgritError):
        gpu.cycle_levels([gpu.scheme(nx), gpu.scheme(nx, k=1)], p, T(np.zeros(nx)), u)
    v = T(np.zeros((257, 64)))
    with pytest.raises(gpu.MgritError):
        gpu.cycle_levels([gpu.scheme(64), gpu.scheme(64, flux=1)], p, T(np.zeros(64)), v)


def cfl_problem(k, stepper, nt):
    nx, T_end = 128, 0.475
    return W.Problem("e3", 0, k, stepper, nx, nt, T_end / nt, 2, 5, 0, W.cell_average_sin(nx, 1, 0.0))


@pytest.mark.parametrize("k,stepper,nt", [(0, 3, 1024), (2, 3, 1024), (2, 3, 2048)])
def test_cfl_experiment_parity(orc, gpu, k, stepper, nt):
    """Fig. MGRITcfl with the Roe flux (N_x = 128, T = 0.475, 5 levels, m = 2,
    u0 = sin 2 pi x) at the coarsest CFL numbers where MGRIT converges
    (0.95, 0.48): 3 cycles equal the oracle's iterates."""
    pb = cfl_problem(k, stepper, nt)
    so, sg = schemes(orc, gpu, pb.nx, k=k, stepper=stepper, numflux=1)
    ug, hg = gpu_iterates(gpu, [sg] * 5, pb, 3)
    po = orc.params(nt, pb.dt, 2, 5, relax=0, max_iter=3, tol=-1.0)
    uo, ho, _, _ = orc.mgrit(so, po, pb.u0)
    assert np.all(rel_lines(ug, uo) < TOL)


def test_cfl_experiment_shape_on_gpu(orc, gpu):
    """Where the coarse levels are unstable (WENO5 + FE at c = 0.95, SSPRK3 at
    c = 1.9) round-off is amplified by ~1e11 in two cycles (measured on the
    oracle with a 1e-15 perturbation), so iterates are compared through the
    experiment's findings instead: the GPU runs show the same shape as the
    oracle's (r_0 equal to 1e-12, FE diverging at c = 0.95, s = 5 far less
    converged than s = 1 at c = 1.9)."""

    def rel_err(k, stepper, nt, iters):
        pb = cfl_problem(k, stepper, nt)
        sg = gpu.scheme(pb.nx, k=k, stepper=stepper, numflux=1)
        traj = T(np.zeros((nt + 1, pb.nx)))
        gpu.serial(sg, pb.dt, nt, T(pb.u0), traj)
        us = H(traj)
        ug, hg = gpu_iterates(gpu, [sg] * 5, pb, iters)
        so = orc.scheme(pb.nx, k=k, stepper=stepper, numflux=1)
        _, ho, _, _ = orc.mgrit(so, orc.params(nt, pb.dt, 2, 5, relax=0, max_iter=0, tol=-1.0), pb.u0)
        assert abs(hg[0] - ho[0]) <= 1e-12 * ho[0]
        with np.errstate(all="ignore"):
            return np.linalg.norm(ug - us) / np.linalg.norm(us)

    fe = rel_err(2, 1, 1024, 3)
    assert not np.isfinite(fe) or fe > 1.0
    s1 = rel_err(0, 3, 512, 3)
    s5 = rel_err(2, 3, 512, 3)
    assert s5 > 1e3 * s1


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 3])
def test_batch_of_new_schemes_equals_single_solves(gpu, k):
    """A batch mixing LF and Roe, Burgers and advection problems of WENO
    degree k: iterates bitwise equal to each problem's own solve."""
    m = 4
    nxs = [64, 100, 300, 1000, 2050] + ([4098] if k == 1 else [])
    g = np.random.default_rng(50 + k)
    probs = []
    for i, nx in enumerate(nxs):
        flux, numflux = i % 2, (i // 2) % 2
        a = float(g.uniform(0.5, 1.5)) if flux else 1.0
        u0 = W.random_lines(300 + i, 1, nx)[0]
        dt = 0.6 / nx / (np.max(np.abs(u0)) if flux == 0 else a)
        nt = 4 * m * max(1, nx // (4 * m))
        probs.append((gpu.scheme(nx, flux=flux, a=a, k=k, numflux=numflux), nt, dt, u0))
    p = gpu.params(0, 0.0, m, 2, relax=1, max_iter=2, tol=-1.0, sync_every=2)
    table, us = [], []
    for sch, nt, dt, u0 in probs:
        u = T(np.zeros((nt + 1, sch.nx)))
        us.append(u)
        table.append((sch, nt, dt, T(u0), u))
    gpu.cycle_batched(table, p)
    for (sch, nt, dt, u0), ub in zip(probs, us):
        q = gpu.params(nt, dt, m, 2, relax=1, max_iter=2, tol=-1.0, sync_every=2)
        u = T(np.zeros((nt + 1, sch.nx)))
        gpu.cycle(sch, q, T(u0), u)
        assert same(H(ub), H(u)), sch.nx
