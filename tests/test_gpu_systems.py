"""GPU parity of the systems (shallow water and Euler; characteristic-wise
WENO of degree 0-3, LF and Roe fluxes) against the oracle: Phi on
independent lines of every launch width, serial stepping, relaxation,
MGRIT cycles (the paper's high-order experiment for both systems, FCF and
F-cycles, a scheme per level), conservation, and the calls that do not cover
systems.  Bar: 1e-12 relative L2 per line."""
import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
GAMMA = 5.0 / 3.0


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


def schemes(orc, gpu, sysname, nx, **kw):
    if sysname == "sw":
        return orc.shallow_water_scheme(nx, **kw), gpu.shallow_water_scheme(nx, **kw)
    return orc.euler_scheme(nx, **kw), gpu.euler_scheme(nx, **kw)


def state_lines(sysname, nlines, nx, seed):
    """Physical lines: half smooth (a few modes), half with jumps; returns
    (lines [nlines, D nx], largest wave speed)."""
    g = np.random.default_rng(seed)
    out, smax = [], 0.0
    for b in range(nlines):
        if b % 2 == 0:
            m = W.random_lines(seed * 10 + b, 3, nx, mean=0.0, amp=0.6)
            a, v, c = 1.0 + m[0], 0.5 * m[1], 1.0 + m[2]
        else:
            cuts = np.sort(g.choice(np.arange(1, nx), size=min(3, nx - 1), replace=False))
            a, v, c = np.ones(nx), np.zeros(nx), np.ones(nx)
            for seg in np.split(np.arange(nx), cuts):
                a[seg], v[seg], c[seg] = g.uniform(0.5, 1.5), g.uniform(-0.5, 0.5), g.uniform(0.5, 1.5)
        if sysname == "sw":
            h = a
            out.append(np.concatenate([h, h * v]))
            smax = max(smax, float(np.max(np.abs(v) + np.sqrt(9.81 * h))))
        else:
            rho, p = a, c
            out.append(np.concatenate([rho, rho * v, p / (GAMMA - 1) + 0.5 * rho * v * v]))
            smax = max(smax, float(np.max(np.abs(v) + np.sqrt(GAMMA * p / rho))))
    return np.array(out), smax


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("nx", [8, 64, 100, 257, 512])
@pytest.mark.parametrize("k,numflux", [(0, 0), (1, 0), (2, 0), (3, 0), (0, 1), (2, 1), (3, 1)])
def test_phi_parity(orc, gpu, sysname, nx, k, numflux):
    u, smax = state_lines(sysname, 4, nx, nx + 7 * k + numflux)
    so, sg = schemes(orc, gpu, sysname, nx, k=k, stepper=3, numflux=numflux)
    dt = 0.5 / nx / smax
    out = T(np.zeros_like(u))
    gpu.phi(sg, dt, T(u), out)
    assert np.all(rel_lines(H(out), orc.phi(so, dt, u)) < TOL)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("stepper,k,numflux", [(1, 2, 0), (2, 1, 1), (1, 0, 1)])
def test_phi_parity_steppers(orc, gpu, sysname, stepper, k, numflux):
    nx = 128
    u, smax = state_lines(sysname, 4, nx, 3 + stepper)
    so, sg = schemes(orc, gpu, sysname, nx, k=k, stepper=stepper, numflux=numflux)
    dt = 0.3 / nx / smax
    out = T(np.zeros_like(u))
    gpu.phi(sg, dt, T(u), out)
    assert np.all(rel_lines(H(out), orc.phi(so, dt, u)) < TOL)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_serial_parity_and_conservation(orc, gpu, sysname):
    nx, nt = 200, 60
    u, smax = state_lines(sysname, 2, nx, 11)
    u0 = u[1]
    so, sg = schemes(orc, gpu, sysname, nx, k=2, numflux=1)
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
def test_relax_parity(orc, gpu, sysname):
    """F-relaxation of 8 chunks of m = 4 steps (mgrit_relax) equals stepping
    each chunk from its C-point with the oracle."""
    nx, m, n = 64, 4, 32
    u, smax = state_lines(sysname, n + 1, nx, 21)
    so, sg = schemes(orc, gpu, sysname, nx, k=3)
    dt = 0.5 / nx / smax
    a = T(u)
    gpu.relax(sg, dt, m, 0, a, None, n)
    ref = u.copy()
    for c in range(n // m):
        x = ref[c * m]
        for j in range(1, m):
            x = orc.phi(so, dt, x)
            ref[c * m + j] = x
    assert np.all(rel_lines(H(a), ref) < TOL)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("s_,numflux", [(1, 0), (5, 0), (3, 1), (7, 1)])
def test_high_order_experiment_parity(orc, gpu, sysname, s_, numflux):
    """Fig. MGRITweno for shallow water and Euler: 4 cycles on the GPU equal
    the oracle's iterates and residual history."""
    k = {1: 0, 3: 1, 5: 2, 7: 3}[s_]
    pb = W.e4_system(sysname, k, numflux)
    so, sg = schemes(orc, gpu, sysname, pb.nx, k=k, numflux=numflux)
    p = gpu.params(pb.nt, pb.dt, pb.m, pb.levels, relax=0, max_iter=4, tol=-1.0)
    u = T(np.zeros((pb.nt + 1, pb.u0.size)))
    rc, hg, n = gpu.cycle(sg, p, T(pb.u0), u)
    po = orc.params(pb.nt, pb.dt, pb.m, pb.levels, relax=0, max_iter=4, tol=-1.0)
    uo, ho, _, _ = orc.mgrit(so, po, pb.u0)
    assert np.all(rel_lines(H(u), uo) < TOL)
    # residuals fall to round-off within 4 cycles at s = 1: absolute floor
    np.testing.assert_allclose(hg, ho, rtol=1e-10, atol=1e-12 * ho[0])


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_cycles_fcf_fcycle_and_levels(orc, gpu, sysname):
    """FCF-relaxation, F-cycle, 4 levels; then a scheme per level (s = 5, 3, 1,
    SSPRK3/2/1): the GPU iterates equal the oracle's."""
    pb = W.e4_system(sysname, 2, 0)
    so, sg = schemes(orc, gpu, sysname, pb.nx, k=2)
    for relax, cycle in ((1, 0), (1, 1)):
        p = gpu.params(pb.nt, pb.dt, pb.m, 4, relax=relax, cycle=cycle, max_iter=2, tol=-1.0)
        u = T(np.zeros((pb.nt + 1, pb.u0.size)))
        gpu.cycle(sg, p, T(pb.u0), u)
        po = orc.params(pb.nt, pb.dt, pb.m, 4, relax=relax, cycle=cycle, max_iter=2, tol=-1.0)
        uo, _, _, _ = orc.mgrit(so, po, pb.u0)
        assert np.all(rel_lines(H(u), uo) < TOL), (relax, cycle)
    ks, ds = [2, 1, 0], [3, 2, 1]
    sos = [schemes(orc, gpu, sysname, pb.nx, k=k, stepper=d)[0] for k, d in zip(ks, ds)]
    sgs = [schemes(orc, gpu, sysname, pb.nx, k=k, stepper=d)[1] for k, d in zip(ks, ds)]
    p = gpu.params(pb.nt, pb.dt, pb.m, 3, relax=0, max_iter=3, tol=-1.0)
    u = T(np.zeros((pb.nt + 1, pb.u0.size)))
    gpu.cycle_levels(sgs, p, T(pb.u0), u)
    po = orc.params(pb.nt, pb.dt, pb.m, 3, relax=0, max_iter=3, tol=-1.0)
    uo, _, _, _ = orc.mgrit_levels(sos, po, pb.u0)
    assert np.all(rel_lines(H(u), uo) < TOL)


def test_systems_unsupported_calls(gpu):
    s = gpu.euler_scheme(64)
    w = T(np.ones((1, 3 * 64)))
    with pytest.raises(gpu.MgritError):
        gpu.phi_vjp(s, 1e-3, w, w, w)
    with pytest.raises(gpu.MgritError):
        gpu.autotune(s, 16, 2)
    big = gpu.shallow_water_scheme(70000)
    v = T(np.ones((1, 2 * 70000)))
    with pytest.raises(gpu.MgritError):
        gpu.phi(big, 1e-4, v, v)
    p = gpu.params(0, 0.0, 4, 2, relax=1, max_iter=1, tol=-1.0)
    u0 = T(np.ones(3 * 64))
    u = T(np.zeros((65, 3 * 64)))
    with pytest.raises(gpu.MgritError):
        gpu.cycle_batched([(s, 64, 1e-3, u0, u)], p)
