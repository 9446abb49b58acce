"""GPU parity of the discrete adjoint on split lines (one line over several
workgroups, one global synchronisation per reverse Runge-Kutta stage): the
reverse sweep against the oracle's, forced splits of short lines against
the one-workgroup adjoint, and the adjoint workload's 4096-cell lines
(N_T = 2048, checkpoints every 32 steps) against the oracle and central
differences."""
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


def rel(x, ref):
    return np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300)


def gpu_gradient(gpu, sg, dt, nt, every, u0, tgt, parallel=0):
    ck = T(np.zeros((nt // every + 1, u0.size)))
    gpu.checkpoints(sg, dt, nt, every, T(u0), ck)
    uT = H(ck)[-1]
    lam0 = T(np.zeros(u0.size))
    gpu.adjoint(sg, dt, nt, every, ck, T(uT - tgt), lam0, parallel_segments=parallel)
    return 0.5 * np.sum((uT - tgt) ** 2), H(lam0)


@pytest.mark.parametrize("nx,cfg", [(1000, (1, 4)), (1024, (2, 4)), (768, (2, 8)), (600, (1, 4))])
@pytest.mark.parametrize("k,stepper,flux", [(2, 3, 0), (2, 2, 1), (0, 1, 0), (2, 1, 0)])
def test_split_adjoint_vs_oracle_and_one_workgroup(orc, tiled, nx, cfg, k, stepper, flux):
    nt, every = 48, 16
    u0 = W.random_lines(80 + nx, 1, nx)[0]
    tgt = u0 + 0.02 * W.random_lines(81, 1, nx, mean=0.0)[0]
    a = 0.9
    dt = 0.7 / nx / (np.max(np.abs(u0)) if flux == 0 else a)
    so = orc.scheme(nx, flux=flux, k=k, stepper=stepper, a=a)
    sg = tiled.scheme(nx, flux=flux, k=k, stepper=stepper, a=a)
    J_one, g_one = gpu_gradient(tiled, sg, dt, nt, every, u0, tgt, parallel=2)
    tiled.set_tiled_config(nx, nx, *cfg)
    J_split, g_split = gpu_gradient(tiled, sg, dt, nt, every, u0, tgt, parallel=2)
    assert J_split == J_one  # the forward sweeps are bitwise equal
    unstable = k == 2 and stepper == 1
    # the split reverse sweep sums the adjoint of alpha_LF in another order
    assert rel(g_split, g_one) < (1e-9 if unstable else 1e-12), rel(g_split, g_one)
    if unstable:
        # WENO5 + forward Euler is unstable (sec 4): round-off differences
        # between the oracle's and the kernels' trajectories grow, so only the
        # split and one-workgroup kernels (bitwise equal forward) are compared
        return
    Jo, go = orc.serial_adjoint(so, dt, nt, u0, tgt)
    assert abs(J_split - Jo) <= 1e-12 * max(Jo, 1e-300)
    assert rel(g_split, go) < 1e-10, rel(g_split, go)


def test_adjoint_workload_reduced_steps_vs_oracle(orc, gpu):
    """The 4096-cell adjoint workload over its first 256 steps: the forward runs
    on one workgroup, the reverse sweep on 8 tiles of 512 cells (its default
    split); the gradient equals the oracle's reverse sweep."""
    nx, nt, every = 4096, 256, 32
    pb = W.w4_adjoint(nx=nx, nt=nt)
    assert gpu.tiled_config(nx)[2] == 1  # the forward fits one workgroup
    sg = gpu.scheme(nx)
    J, grad = gpu_gradient(gpu, sg, pb.dt, nt, every, pb.u0, pb.extra["u_target"], parallel=4)
    Jo, go = orc.serial_adjoint(orc.scheme(nx), pb.dt, nt, pb.u0, pb.extra["u_target"])
    assert abs(J - Jo) <= 1e-12 * Jo
    assert rel(grad, go) < 1e-10, rel(grad, go)


def test_adjoint_workload_full_size(orc, gpu):
    """N_x = 4096, N_T = 2048, checkpoints every 32 steps: dJ/du0 against the
    oracle's reverse sweep (1e-10, the bar of every GPU-vs-CPU reverse sweep)
    and against central differences (h = 1e-6) of the GPU forward in all 16
    of the workload's unit directions."""
    pb = W.w4_adjoint()
    nx, nt, every = pb.nx, pb.nt, pb.extra["checkpoint_every"]
    sg = gpu.scheme(nx)
    tgt = pb.extra["u_target"]
    J, grad = gpu_gradient(gpu, sg, pb.dt, nt, every, pb.u0, tgt, parallel=16)
    Jo, go = orc.serial_adjoint(orc.scheme(nx), pb.dt, nt, pb.u0, tgt)
    assert abs(J - Jo) <= 1e-11 * Jo
    assert rel(grad, go) < 1e-10, rel(grad, go)
    print("full-size adjoint: rel L2 vs oracle %.3e" % rel(grad, go))
    h = 1e-6

    def Jf(u):
        ck = T(np.zeros((nt // every + 1, nx)))
        gpu.checkpoints(sg, pb.dt, nt, every, T(u), ck)
        d = H(ck)[-1] - tgt
        return 0.5 * d @ d

    assert len(pb.extra["directions"]) == 16
    for d in pb.extra["directions"]:
        fd = (Jf(pb.u0 + h * d) - Jf(pb.u0 - h * d)) / (2 * h)
        assert abs(fd - grad @ d) <= 1e-6 * max(abs(fd), 1e-12), (fd, grad @ d)
