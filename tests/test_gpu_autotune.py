"""The launch-shape autotuner (mgrit_autotune): it picks a compiled
configuration that covers the line, installs it as the override of its
regime, and the results stay bitwise equal (every configuration evaluates
the same per-cell operations); a batch tuned this way gives the same
iterates as the untuned batch."""
import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_09404_amd import mgrit

    mgrit.load()
    yield mgrit
    mgrit.clear_kernel_config()


def T(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def H(t):
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("nx", [100, 1024, 3000])
@pytest.mark.parametrize("k,numflux", [(2, 0), (3, 1), (0, 0)])
def test_autotune_installs_a_covering_config(gpu, nx, k, numflux):
    s = gpu.scheme(nx, k=k, numflux=numflux)
    u = W.random_lines(9, 64, nx)
    dt = 0.5 / nx / np.max(np.abs(u))
    before = T(np.zeros_like(u))
    gpu.phi(s, dt, T(u), before)
    for nlines in (512, 1):
        cpt, nw, ms = gpu.autotune(s, nlines, 4)
        assert 64 * cpt * nw >= nx and ms > 0.0
        assert gpu.kernel_config(nx, nlines) == (cpt, nw)
    after = T(np.zeros_like(u))
    gpu.phi(s, dt, T(u), after)
    assert np.array_equal(H(before), H(after))


def test_autotuned_batch_equals_untuned(gpu):
    m = 4
    g = np.random.default_rng(7)
    probs = []
    for i, nx in enumerate([64, 300, 1000, 2050, 4096]):
        flux = i % 2
        a = float(g.uniform(0.5, 1.5)) if flux else 1.0
        u0 = W.random_lines(700 + i, 1, nx)[0]
        dt = 0.6 / nx / (np.max(np.abs(u0)) if flux == 0 else a)
        probs.append((gpu.scheme(nx, flux=flux, a=a), 4 * m * max(1, nx // (4 * m)), dt, u0))
    p = gpu.params(0, 0.0, m, 2, relax=1, max_iter=2, tol=-1.0, sync_every=2)

    def run():
        table, us = [], []
        for sch, nt, dt, u0 in probs:
            u = T(np.zeros((nt + 1, sch.nx)))
            us.append(u)
            table.append((sch, nt, dt, T(u0), u))
        gpu.cycle_batched(table, p)
        return [H(u) for u in us], table

    ref, table = run()
    tuned = gpu.autotune_batch(table, nsteps=4)
    assert sorted(tuned) == [64, 300, 1000, 2050, 4096]
    got, _ = run()
    for a, b in zip(ref, got):
        with np.errstate(invalid="ignore"):
            assert np.all((a == b) | (np.isnan(a) & np.isnan(b)))


@pytest.mark.parametrize("nx,nlines", [(8192, 64), (6002, 64), (65536, 16)])
def test_split_line_autotune(gpu, nx, nlines):
    """mgrit_autotune_tiled times every compiled split-line shape, including
    two intervals (chunks) per workgroup, installs the fastest, and results
    stay bitwise equal."""
    s = gpu.scheme(nx)
    u = W.random_lines(19, 4, nx)
    dt = 0.5 / nx / np.max(np.abs(u))
    before = T(np.zeros_like(u))
    gpu.phi(s, dt, T(u), before)
    try:
        cpt, nw, iv, ms = gpu.autotune_tiled(s, nlines, 2)
        assert ms > 0.0 and iv in (1, 2)
        tc = gpu.tiled_config(nx)
        assert tc[:2] == (cpt, nw) and tc[2] >= 1
        assert gpu.tiled_intervals(nx) == iv
        after = T(np.zeros_like(u))
        gpu.phi(s, dt, T(u), after)
        assert np.array_equal(H(before), H(after))
    finally:
        gpu.clear_tiled_config()
