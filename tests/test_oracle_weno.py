"""Pins of the reference WENO reconstruction (sec 2.1.1) against facts fixed by
mathematics and by the paper's printed tables, independent of the reference's
own formulas."""
import os

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

from paper_2104_09404_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "weno5_k2_tables.txt")


def cell_avgs(coef, cells):
    """Exact averages of the polynomial ``coef`` over unit cells [d, d+1]."""
    Q = P.polyint(coef)
    return np.array([P.polyval(d + 1, Q) - P.polyval(d, Q) for d in cells])


def load_golden():
    blocks, cur, scale = {}, None, 1.0
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line[1:-1]
                blocks[cur] = []
                continue
            if line.startswith("scale"):
                scale = float(line.split()[1])
                blocks[cur + "_scale"] = scale
                continue
            blocks[cur].append([float(x) for x in line.split()])
    return {k: (np.array(v) / blocks[k + "_scale"] if not k.endswith("_scale") else v)
            for k, v in blocks.items() if not k.endswith("_scale")}


# window v = averages over cells i-2..i+2, with cell i = [0, 1], so x_{i+1/2} = 1
WINDOW = [-2, -1, 0, 1, 2]


def test_candidates_exact_on_quadratics(orc):
    """Each candidate polynomial of degree 2 reproduces any quadratic at x_{i+1/2}
    (eq C): this pins the c table and the stencil convention."""
    g = np.random.default_rng(0)
    for _ in range(50):
        coef = g.uniform(-3, 3, size=3)
        v = cell_avgs(coef, WINDOW)
        p = orc.weno5_candidates(v)
        np.testing.assert_allclose(p, P.polyval(1.0, coef), rtol=0, atol=1e-13)


def test_candidates_not_exact_on_cubics(orc):
    """A cubic is NOT reproduced by the 3-point candidates (sanity of the test above)."""
    coef = np.array([0.0, 0.0, 0.0, 1.0])
    v = cell_avgs(coef, WINDOW)
    p = orc.weno5_candidates(v)
    assert np.max(np.abs(p - 1.0)) > 1e-3


def test_linear_weights_exact_on_quartics(orc):
    """With eps -> infinity the weights become d_r and the combination is the
    5-point reconstruction, exact for degree-4 polynomials (eq D with s = 2k+1 = 5):
    this pins d and, together with the test above, the stencil convention."""
    g = np.random.default_rng(1)
    for _ in range(50):
        coef = g.uniform(-3, 3, size=5)
        v = cell_avgs(coef, WINDOW)
        val = orc.weno5_left(v, 1e30)
        assert abs(val - P.polyval(1.0, coef)) < 1e-12 * max(1.0, np.max(np.abs(coef)))


def test_nonlinear_weights_exact_on_quadratics(orc):
    """Any convex combination of exact candidates is exact: quadratics are reproduced
    with the nonlinear weights for any eps."""
    g = np.random.default_rng(2)
    for _ in range(20):
        coef = g.uniform(-3, 3, size=3)
        v = cell_avgs(coef, WINDOW)
        for eps in (1e-6, 1e-2, 1.0):
            assert abs(orc.weno5_left(v, eps) - P.polyval(1.0, coef)) < 1e-12


def beta_by_definition(q, cells):
    """eq B by its definition: fit the quadratic with cell averages q on ``cells``
    and integrate sum_l dx^{2l-1} (d^l p/dx^l)^2 over the reconstruction cell [0, 1]
    (dx = 1; the indicator is scale free)."""
    M = np.array([[((d + 1) ** (j + 1) - d ** (j + 1)) / (j + 1) for j in range(3)] for d in cells])
    coef = np.linalg.solve(M, q)
    total = 0.0
    for l in (1, 2):
        dl = P.polyder(coef, l)
        sq = P.polymul(dl, dl)
        I = P.polyint(sq)
        total += P.polyval(1.0, I) - P.polyval(0.0, I)
    return total


def test_beta_matches_integral_definition(orc):
    """The printed B_r reproduce the smoothness-indicator integral of eq B for the
    stencil r = {i-r, i-r+1, i-r+2}."""
    g = np.random.default_rng(3)
    for _ in range(50):
        v = g.uniform(-2, 2, size=5)
        beta = orc.weno5_beta(v)
        for r in range(3):
            cells = [-r, -r + 1, -r + 2]
            q = v[2 - r: 5 - r]
            ref = beta_by_definition(q, cells)
            assert abs(beta[r] - ref) < 1e-11 * max(1.0, abs(ref))


def test_tables_match_printed_golden(orc):
    """The candidate weights and B matrices equal the paper's printed k = 2 tables
    (tests/golden/weno5_k2_tables.txt)."""
    tab = load_golden()
    # c_{r,j}: response of candidate r to a unit average on its j-th stencil cell
    for r in range(3):
        for j in range(3):
            v = np.zeros(5)
            v[2 - r + j] = 1.0
            assert orc.weno5_candidates(v)[r] == pytest.approx(tab["c"][r, j], abs=1e-15)
    # B_r from the quadratic form: B_aa = beta(e_a), B_ab = (beta(e_a+e_b) - B_aa - B_bb)/2
    for r in range(3):
        Bm = np.zeros((3, 3))
        for a in range(3):
            e = np.zeros(5)
            e[2 - r + a] = 1.0
            Bm[a, a] = orc.weno5_beta(e)[r]
        for a in range(3):
            for b in range(3):
                if a != b:
                    e = np.zeros(5)
                    e[2 - r + a] = 1.0
                    e[2 - r + b] = 1.0
                    Bm[a, b] = (orc.weno5_beta(e)[r] - Bm[a, a] - Bm[b, b]) / 2
        np.testing.assert_allclose(Bm, tab["B%d" % r], atol=1e-13)
    # d_r: with eps -> infinity the output is sum_r d_r p_r
    g = np.random.default_rng(4)
    v = g.uniform(-1, 1, 5)
    p = orc.weno5_candidates(v)
    assert orc.weno5_left(v, 1e30) == pytest.approx(float(tab["d"][:, 0] @ p), abs=1e-14)


def test_eno_property_at_a_jump(orc):
    """Near a jump the weights of the stencils crossing it vanish: cell averages
    (0, 0, 0, 1, 1) reconstruct ~0 at x_{i+1/2}."""
    v = np.array([0.0, 0.0, 0.0, 1.0, 1.0])
    assert abs(orc.weno5_left(v, 1e-6)) < 1e-8
    v = np.array([0.0, 0.0, 1.0, 1.0, 1.0])
    assert abs(orc.weno5_left(v, 1e-6) - 1.0) < 1e-8


@pytest.mark.parametrize("eps,min_order", [(1e-6, 4.8), (1e30, 4.9)])
def test_weno5_fifth_order_on_smooth_burgers(orc, eps, min_order):
    """Convergence study of A(u) (eq spaceDisc with WENO5 + LF) against the exact
    cell average of -f(u)_x for smooth Burgers data: fitted L1 order about 5."""
    f = lambda u: 0.5 * u * u
    ns = [32, 64, 128, 256]
    errs = []
    for nx in ns:
        u = 0.5 + 0.25 * W.cell_average_sin(nx, 1, 0.0)
        A, _ = orc.spatial_operator(orc.scheme(nx, eps=eps), u)
        x = W.cell_edges(nx)
        ue = 0.5 + 0.25 * np.sin(2 * np.pi * x)
        Aex = -(f(ue[1:]) - f(ue[:-1])) * nx
        errs.append(np.mean(np.abs(A - Aex)))
    order = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert order > min_order, (errs, order)


def test_first_order_reconstruction_is_trivial(orc):
    """k = 0: u^-_{i+1/2} = u_i, u^+_{i+1/2} = u_{i+1} (end of sec 2.1.1).  With
    linear advection (a > 0, alpha = |a|) the LF flux is then a u_i exactly."""
    g = np.random.default_rng(5)
    nx = 16
    u = g.uniform(-1, 1, nx)
    a = 0.7
    A, alpha = orc.spatial_operator(orc.scheme(nx, flux=1, k=0, a=a), u)
    assert alpha == a
    F = a * u
    np.testing.assert_allclose(A, -(F - np.roll(F, 1)) * nx, atol=1e-13)


def test_reflection_symmetry_burgers(orc):
    """Burgers is invariant under u(x) -> -u(-x); the discrete operator (with the
    mirror reconstruction for u^+) commutes with that reflection."""
    g = np.random.default_rng(6)
    for k in (0, 2):
        u = W.shock_lines(7, 1, 40)[0] + 0.1 * g.standard_normal(40)
        s = orc.scheme(40, k=k)
        A, _ = orc.spatial_operator(s, u)
        Ar, _ = orc.spatial_operator(s, -u[::-1].copy())
        np.testing.assert_allclose(Ar, -A[::-1], atol=1e-12 * np.max(np.abs(A)))
