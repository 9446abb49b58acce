"""Pins of the oracle's scheme variants against what the paper and the
mathematics fix, independently of the oracle's own formulas:

* WENO of degree k = 1, 2, 3 (orders s = 3, 5, 7; sec 2.1.1, eq C, B, omega, D),
  whose tables the oracle derives from their definitions: the printed k = 2
  tables, the textbook WENO3 (Jiang & Shu 1996) and WENO7 (Balsara & Shu 2000)
  coefficients, exactness on polynomials, closed-form smoothness indicators,
  order of accuracy of the spatial operator;
* the Roe flux with the Harten-Hyman entropy fix (sec 2.1.3, eq roeflux; the
  reading with the 1/2 on the dissipation and lambda^2 in q_H): equal to the
  exact Godunov flux of Burgers' equation, upwind for advection, the Godunov
  and upwind schemes at first order, an opening transonic rarefaction;
* MGRIT with a different scheme on each level (Fig. MGRITweno_diffOrd);
* the qualitative findings of Fig. MGRITweno, MGRITweno_diffOrd and
  MGRITcfl (the curves themselves are not available, so parity of the
  histories is unpinned).
"""
import math

import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

K_OF_S = {1: 0, 3: 1, 5: 2, 7: 3}


def cell_averages(coef, offsets):
    """Exact averages of the polynomial sum_n coef[n] x^n over the cells
    [o - 1/2, o + 1/2] (dx = 1)."""
    P = np.polynomial.Polynomial(coef).integ()
    return np.array([P(o + 0.5) - P(o - 0.5) for o in offsets])


# ---------------------------------------------------------------------------
# WENO tables
# ---------------------------------------------------------------------------
def test_derived_k2_tables_equal_printed(orc):
    """The tables the oracle derives for k = 2 are the printed ones."""
    c, d, B = orc.weno_tables(2)
    c_printed = np.array([[2, 5, -1], [-1, 5, 2], [2, -7, 11]]) / 6.0
    d_printed = np.array([3, 6, 1]) / 10.0
    B_printed = np.array([
        [[20, -31, 11], [-31, 50, -19], [11, -19, 8]],
        [[8, -13, 5], [-13, 26, -13], [5, -13, 8]],
        [[8, -19, 11], [-19, 50, -31], [11, -31, 20]],
    ]) / 6.0
    np.testing.assert_allclose(c, c_printed, rtol=0, atol=1e-15)
    np.testing.assert_allclose(d, d_printed, rtol=0, atol=1e-15)
    np.testing.assert_allclose(B, B_printed, rtol=0, atol=1e-14)


def test_weno3_textbook(orc):
    """k = 1: candidates (q_i + q_{i+1})/2 and (3 q_i - q_{i-1})/2, linear
    weights 2/3 and 1/3, indicators (q_{i+1} - q_i)^2 and (q_i - q_{i-1})^2;
    the reconstruction is the Jiang-Shu WENO3 formula."""
    c, d, B = orc.weno_tables(1)
    np.testing.assert_allclose(c, [[0.5, 0.5], [-0.5, 1.5]], atol=1e-16)
    np.testing.assert_allclose(d, [2 / 3, 1 / 3], atol=1e-16)
    for r in range(2):
        np.testing.assert_allclose(B[r], [[1, -1], [-1, 1]], atol=1e-15)
    g = np.random.default_rng(3)
    for _ in range(50):
        qm, q0, qp = g.normal(size=3)
        eps = 1e-6
        b0, b1 = (qp - q0) ** 2, (q0 - qm) ** 2
        a0, a1 = (2 / 3) / (eps + b0) ** 2, (1 / 3) / (eps + b1) ** 2
        ref = (a0 * 0.5 * (q0 + qp) + a1 * 0.5 * (3 * q0 - qm)) / (a0 + a1)
        assert abs(orc.weno_left(1, [qm, q0, qp], eps) - ref) < 1e-14 * max(1.0, abs(ref))


def test_weno7_textbook(orc):
    """k = 3: the WENO7 candidate and linear weights (stencils from the right,
    cells i..i+3 first) and the smoothness indicator of the leftmost stencil
    (cells i-3..i, in units of 1/240)."""
    c, d, B = orc.weno_tables(3)
    np.testing.assert_allclose(d, np.array([4, 18, 12, 1]) / 35.0, atol=1e-16)
    c_ref = np.array([[3, 13, -5, 1], [-1, 7, 7, -1], [1, -5, 13, 3], [-3, 13, -23, 25]]) / 12.0
    np.testing.assert_allclose(c, c_ref, atol=1e-15)
    # beta = q0 (547 q0 - 3882 q1 + 4642 q2 - 1854 q3) + q1 (7043 q1 - 17246 q2 + 7042 q3)
    #        + q2 (11003 q2 - 9402 q3) + 2107 q3^2, all over 240
    B_ref = np.array([[547, -1941, 2321, -927], [-1941, 7043, -8623, 3521],
                      [2321, -8623, 11003, -4701], [-927, 3521, -4701, 2107]]) / 240.0
    np.testing.assert_allclose(B[3], B_ref, atol=1e-12)
    # the rightmost stencil is its mirror image
    np.testing.assert_allclose(B[0], B_ref[::-1, ::-1], atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_weno_exact_on_polynomials_of_degree_k(orc, k):
    """Every candidate reproduces a polynomial of degree <= k, so does any
    convex combination: the reconstruction is exact whatever the weights."""
    g = np.random.default_rng(10 + k)
    for _ in range(20):
        coef = g.normal(size=k + 1)
        v = cell_averages(coef, range(-k, k + 1))
        exact = np.polynomial.Polynomial(coef)(0.5)
        for eps in (1e-6, 1e-40):
            assert abs(orc.weno_left(k, v, eps) - exact) < 1e-13 * max(1.0, np.abs(coef).sum())


@pytest.mark.parametrize("k", [1, 2, 3])
def test_weno_linear_weights_exact_on_degree_2k(orc, k):
    """With eps far above every indicator the weights are the d_r of eq D,
    whose combination is the degree-2k reconstruction over 2k+1 cells."""
    g = np.random.default_rng(20 + k)
    for _ in range(20):
        coef = g.normal(size=2 * k + 1)
        v = cell_averages(coef, range(-k, k + 1))
        exact = np.polynomial.Polynomial(coef)(0.5)
        assert abs(orc.weno_left(k, v, 1e20) - exact) < 1e-12 * max(1.0, np.abs(coef).sum())


@pytest.mark.parametrize("k", [1, 2, 3])
def test_beta_closed_forms(orc, k):
    """eq B on data of a polynomial P that every stencil reproduces: beta_r =
    sum_l int_{-1/2}^{1/2} (P^(l))^2 dx.  P = x: 1; P = x^2: 1/3 + 4;
    P = x^3: 9/80 + 3 + 36."""
    c, d, B = orc.weno_tables(k)
    cases = [([0, 1], 1.0)]
    if k >= 2:
        cases.append(([0, 0, 1], 1 / 3 + 4))
    if k >= 3:
        cases.append(([0, 0, 0, 1], 9 / 80 + 3 + 36))
    for coef, beta in cases:
        for r in range(k + 1):
            q = cell_averages(coef, range(-r, -r + k + 1))
            assert abs(q @ B[r] @ q - beta) < 1e-12 * beta


@pytest.mark.parametrize("k", [1, 2, 3])
def test_weno_eno_property_at_a_step(orc, k):
    """A unit step between cells i and i+1: the one stencil left of it has
    beta = 0 and takes (almost) all the weight, so u^- stays at the left
    value instead of interpolating across the jump."""
    v = np.array([0.0] * (k + 1) + [1.0] * k)
    assert abs(orc.weno_left(k, v, 1e-6)) < 1e-9


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("a", [1.0, -0.6])
def test_spatial_order_of_accuracy(orc, k, a):
    """Advection with the Roe (upwind) flux and linear weights on exact cell
    averages of sin(2 pi x): A(u)_i approximates -a (u(x_{i+1/2}) -
    u(x_{i-1/2}))/dx to order 2k+1 (u^- for a > 0, the mirror-image u^+ for
    a < 0)."""
    errs = []
    for nx in (16, 32):
        u = W.cell_average_sin(nx, 1, 0.3)
        x = W.cell_edges(nx)
        ue = np.sin(2 * math.pi * x + 0.3)
        exact = -a * (ue[1:] - ue[:-1]) * nx
        s = orc.scheme(nx, flux=1, a=a, k=k, eps=1e20, numflux=1)
        A, _ = orc.spatial_operator(s, u)
        errs.append(np.max(np.abs(A - exact)))
    rate = math.log2(errs[0] / errs[1])
    assert rate > 2 * k + 1 - 0.25, (errs, rate)


# ---------------------------------------------------------------------------
# Roe flux with the Harten-Hyman fix
# ---------------------------------------------------------------------------
def godunov_burgers(ul, ur):
    """Exact Riemann-problem flux of Burgers' equation (convex f = u^2/2)."""
    f = lambda u: 0.5 * u * u  # noqa: E731
    if ul <= ur:
        return 0.0 if ul <= 0.0 <= ur else min(f(ul), f(ur))
    return max(f(ul), f(ur))


def test_roe_burgers_is_the_godunov_flux(orc):
    """With the 1/2 on the dissipation and lambda^2 in q_H, the scheme is the
    exact Godunov flux of Burgers' equation: upwind through shocks and
    one-sided rarefactions, zero through transonic rarefactions."""
    s = orc.scheme(16, numflux=1)
    pts = [-2.0, -1.3, -0.5, -1e-3, 0.0, 1e-3, 0.4, 1.0, 1.7]
    g = np.random.default_rng(4)
    pairs = [(a, b) for a in pts for b in pts] + [tuple(x) for x in g.uniform(-3, 3, size=(500, 2))]
    for ul, ur in pairs:
        ref = godunov_burgers(ul, ur)
        assert abs(orc.roe_flux(s, ul, ur) - ref) < 1e-15 * (1.0 + ul * ul + ur * ur), (ul, ur)


@pytest.mark.parametrize("a", [0.7, -1.3])
def test_roe_advection_is_upwind(orc, a):
    s = orc.scheme(16, flux=1, a=a, numflux=1)
    g = np.random.default_rng(5)
    for ul, ur in g.normal(size=(100, 2)):
        ref = a * (ul if a > 0 else ur)
        assert abs(orc.roe_flux(s, ul, ur) - ref) < 1e-15 * (1 + abs(ul) + abs(ur))


def test_roe_consistency(orc):
    s = orc.scheme(16, numflux=1)
    for u in np.linspace(-2, 2, 41):
        assert abs(orc.roe_flux(s, u, u) - 0.5 * u * u) < 1e-15 * (1 + u * u)


@pytest.mark.parametrize("flux", [0, 1])
def test_roe_first_order_is_godunov_or_upwind_scheme(orc, flux):
    """k = 0 and forward Euler: Godunov's scheme for Burgers, the upwind scheme
    for advection, written here from their textbook definitions."""
    nx = 50
    g = np.random.default_rng(6 + flux)
    u = g.uniform(-1.0, 1.0, size=nx)
    a = -0.8
    dx = 1.0 / nx
    dt = 0.4 * dx
    s = orc.scheme(nx, flux=flux, a=a, k=0, stepper=1, numflux=1)
    out = orc.phi(s, dt, u)
    if flux == 0:
        G = np.array([godunov_burgers(u[i], u[(i + 1) % nx]) for i in range(nx)])
    else:
        G = a * np.roll(u, -1)  # a < 0: the upwind value is the right cell
    ref = u - dt / dx * (G - np.roll(G, 1))
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_roe_advection_equals_lf_with_alpha_a(orc, k):
    """For advection, Roe's dissipation |a| equals the LF one with alpha = |a|:
    the two Phi agree to round-off for every reconstruction."""
    nx, a = 40, -0.9
    u = W.random_lines(7, 1, nx)[0]
    dt = 0.5 / nx / abs(a)
    roe = orc.phi(orc.scheme(nx, flux=1, a=a, k=k, stepper=3, numflux=1), dt, u)
    lf = orc.phi(orc.scheme(nx, flux=1, a=a, k=k, stepper=3, alpha_fixed=abs(a)), dt, u)
    np.testing.assert_allclose(roe, lf, rtol=0, atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_roe_conserves_mass(orc, k):
    nx = 64
    u = W.shock_lines(8, 1, nx)[0]
    s = orc.scheme(nx, k=k, stepper=3, numflux=1)
    out = orc.phi(s, 0.5 / nx / np.max(np.abs(u)), u)
    assert abs(out.sum() - u.sum()) < 1e-13 * np.abs(u).sum()


def test_roe_opens_a_transonic_rarefaction(orc):
    """u = -1 on the left half, +1 on the right: without an entropy fix the Roe
    flux keeps this expansion shock (F = 1/2 on both sides of it); with the
    Harten-Hyman fix the flux through it is 0, so after one first-order step
    the cells beside the jump move by dt/(2 dx) towards each other."""
    nx = 20
    u = np.where(np.arange(nx) < nx // 2, -1.0, 1.0)
    dx, dt = 1.0 / nx, 0.2 / nx
    out = orc.phi(orc.scheme(nx, k=0, stepper=1, numflux=1), dt, u)
    j = nx // 2
    assert out[j - 1] == pytest.approx(-1.0 + 0.5 * dt / dx, abs=1e-15)
    assert out[j] == pytest.approx(1.0 - 0.5 * dt / dx, abs=1e-15)
    unchanged = np.ones(nx, bool)
    unchanged[[j - 1, j]] = False
    np.testing.assert_array_equal(out[unchanged], u[unchanged])  # the shock at x = 0 stays


# ---------------------------------------------------------------------------
# a scheme per level
# ---------------------------------------------------------------------------
def test_levels_with_one_scheme_equal_mgrit(orc):
    pb = W.e4_high_order(2, 1, max_iter=3)
    s = orc.scheme(pb.nx, k=2, stepper=3, numflux=1)
    p = orc.params(pb.nt, pb.dt, pb.m, pb.levels, max_iter=3, tol=-1.0)
    a = orc.mgrit(s, p, pb.u0)
    b = orc.mgrit_levels([s] * pb.levels, p, pb.u0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_levels_fine_scheme_fixes_the_solution(orc):
    """Coarse levels with other schemes change the iterates, not what they
    converge to: after j cycles of F-relaxation the first j chunks equal
    serial stepping with the level-0 scheme, and the converged iterate is
    the serial solution."""
    pb = W.e4_high_order(2, 0)
    s0 = orc.scheme(pb.nx, k=2, stepper=3)
    schemes = [s0, orc.scheme(pb.nx, k=1, stepper=2), orc.scheme(pb.nx, k=0, stepper=1, numflux=1)]
    us = orc.serial(s0, pb.dt, pb.nt, pb.u0)
    m_chunk = pb.m
    one = None
    for j in (1, 2, 3):
        p = orc.params(pb.nt, pb.dt, pb.m, pb.levels, max_iter=j, tol=-1.0)
        u, hist, it, st = orc.mgrit_levels(schemes, p, pb.u0)
        assert np.array_equal(u[: j * m_chunk + 1], us[: j * m_chunk + 1])
        if j == 1:
            one = u
    same = orc.mgrit(s0, orc.params(pb.nt, pb.dt, pb.m, pb.levels, max_iter=1, tol=-1.0), pb.u0)[0]
    assert np.max(np.abs(one - same)) > 1e-6  # the coarse schemes are used
    p = orc.params(pb.nt, pb.dt, pb.m, pb.levels, max_iter=200, tol=1e-11)
    u, hist, it, st = orc.mgrit_levels([s0, orc.scheme(pb.nx, k=1, stepper=3), orc.scheme(pb.nx, k=0, stepper=3)],
                                       p, pb.u0)
    assert st == 0
    assert np.max(np.abs(u - us)) < 1e-9


# ---------------------------------------------------------------------------
# the paper's high-order experiments (shapes only)
# ---------------------------------------------------------------------------
def error_curve(orc, schemes, pb, n, relative=False):
    """||u_k - u_S|| (space-time, scaled by sqrt(dx), or relative to ||u_S||)
    after k = 0..n cycles, each cycle continuing from the previous iterate."""
    us = orc.serial(schemes[0], pb.dt, pb.nt, pb.u0)
    scale = 1.0 / np.linalg.norm(us) if relative else math.sqrt(pb.dx)
    errs, u = [], None
    for j in range(n + 1):
        p = orc.params(pb.nt, pb.dt, pb.m, pb.levels, relax=pb.relax, max_iter=1 if j else 0, tol=-1.0,
                       init=1 if j else 0)
        u, _, _, _ = orc.mgrit_levels(schemes, p, pb.u0, u)
        with np.errstate(all="ignore"):
            errs.append(np.linalg.norm(u - us) * scale)
    return np.array(errs)


@pytest.mark.parametrize("numflux", [0, 1])
def test_high_order_experiment_shape(orc, numflux):
    """Fig. MGRITweno (Burgers, LF left / Roe right): s = 1 converges fastest,
    performance worsens from s = 5 to s = 7, and s = 3 is the exception that
    behaves worst."""
    err = {}
    for s_ in (1, 3, 5, 7):
        pb = W.e4_high_order(K_OF_S[s_], numflux)
        sch = orc.scheme(pb.nx, k=K_OF_S[s_], stepper=3, numflux=numflux)
        err[s_] = error_curve(orc, [sch] * 3, pb, 3)[3]
    assert err[1] < err[5] < err[7] < err[3], err
    assert err[1] < 1e-10 and err[3] > 1e-6


@pytest.mark.parametrize("numflux", [0, 1])
def test_order_across_levels_shape(orc, numflux):
    """Fig. MGRITweno_diffOrd: changing s (and the RK order d) across levels is
    worse than rediscretising with one scheme; decreasing the order towards
    the coarse levels is the more promising direction."""
    pb = W.e4_high_order(2, numflux)

    def run(ss, ds):
        sch = [orc.scheme(pb.nx, k=K_OF_S[a], stepper=d, numflux=numflux) for a, d in zip(ss, ds)]
        return error_curve(orc, sch, pb, 8)

    const = run([5, 5, 5], [3, 3, 3])
    dec = run([5, 3, 1], [3, 3, 3])
    dec_d = run([5, 3, 1], [3, 2, 1])
    inc = run([1, 3, 5], [3, 3, 3])
    assert const[6] < 1e-9
    for alt in (dec, dec_d, inc):
        assert alt[6] > 1e3 * const[6]
    assert dec[8] < inc[8] and dec_d[8] < inc[8]
    assert dec[8] < dec[2]


def test_cfl_experiment_shape(orc):
    """Fig. MGRITcfl with the Roe flux (N_x = 128, T = 0.475, 5 levels, m = 2,
    u0 = sin(2 pi x)), coarsest CFL c = 972.8/N_t: WENO5 with forward Euler
    diverges at c = 0.95 after a few iterations; with SSPRK3, s = 1 and s = 5
    converge for c <= 0.95, more slowly as c grows; at c = 1.9 s = 5 is far
    more sensitive than s = 1; both diverge at c = 3.8."""
    nx, T = 128, 0.475
    u0 = W.cell_average_sin(nx, 1, 0.0)

    def curve(k, stepper, nt, n):
        pb = W.Problem("e3", 0, k, stepper, nx, nt, T / nt, 2, 5, 0, u0)
        return error_curve(orc, [orc.scheme(nx, k=k, stepper=stepper, numflux=1)] * 5, pb, n, relative=True)

    fe = curve(2, 1, 1024, 3)
    assert not np.all(np.isfinite(fe)) or fe[-1] > 1.0
    e3 = {}
    for k in (0, 2):
        e3[k] = [curve(k, 3, nt, 3)[3] for nt in (2048, 1024, 512)]
        assert e3[k][0] < e3[k][1] < 1e-6, e3  # relative space-time error after 3 cycles
    assert e3[2][2] > 1e3 * e3[0][2]
    for k in (0, 2):
        last = curve(k, 3, 256, 2)[-1]
        assert not np.isfinite(last) or last > 1.0
