"""Pins of the oracle's systems (sec 2: shallow water, eq shallowWater;
Euler, eq Euler with gamma = 5/3), independently of the oracle's formulas:

* fluxes at rest states and in Galilean form;
* the eigen-decomposition against a finite-difference Jacobian of the flux;
* Roe's property f(u+) - f(u-) = A_hat (u+ - u-) of the Roe averages
  (readings R18, R19), Roe's flux consistent and upwind in supersonic flow;
* constant states and conservation under Phi;
* the characteristic-wise reconstruction exact on polynomial data;
* alpha_LF of a system taken over the reconstructed states u^-/+ of every
  interface (eq eigs), with the closed-form eigenvalues of sec 2.1.3;
* the characteristic decomposition on the central cell's eigenvectors
  (sec 2.1.1), through a stencil that varies along one closed-form
  eigenvector of that cell;
* order of accuracy on an exactly advected entropy wave (Euler) and by
  self-convergence (shallow water);
* the shape of Fig. MGRITweno for both systems (s = 1 converges fastest).
"""
import math

import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W

G, GAMMA = 9.81, 5.0 / 3.0


def sw_state(h, v):
    return np.array([h, h * v])


def euler_state(rho, v, p):
    return np.array([rho, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * v * v])


def random_states(sysname, n, seed, vmax=1.0):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        if sysname == "sw":
            out.append(sw_state(g.uniform(0.5, 2.0), g.uniform(-vmax, vmax)))
        else:
            out.append(euler_state(g.uniform(0.5, 2.0), g.uniform(-vmax, vmax), g.uniform(0.5, 2.0)))
    return out


def schemes(orc, sysname, nx, **kw):
    return orc.shallow_water_scheme(nx, **kw) if sysname == "sw" else orc.euler_scheme(nx, **kw)


def test_flux_closed_forms(orc):
    sw = orc.shallow_water_scheme(8)
    np.testing.assert_allclose(orc.sys_flux(sw, sw_state(0.7, 0.0)), [0.0, 0.5 * G * 0.49], rtol=1e-15)
    eu = orc.euler_scheme(8)
    E = 2.5
    np.testing.assert_allclose(orc.sys_flux(eu, np.array([1.3, 0.0, E])), [0.0, (GAMMA - 1) * E, 0.0],
                               rtol=1e-15, atol=1e-300)
    # Galilean form: f = v u + (0, p, p v)
    for u in random_states("euler", 20, 1):
        rho, v = u[0], u[1] / u[0]
        p = (GAMMA - 1) * (u[2] - 0.5 * rho * v * v)
        np.testing.assert_allclose(orc.sys_flux(eu, u), v * u + np.array([0.0, p, p * v]), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_eigenstructure_matches_jacobian(orc, sysname):
    """J_f(u) R = R diag(lambda) with J_f from central differences of f;
    L R = I; the eigenvalues ascend and are v -/+ c (and v for Euler)."""
    s = schemes(orc, sysname, 8)
    for u in random_states(sysname, 20, 2):
        lam, R, L = orc.sys_eig(s, u)
        D = u.size
        J = np.zeros((D, D))
        for j in range(D):
            h = 1e-6 * max(1.0, abs(u[j]))
            e = np.zeros(D)
            e[j] = h
            J[:, j] = (orc.sys_flux(s, u + e) - orc.sys_flux(s, u - e)) / (2 * h)
        np.testing.assert_allclose(J @ R, R @ np.diag(lam), atol=2e-7 * np.max(np.abs(J)))
        np.testing.assert_allclose(L @ R, np.eye(D), atol=1e-13)
        assert np.all(np.diff(lam) > 0)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_roe_property(orc, sysname):
    """The Roe-averaged matrix A_hat = R diag(lambda) L satisfies
    f(u+) - f(u-) = A_hat (u+ - u-) exactly, and A_hat(u, u) = J_f(u)."""
    s = schemes(orc, sysname, 8)
    st = random_states(sysname, 60, 3, vmax=2.0)
    for uL, uR in zip(st[0::2], st[1::2]):
        lam, R, L = orc.sys_roe_eig(s, uL, uR)
        A = R @ np.diag(lam) @ L
        df = orc.sys_flux(s, uR) - orc.sys_flux(s, uL)
        np.testing.assert_allclose(A @ (uR - uL), df, rtol=1e-12, atol=1e-12 * np.max(np.abs(df)))
        lam2, R2, L2 = orc.sys_eig(s, uL)
        lam3, R3, L3 = orc.sys_roe_eig(s, uL, uL)
        np.testing.assert_allclose(lam3, lam2, rtol=1e-14)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_roe_flux_consistent_and_upwind(orc, sysname):
    """F(u, u) = f(u); with every wave moving right (left) at both states
    and at the Roe state, the flux is f(u-) (f(u+))."""
    s = schemes(orc, sysname, 8, numflux=1)
    for u in random_states(sysname, 20, 4, vmax=2.0):
        np.testing.assert_allclose(orc.sys_roe_flux(s, u, u), orc.sys_flux(s, u), rtol=1e-14, atol=1e-14)
    g = np.random.default_rng(5)
    checked = 0
    for sign in (1.0, -1.0):
        for _ in range(40):
            if sysname == "sw":
                uL, uR = sw_state(g.uniform(0.1, 0.3), sign * g.uniform(3, 5)), sw_state(g.uniform(0.1, 0.3),
                                                                                        sign * g.uniform(3, 5))
            else:
                uL = euler_state(g.uniform(0.5, 2), sign * g.uniform(4, 6), g.uniform(0.5, 1))
                uR = euler_state(g.uniform(0.5, 2), sign * g.uniform(4, 6), g.uniform(0.5, 1))
            lams = [orc.sys_eig(s, uL)[0], orc.sys_eig(s, uR)[0], orc.sys_roe_eig(s, uL, uR)[0]]
            if not all(np.all(sign * l > 0) for l in lams):
                continue
            ref = orc.sys_flux(s, uL if sign > 0 else uR)
            np.testing.assert_allclose(orc.sys_roe_flux(s, uL, uR), ref, rtol=1e-13, atol=1e-13)
            checked += 1
    assert checked > 40


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("k,numflux", [(0, 0), (2, 0), (3, 1), (1, 1)])
def test_constant_state_and_conservation(orc, sysname, k, numflux):
    nx = 32
    s = schemes(orc, sysname, nx, k=k, numflux=numflux)
    u = (sw_state(0.8, 0.4) if sysname == "sw" else euler_state(1.1, 0.3, 0.9))
    const = np.repeat(u, nx)
    np.testing.assert_allclose(orc.phi(s, 1e-3, const), const, rtol=1e-14)
    sn = W.cell_average_sin(nx, 1, 0.4)
    if sysname == "sw":
        v = np.concatenate([1.0 + 0.3 * sn, 0.2 * W.cell_average_sin(nx, 2, 0.1)])
    else:
        v = np.concatenate([1.0 + 0.3 * sn, 0.2 * sn, 2.0 + 0.5 * W.cell_average_sin(nx, 3, 0.2)])
    out = orc.phi(s, 0.2 / nx, v)
    D = v.size // nx
    for d in range(D):
        assert abs(out[d * nx:(d + 1) * nx].sum() - v[d * nx:(d + 1) * nx].sum()) < 1e-13 * nx


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_characteristic_reconstruction_exact_on_polynomials(orc, sysname, k):
    """Components that are cell averages of polynomials of degree <= k: the
    characteristic variables of each cell are constant combinations of them,
    so every interface value is exact (cells whose stencil does not wrap)."""
    nx = 40
    s = schemes(orc, sysname, nx, k=k)
    g = np.random.default_rng(6 + k)
    base = (np.array([1.0, 0.2]) if sysname == "sw" else np.array([1.0, 0.2, 2.0]))
    comps, polys = [], []
    for b in base:
        coef = np.zeros(k + 1)
        coef[0] = b
        coef[1:] = g.normal(size=k) * 1e-3 / np.arange(1, k + 1) ** 2
        P = np.polynomial.Polynomial(coef)
        I = P.integ()
        x = np.arange(nx + 1) - 20.0  # cell edges, dx = 1 in the polynomial's units
        comps.append(I(x[1:]) - I(x[:-1]))
        polys.append(P)
    u = np.concatenate(comps)
    um, up = orc.sys_recon(s, u)
    for i in range(k, nx - k):
        for d, P in enumerate(polys):
            assert abs(um[d, i] - P(i - 20.0 + 1.0)) < 1e-13
            assert abs(up[d, i] - P(i - 20.0)) < 1e-13


def test_euler_entropy_wave_order(orc):
    """rho = 1 + 0.2 sin 2 pi x, v = 1, p = 1 is advected unchanged at speed 1
    (a contact): WENO5 + SSPRK3 with the characteristic reconstruction
    converges at order > 4 (dt ~ dx^(5/3))."""
    T = 0.1
    errs = []
    for nx in (32, 64):
        s = orc.euler_scheme(nx, k=2, stepper=3)
        rho = 1.0 + 0.2 * W.cell_average_sin(nx, 1, 0.0)
        u0 = np.concatenate([rho, rho, 1.0 / (GAMMA - 1) + 0.5 * rho])
        dx = 1.0 / nx
        nt = int(math.ceil(T / (0.5 * dx ** (5.0 / 3.0))))
        dt = T / nt
        uT = orc.serial(s, dt, nt, u0)[-1]
        rho_ex = 1.0 + 0.2 * W.cell_average_sin(nx, 1, -2 * math.pi * T)
        errs.append(np.max(np.abs(uT[:nx] - rho_ex)))
    assert math.log2(errs[0] / errs[1]) > 4.0, errs


def test_shallow_water_self_convergence(orc):
    """A smooth wave of height 1 + 0.1 sin 2 pi x at rest, evolved to T = 0.05
    (before it steepens into a bore): the differences between successive
    grids shrink at order > 3.5 for WENO5 + SSPRK3 (dt ~ dx^(5/3))."""
    T = 0.05
    sols = []
    for nx in (32, 64, 128):
        s = orc.shallow_water_scheme(nx, k=2, stepper=3)
        h = 1.0 + 0.1 * W.cell_average_sin(nx, 1, 0.0)
        u0 = np.concatenate([h, np.zeros(nx)])
        nt = int(math.ceil(T / (0.1 * (1.0 / nx) ** (5.0 / 3.0))))
        sols.append(orc.serial(s, T / nt, nt, u0)[-1][:nx])

    def coarsen(a):
        return 0.5 * (a[0::2] + a[1::2])

    e1 = np.max(np.abs(sols[0] - coarsen(sols[1])))
    e2 = np.max(np.abs(sols[1] - coarsen(sols[2])))
    assert math.log2(e1 / e2) > 3.5, (e1, e2)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("numflux", [0, 1])
def test_high_order_experiment_shape(orc, sysname, numflux):
    """Fig. MGRITweno for shallow water and Euler (N_x = 64, N_T = 400, T = 0.5,
    3-level V-cycle, m = 2, F-relaxation; u0 = ((1 + sin(2 pi x)/2)/11, 0) and
    (1, 0, 1 + sin(2 pi x)/2)): s = 1 converges fastest."""
    pb = W.e4_system(sysname, 0, numflux)
    err = {}
    for k in (0, 1, 2, 3):
        s = schemes(orc, sysname, pb.nx, k=k, numflux=numflux)
        us = orc.serial(s, pb.dt, pb.nt, pb.u0)
        p = orc.params(pb.nt, pb.dt, pb.m, pb.levels, relax=0, max_iter=3, tol=-1.0)
        u, _, _, _ = orc.mgrit(s, p, pb.u0)
        err[k] = np.linalg.norm(u - us) / np.linalg.norm(us)
    assert all(err[0] < 1e-2 * err[k] for k in (1, 2, 3)), err


@pytest.mark.parametrize("sysname", ["sw", "euler"])
def test_entropy_fix_inactive_in_shocks(orc, sysname):
    """The Harten-Hyman fix acts on rarefactions only: where every wave family
    is compressive with the Roe speed between the two sides (lambda_k(u+) <=
    lambda_hat_k <= lambda_k(u-)), delta_k = 0 and the flux is the plain Roe
    flux (f(u-) + f(u+))/2 - |A_hat| (u+ - u-)/2, also for near-sonic shocks
    (|lambda_hat| small)."""
    s = schemes(orc, sysname, 8, numflux=1)
    g = np.random.default_rng(9)
    checked = near_sonic = 0
    for _ in range(4000):
        if sysname == "sw":
            hL, hR = g.uniform(0.5, 2.0), g.uniform(0.5, 2.0)
            vL = g.uniform(-5, 5)
            uL, uR = sw_state(hL, vL), sw_state(hR, vL - g.uniform(0.5, 4))
        else:
            vL = g.uniform(-3, 3)
            uL = euler_state(g.uniform(0.5, 2), vL, g.uniform(0.5, 2))
            uR = euler_state(g.uniform(0.5, 2), vL - g.uniform(0.5, 4), g.uniform(0.5, 2))
        lL, lR = orc.sys_eig(s, uL)[0], orc.sys_eig(s, uR)[0]
        lam, R, L = orc.sys_roe_eig(s, uL, uR)
        if not (np.all(lR <= lam) and np.all(lam <= lL)):
            continue
        plain = 0.5 * (orc.sys_flux(s, uL) + orc.sys_flux(s, uR)) - 0.5 * (R @ np.diag(np.abs(lam)) @ L) @ (uR - uL)
        np.testing.assert_allclose(orc.sys_roe_flux(s, uL, uR), plain, rtol=1e-12, atol=1e-12)
        checked += 1
        near_sonic += int(np.any(np.abs(lam) < (lL - lam)))
    assert checked > 100 and near_sonic > 10, (checked, near_sonic)


def closed_form_speeds(sysname, u):
    """|lambda_k| of sec 2.1.3 written from the primitive variables:
    v -/+ sqrt(g h) for shallow water, v - c, v, v + c with c^2 = gamma p / rho
    for Euler (u holds one state per column)."""
    if sysname == "sw":
        h, v = u[0], u[1] / u[0]
        c = np.sqrt(G * h)
        return np.abs(np.stack([v - c, v + c]))
    rho, v = u[0], u[1] / u[0]
    p = (GAMMA - 1.0) * (u[2] - 0.5 * rho * v * v)
    c = np.sqrt(GAMMA * p / rho)
    return np.abs(np.stack([v - c, v, v + c]))


def wavy_line(sysname, nx, seed):
    """A periodic line with a steep front and a smooth hump, physical
    everywhere (h, rho, p > 0) and with velocities of both signs."""
    g = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    front = np.tanh((x - 0.3) * 40.0) * 0.3
    hump = 0.2 * np.sin(2 * np.pi * x + g.uniform(0, 2 * np.pi))
    if sysname == "sw":
        h = 1.0 + front + hump
        v = 0.8 * np.cos(2 * np.pi * x + g.uniform(0, 2 * np.pi))
        return np.concatenate([h, h * v])
    rho = 1.0 + front + hump
    v = 0.9 * np.cos(2 * np.pi * x + g.uniform(0, 2 * np.pi))
    p = 1.0 + 0.5 * front - hump
    return np.concatenate([rho, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * v * v])


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_lf_speed_is_taken_over_reconstructed_states(orc, sysname, k):
    """eq eigs (sec 2.1.2): alpha_LF of a system is the largest |lambda_k| of
    the closed-form eigenvalues over both reconstructed states u^- and u^+ of
    every interface, not over the cell averages.  The line is chosen so that
    the two maxima differ, and u^+/- come from the reconstruction that the
    polynomial and reference-state pins fix."""
    nx = 32
    s = schemes(orc, sysname, nx, k=k)
    u = wavy_line(sysname, nx, 40 + k)
    D = u.size // nx
    um, up = orc.sys_recon(s, u)
    expect = max(closed_form_speeds(sysname, um.reshape(D, nx)).max(),
                 closed_form_speeds(sysname, up.reshape(D, nx)).max())
    from_averages = closed_form_speeds(sysname, u.reshape(D, nx)).max()
    assert abs(expect - from_averages) > 1e-6 * expect, (expect, from_averages)
    _, alpha = orc.spatial_operator(s, u)
    assert abs(alpha - expect) <= 1e-14 * expect, (alpha, expect)


@pytest.mark.parametrize("sysname", ["sw", "euler"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_characteristic_reconstruction_on_central_cell(orc, sysname, k):
    """sec 2.1.1 decomposes a cell's stencil on the eigenvectors of that
    cell's own state u_c.  With the stencil u_j = u_c + s_j r_q(u_c), where
    r_q is the closed-form right eigenvector (sec 2.1.3) and s_0 = 0 at the
    central cell, the characteristic variables are constants except the q-th,
    which is l_q.u_c + s_j.  Hence u^-_{i+1/2} = u_c + W(s) r_q(u_c) and
    u^+_{i-1/2} = u_c + W(reversed s) r_q(u_c), W being the scalar WENO
    pinned by the golden tables.  The s_j jump at amplitude 1e-3, where the
    smoothness indicators are of the size of eps and W is far from linear, so
    a decomposition on another cell's eigenvectors misses by about 1e-7.  The
    bound 1e-11 allows for eq B's quadratic forms acting on the values
    themselves: an offset of order 1 costs about 1e-15 in beta, a relative
    1e-9 at beta ~ eps, which W turns into about 1e-12 at this amplitude."""
    nx, i = 16, 8
    s = schemes(orc, sysname, nx, k=k)
    if sysname == "sw":
        h, v = 1.2, 0.4
        c = math.sqrt(G * h)
        uc = sw_state(h, v)
        vecs = [np.array([1.0, v - c]), np.array([1.0, v + c])]
    else:
        rho, v, p = 1.1, 0.3, 0.9
        c = math.sqrt(GAMMA * p / rho)
        uc = euler_state(rho, v, p)
        H = (uc[2] + p) / rho
        vecs = [np.array([1.0, v - c, H - v * c]), np.array([1.0, v, 0.5 * v * v]),
                np.array([1.0, v + c, H + v * c])]
    shapes = {1: [-0.4, 0.0, 1.0], 2: [-0.3, 0.1, 0.0, 1.0, 1.2],
              3: [0.3, -0.2, 0.1, 0.0, 1.0, 1.1, 0.9]}
    sj = 1e-3 * np.array(shapes[k])
    D = uc.size
    for q, r in enumerate(vecs):
        line = np.tile(uc[:, None], (1, nx))
        for j in range(2 * k + 1):
            line[:, i - k + j] = uc + sj[j] * r
        um, up = orc.sys_recon(s, line.reshape(-1))
        want_m = uc + orc.weno_left(k, sj) * r
        want_p = uc + orc.weno_left(k, sj[::-1].copy()) * r
        np.testing.assert_allclose(um.reshape(D, nx)[:, i], want_m, rtol=0, atol=1e-11)
        np.testing.assert_allclose(up.reshape(D, nx)[:, i], want_p, rtol=0, atol=1e-11)
