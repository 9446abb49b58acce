"""Pins of the reference flux and time steppers (sec 2.1.2, 2.2) against closed
forms: the classical Lax-Friedrichs scheme, the exact upwind shift, the
Runge-Kutta stability polynomials and discrete conservation."""
import numpy as np
import pytest

from paper_2104_09404_amd import workloads as W


def test_lf_sign_reproduces_fine_lf_scheme(orc):
    """k = 0 + LF flux with alpha_LF = dx/dt + forward Euler equals the classical
    Lax-Friedrichs scheme of eq fineLF, u_i^{n+1} = (u_{i+1}+u_{i-1})/2
    - dt (f(u_{i+1}) - f(u_{i-1}))/(2 dx) (sec 3.3.1).  This fixes the sign of the
    dissipative term of eq LFflux (reading: minus)."""
    nx = 64
    dx = 1.0 / nx
    dt = 0.4 * dx
    u = W.w0_burgers_k0().u0
    s = orc.scheme(nx, flux=0, k=0, stepper=1, alpha_fixed=dx / dt)
    out = orc.phi(s, dt, u)
    f = 0.5 * u * u
    up, um = np.roll(u, -1), np.roll(u, 1)
    ref = 0.5 * (up + um) - dt * (np.roll(f, -1) - np.roll(f, 1)) / (2 * dx)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-15)


def test_upwind_cfl_one_is_an_exact_shift(orc):
    """Linear advection, k = 0, forward Euler at CFL 1: u_i^{n+1} = u_{i-1}^n, and
    after N_x steps the data return to u0."""
    nx = 64
    dx = 1.0 / nx
    u0 = W.random_lines(0, 1, nx)[0]
    s = orc.scheme(nx, flux=1, k=0, stepper=1, a=1.0)
    one = orc.phi(s, dx, u0)
    np.testing.assert_allclose(one, np.roll(u0, 1), rtol=0, atol=1e-15)
    traj = orc.serial(s, dx, nx, u0)
    np.testing.assert_allclose(traj[-1], u0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("stepper,R", [
    (1, lambda z: 1 + z),
    (2, lambda z: 1 + z + z ** 2 / 2),
    (3, lambda z: 1 + z + z ** 2 / 2 + z ** 3 / 6),
])
@pytest.mark.parametrize("theta_k", [1, 3, 7])
def test_ssprk_amplification_on_fourier_modes(orc, stepper, R, theta_k):
    """k = 0 linear advection is the circulant upwind operator L u = -c(u - S u)/dt;
    one step of eq SSPRK1/2/3 multiplies the mode e^{i theta j} by the stability
    polynomial R(z), z = -c (1 - e^{-i theta})."""
    nx = 32
    c = 0.6
    dx = 1.0 / nx
    dt = c * dx
    theta = 2 * np.pi * theta_k / nx
    j = np.arange(nx)
    phase = 0.3
    u = np.cos(theta * j + phase)
    s = orc.scheme(nx, flux=1, k=0, stepper=stepper, a=1.0)
    out = orc.phi(s, dt, u)
    z = -c * (1 - np.exp(-1j * theta))
    ref = np.real(R(z) * np.exp(1j * (theta * j + phase)))
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("k,stepper", [(0, 1), (2, 3), (2, 1), (2, 2)])
def test_conservation(orc, k, stepper):
    """Periodic finite volumes telescope (eq spaceDisc): sum_i u_i is conserved by
    every step, up to round-off."""
    nx = 128
    dx = 1.0 / nx
    u = W.shock_lines(1, 1, nx)[0]
    s = orc.scheme(nx, flux=0, k=k, stepper=stepper)
    dt = 0.4 * dx / np.max(np.abs(u))
    traj = orc.serial(s, dt, 50, u)
    sums = traj.sum(axis=1)
    assert np.max(np.abs(sums - sums[0])) < 50 * nx * 1e-16 * 4 * np.max(np.abs(u)) * 10


def test_weno5_rk3_advection_convergence(orc):
    """WENO5 + SSPRK3 for linear advection of a sine to T = 0.25 with dt ~ dx^{5/3}
    (so the time error is also fifth order) against the exact translate: order
    close to five."""
    errs = []
    ns = [16, 32, 64]
    T = 0.25
    for nx in ns:
        dx = 1.0 / nx
        nt = int(np.ceil(T / (0.5 * dx ** (5.0 / 3.0))))
        dt = T / nt
        u0 = W.cell_average_sin(nx, 1, 0.0)
        s = orc.scheme(nx, flux=1, k=2, stepper=3, a=1.0)
        traj = orc.serial(s, dt, nt, u0)
        exact = W.cell_average_sin(nx, 1, -2 * np.pi * T)
        errs.append(np.mean(np.abs(traj[-1] - exact)))
    order = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert order > 4.5, (errs, order)


def test_alpha_is_global_max_of_reconstructions(orc):
    """alpha_LF is the maximum of |lambda| over all interfaces and both sides
    (eq eigs); for Burgers lambda = u, so alpha >= max|u| for k = 0 exactly."""
    u = W.shock_lines(3, 1, 50)[0]
    _, alpha0 = orc.spatial_operator(orc.scheme(50, k=0), u)
    assert alpha0 == np.max(np.abs(u))
    _, alpha2 = orc.spatial_operator(orc.scheme(50, k=2), u)
    assert alpha2 >= 0.9 * np.max(np.abs(u))
