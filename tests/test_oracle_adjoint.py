"""Pins of the reference discrete adjoint (the derivative of sec 2.1-2.2, written
by hand): complex-step Jacobian-vector products of an independent evaluation of
the scheme (dot-product test), central finite differences of the serial solve,
a Taylor test, and the exact transpose of the closed-form linear upwind step."""
import numpy as np
import pytest

import complex_step as CS
from paper_2104_09404_amd import workloads as W


def test_weno_gradient_matches_complex_step(orc):
    g = np.random.default_rng(0)
    wins = list(g.uniform(-1, 1, (50, 5))) + list(W.shock_lines(9, 20, 5))
    for w in wins:
        grad = orc.weno5_left_grad(w, 1e-6)
        for j in range(5):
            e = np.zeros(5)
            e[j] = 1.0
            ref = np.imag(CS.weno_left((w + 1e-200j * e)[None, :], 1e-6))[0] / 1e-200
            assert abs(grad[j] - ref) <= 1e-11 * max(1.0, abs(ref)), (w, j, grad[j], ref)


@pytest.mark.parametrize("k", [0, 2])
@pytest.mark.parametrize("flux", [0, 1])
def test_operator_vjp_dot_product(orc, k, flux):
    """<J_A v, w> = <v, J_A^T w> with J_A v from the complex step."""
    nx = 40
    a = 0.8
    s = orc.scheme(nx, flux=flux, k=k, a=a)
    g = np.random.default_rng(1 + k + flux)
    for u in (W.random_lines(5, 1, nx)[0], W.shock_lines(5, 1, nx)[0]):
        v = g.standard_normal(nx)
        w = g.standard_normal(nx)
        Jv = CS.jvp(lambda x: CS.spatial_operator(x, k, flux, a), u, v)
        JTw = orc.spatial_operator_vjp(s, u, w)
        lhs, rhs = Jv @ w, v @ JTw
        scale = np.linalg.norm(Jv) * np.linalg.norm(w) + np.linalg.norm(v) * np.linalg.norm(JTw)
        assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)


@pytest.mark.parametrize("stepper", [1, 2, 3])
@pytest.mark.parametrize("k", [0, 2])
def test_phi_vjp_dot_product(orc, stepper, k):
    nx = 32
    s = orc.scheme(nx, k=k, stepper=stepper)
    g = np.random.default_rng(7 * stepper + k)
    u = W.random_lines(11, 1, nx)[0]
    dt = 0.5 / nx / np.max(np.abs(u))
    for _ in range(3):
        v = g.standard_normal(nx)
        w = g.standard_normal(nx)
        Jv = CS.jvp(lambda x: CS.phi(x, dt, k, 0, stepper), u, v)
        JTw = orc.phi_vjp(s, dt, u, w)
        scale = np.linalg.norm(Jv) * np.linalg.norm(w) + np.linalg.norm(v) * np.linalg.norm(JTw)
        assert abs(Jv @ w - v @ JTw) <= 1e-13 * scale


def test_upwind_vjp_is_exact_transpose(orc):
    """k = 0 advection: Phi is the closed-form matrix sum_j Z^j/j!, Z = -c(I - S)."""
    nx = 16
    c = 0.45
    dt = c / nx
    S = np.roll(np.eye(nx), 1, axis=0)
    Z = -c * (np.eye(nx) - S)
    Phi = np.eye(nx) + Z + Z @ Z / 2 + Z @ Z @ Z / 6
    s = orc.scheme(nx, flux=1, k=0, stepper=3, a=1.0)
    u = W.random_lines(2, 1, nx)[0]
    for j in range(nx):
        e = np.zeros(nx)
        e[j] = 1.0
        np.testing.assert_allclose(orc.phi_vjp(s, dt, u, e), Phi.T @ e, atol=1e-15)


def test_serial_adjoint_matches_finite_differences(orc):
    """dJ/du0 against central differences, h = 1e-6, on random unit directions
    (the adjoint workload's recipe at a reduced size)."""
    nx, nt = 64, 40
    pb = W.w4_adjoint(nx=nx, nt=nt, ndirs=4)
    s = orc.scheme(nx)
    J, grad = orc.serial_adjoint(s, pb.dt, nt, pb.u0, pb.extra["u_target"])
    for d in pb.extra["directions"]:
        h = 1e-6
        Jp, _ = orc.serial_adjoint(s, pb.dt, nt, pb.u0 + h * d, pb.extra["u_target"])
        Jm, _ = orc.serial_adjoint(s, pb.dt, nt, pb.u0 - h * d, pb.extra["u_target"])
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - grad @ d) <= 1e-6 * max(abs(fd), 1e-12), (fd, grad @ d)


def test_taylor_remainder_is_second_order(orc):
    nx, nt = 48, 20
    pb = W.w4_adjoint(nx=nx, nt=nt, ndirs=1)
    s = orc.scheme(nx)
    J, grad = orc.serial_adjoint(s, pb.dt, nt, pb.u0, pb.extra["u_target"])
    d = pb.extra["directions"][0]
    rem = []
    hs = [2e-3, 1e-3, 5e-4]
    for h in hs:
        Jh, _ = orc.serial_adjoint(s, pb.dt, nt, pb.u0 + h * d, pb.extra["u_target"])
        rem.append(abs(Jh - J - h * (grad @ d)))
    order = np.polyfit(np.log(hs), np.log(rem), 1)[0]
    assert 1.8 < order < 2.2, (rem, order)
