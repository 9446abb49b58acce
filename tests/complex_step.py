"""Complex-step differentiation of the scheme, for pinning the hand-written
adjoint: with the scheme evaluated in complex arithmetic,
Phi(u + i h v) = Phi(u) + i h J v + O(h^2), so Im(Phi(u + i h v)) / h is the
Jacobian-vector product to round-off for tiny h (no cancellation).  |x| and
max() act on real parts (their analytic continuation on the branch taken).

Independent of the reference oracle's code: the WENO tables are read from the
printed-table fixture (tests/golden/weno5_k2_tables.txt) and the formulas of
sec 2.1.1, 2.1.2 and 2.2 are evaluated with numpy.
"""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "weno5_k2_tables.txt")


def _tables():
    blocks, cur, scale = {}, None, {}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line[1:-1]
                blocks[cur] = []
            elif line.startswith("scale"):
                scale[cur] = float(line.split()[1])
            else:
                blocks[cur].append([float(x) for x in line.split()])
    return {k: np.array(v) / scale[k] for k, v in blocks.items()}


TAB = _tables()
C_TAB = TAB["c"]            # [r][j]
D_TAB = TAB["d"][:, 0]      # [r]
B_TAB = [TAB["B0"], TAB["B1"], TAB["B2"]]


def weno_left(v, eps):
    """v: [..., 5] complex windows u_{i-2..i+2}; stencil r = cells {i-r, i-r+2}."""
    out_num = 0
    out_den = 0
    for r in range(3):
        q = v[..., 2 - r: 5 - r]
        p = q @ C_TAB[r]
        beta = np.einsum("...a,ab,...b->...", q, B_TAB[r], q)
        a = D_TAB[r] / (eps + beta) ** 2
        out_num = out_num + a * p
        out_den = out_den + a
    return out_num / out_den


def spatial_operator(u, k, flux, a=1.0, eps=1e-6, L=1.0):
    n = u.shape[-1]
    dx = L / n
    if k == 0:
        um = u
        up = np.roll(u, -1)
    else:
        idx = np.arange(n)
        win_m = np.stack([u[(idx - 2 + j) % n] for j in range(5)], axis=-1)
        win_p = np.stack([u[(idx + 3 - j) % n] for j in range(5)], axis=-1)
        um = weno_left(win_m, eps)
        up = weno_left(win_p, eps)
    if flux == 0:
        f = lambda x: 0.5 * x * x
        lam_m, lam_p = um, up
    else:
        f = lambda x: a * x
        lam_m = np.full(n, a, dtype=u.dtype)
        lam_p = lam_m
    # alpha = max |lambda| over interfaces and sides; the first attaining it (u^- before u^+)
    cand = np.stack([lam_m, lam_p], axis=-1).reshape(-1)
    i = int(np.argmax(np.abs(cand.real)))
    alpha = cand[i] * np.sign(cand[i].real)
    F = 0.5 * (f(up) + f(um)) - 0.5 * alpha * (up - um)
    return -(F - np.roll(F, 1)) / dx


def phi(u, dt, k, flux, stepper, a=1.0, eps=1e-6):
    A = lambda x: spatial_operator(x, k, flux, a, eps)
    if stepper == 1:
        return u + dt * A(u)
    u1 = u + dt * A(u)
    if stepper == 2:
        return 0.5 * u + 0.5 * u1 + 0.5 * dt * A(u1)
    u2 = 0.75 * u + 0.25 * u1 + 0.25 * dt * A(u1)
    return u / 3.0 + 2.0 / 3.0 * u2 + 2.0 / 3.0 * dt * A(u2)


def jvp(fn, u, v, h=1e-200):
    return np.imag(fn(u.astype(np.complex128) + 1j * h * v)) / h
