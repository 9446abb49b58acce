"""ctypes wrapper around the plain C reference implementation (``mgrit_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark import this module.  The product library never does.

The shared object is compiled with gcc (``-O2 -ffp-contract=off``, no
fast-math) into ``oracle/_build/``; :func:`build` always recompiles,
:func:`lib` compiles only when nothing is built yet.  :func:`timing_phi`
and :func:`timing_mgrit` time the same source built for speed (``-O3
-march=native``, still no fast-math) on the machine they run on; only the
CPU baseline of the benchmark uses that build.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mgrit_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")
SO = os.path.join(BUILD_DIR, "libmgrit_oracle.so")

_lib = None


class Scheme(C.Structure):
    """Mirror of ``orc_scheme`` in mgrit_oracle.c."""

    _fields_ = [
        ("flux", C.c_int32),
        ("k", C.c_int32),
        ("stepper", C.c_int32),
        ("nx", C.c_int32),
        ("a", C.c_double),
        ("eps", C.c_double),
        ("L", C.c_double),
        ("alpha_fixed", C.c_double),
        ("lf_dx_dt", C.c_int32),
        ("numflux", C.c_int32),
    ]


class Params(C.Structure):
    """Mirror of ``orc_params`` in mgrit_oracle.c."""

    _fields_ = [
        ("nt", C.c_int32),
        ("m", C.c_int32),
        ("levels", C.c_int32),
        ("relax", C.c_int32),
        ("cycle", C.c_int32),
        ("max_iter", C.c_int32),
        ("init", C.c_int32),
        ("coarse_guess", C.c_int32),
        ("exact_coarse", C.c_int32),
        ("coarse_integrator", C.c_int32),
        ("dt", C.c_double),
        ("tol", C.c_double),
    ]


def build() -> str:
    """Compile the oracle shared object (always)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    tmp = SO + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
           "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(SO)
        dp = C.POINTER(C.c_double)
        L.orc_weno5_candidates.argtypes = [dp, dp]
        L.orc_weno5_beta.argtypes = [dp, dp]
        L.orc_weno5_left.argtypes = [dp, C.c_double]
        L.orc_weno5_left.restype = C.c_double
        L.orc_spatial_operator.argtypes = [C.POINTER(Scheme), dp, dp]
        L.orc_spatial_operator.restype = C.c_double
        L.orc_phi.argtypes = [C.POINTER(Scheme), C.c_double, dp, dp]
        L.orc_phi_lines.argtypes = [C.POINTER(Scheme), C.c_double, dp, dp, C.c_int64]
        L.orc_serial.argtypes = [C.POINTER(Scheme), C.c_double, C.c_int32, dp, dp]
        L.orc_psi.argtypes = [C.POINTER(Scheme), C.c_int32, C.c_int32, C.c_double, dp, dp]
        L.orc_mgrit.argtypes = [C.POINTER(Scheme), C.POINTER(Params), dp, dp, dp,
                                C.POINTER(C.c_int32)]
        L.orc_mgrit.restype = C.c_int
        L.orc_mgrit_levels.argtypes = [C.POINTER(Scheme), C.POINTER(Params), dp, dp, dp,
                                       C.POINTER(C.c_int32)]
        L.orc_mgrit_levels.restype = C.c_int
        L.orc_weno_tables.argtypes = [C.c_int32, dp, dp, dp]
        L.orc_weno_left.argtypes = [C.c_int32, dp, C.c_double]
        L.orc_weno_left.restype = C.c_double
        L.orc_roe_flux.argtypes = [C.POINTER(Scheme), C.c_double, C.c_double]
        L.orc_roe_flux.restype = C.c_double
        L.orc_ncomp.argtypes = [C.POINTER(Scheme)]
        L.orc_ncomp.restype = C.c_int
        L.orc_sys_flux.argtypes = [C.POINTER(Scheme), dp, dp]
        L.orc_sys_eig.argtypes = [C.POINTER(Scheme), dp, dp, dp, dp]
        L.orc_sys_roe_eig.argtypes = [C.POINTER(Scheme), dp, dp, dp, dp, dp]
        L.orc_sys_roe_flux.argtypes = [C.POINTER(Scheme), dp, dp, dp]
        L.orc_sys_recon.argtypes = [C.POINTER(Scheme), dp, dp, dp]
        L.orc_weno5_left_grad.argtypes = [dp, C.c_double, dp]
        L.orc_spatial_operator_vjp.argtypes = [C.POINTER(Scheme), dp, dp, dp]
        L.orc_phi_vjp.argtypes = [C.POINTER(Scheme), C.c_double, dp, dp, dp]
        L.orc_serial_adjoint.argtypes = [C.POINTER(Scheme), C.c_double, C.c_int32, dp, dp, dp]
        L.orc_serial_adjoint.restype = C.c_double
        _lib = L
    return _lib


TIMING_FLAGS = ["-O3", "-march=native", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]


_timing_lib = None


def timing_lib():
    """The oracle source built for speed (flags TIMING_FLAGS, on the host that
    runs this) in a temporary directory, once per process.  Only the timing
    entry points are declared; parity uses lib()."""
    global _timing_lib
    if _timing_lib is None:
        import tempfile

        tmp = tempfile.mkdtemp(prefix="oracle_timing_")
        so = os.path.join(tmp, "libmgrit_oracle_timing.so")
        subprocess.run(["gcc"] + TIMING_FLAGS + ["-o", so, SRC, "-lm"], check=True)
        L = C.CDLL(so)
        dp = C.POINTER(C.c_double)
        L.orc_phi_lines.argtypes = [C.POINTER(Scheme), C.c_double, dp, dp, C.c_int64]
        L.orc_mgrit.argtypes = [C.POINTER(Scheme), C.POINTER(Params), dp, dp, dp, C.POINTER(C.c_int32)]
        L.orc_mgrit.restype = C.c_int
        _timing_lib = L
    return _timing_lib


def timing_mgrit(s: Scheme, p: Params, u0):
    """One call of the oracle's FAS-MGRIT (the same algorithm as mgrit()) in
    the build of timing_lib(), from the zero initial iterate.  Returns
    (seconds, cycles applied, last residual norm, compiler flags)."""
    import time

    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    u = np.zeros((p.nt + 1, line_len(s)))
    hist = np.full(p.max_iter + 1, np.nan)
    iters = C.c_int32(0)
    L = timing_lib()
    t0 = time.perf_counter()
    L.orc_mgrit(C.byref(s), C.byref(p), _p(u0), _p(u), _p(hist), C.byref(iters))
    el = time.perf_counter() - t0
    n = iters.value
    return el, n, float(hist[n]) if p.levels > 1 else float("nan"), " ".join(["gcc"] + TIMING_FLAGS)


def timing_phi(s: Scheme, dt: float, lines: np.ndarray, budget_s: float):
    """Apply Phi to every row of ``lines`` repeatedly, for about ``budget_s``
    seconds, in the build of timing_lib().  Returns (repetitions, seconds,
    compiler flags)."""
    import time

    L = timing_lib()
    a = np.ascontiguousarray(lines, dtype=np.float64)
    b = np.zeros_like(a)
    nlines = a.size // line_len(s)
    reps = 0
    t0 = time.perf_counter()
    while True:
        L.orc_phi_lines(C.byref(s), dt, _p(a), _p(b), nlines)
        a, b = b, a
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    return reps, el, " ".join(["gcc"] + TIMING_FLAGS)


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def scheme(nx, flux=0, k=2, stepper=3, a=1.0, eps=1e-6, L=1.0, alpha_fixed=0.0, lf_dx_dt=0,
           numflux=0) -> Scheme:
    """k: WENO degree (order s = 2k+1); numflux 0 Lax-Friedrichs, 1 Roe with
    the Harten-Hyman fix (sec 2.1.3)."""
    return Scheme(flux=flux, k=k, stepper=stepper, nx=nx, a=a, eps=eps, L=L,
                  alpha_fixed=alpha_fixed, lf_dx_dt=lf_dx_dt, numflux=numflux)


def fine_lf_scheme(nx, flux=0, a=1.0, L=1.0) -> Scheme:
    """The scheme of eq fineLF: first order, forward Euler, alpha_LF = dx/dt."""
    return scheme(nx, flux=flux, k=0, stepper=1, a=a, L=L, lf_dx_dt=1)


def params(nt, dt, m, levels, relax=0, cycle=0, max_iter=100, tol=1e-10, init=0,
           coarse_guess=0, exact_coarse=0, coarse_integrator=0) -> Params:
    """coarse_integrator: 0 rediscretisation, 1 zeroth-order and 2 first-order
    fine-integrator matching (sec 3.3.1) on levels >= 1."""
    return Params(nt=nt, m=m, levels=levels, relax=relax, cycle=cycle, max_iter=max_iter,
                  init=init, coarse_guess=coarse_guess, exact_coarse=exact_coarse,
                  coarse_integrator=coarse_integrator, dt=dt, tol=tol)


def weno5_candidates(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_weno5_candidates(_p(v), _p(out))
    return out


def weno5_beta(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_weno5_beta(_p(v), _p(out))
    return out


def weno5_left(v, eps=1e-6):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_weno5_left(_p(v), eps)


def shallow_water_scheme(nx, g=9.81, **kw) -> Scheme:
    """Shallow water (D = 2, eq shallowWater); reading R20 for g."""
    return scheme(nx, flux=2, a=g, **kw)


def euler_scheme(nx, gamma=5.0 / 3.0, **kw) -> Scheme:
    """Euler equations of an ideal monatomic gas (D = 3, eq Euler)."""
    return scheme(nx, flux=3, a=gamma, **kw)


def ncomp(s: Scheme) -> int:
    return {2: 2, 3: 3}.get(s.flux, 1)


def line_len(s: Scheme) -> int:
    """Doubles per time node: the D components one after the other, nx each."""
    return ncomp(s) * s.nx


def sys_flux(s: Scheme, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(ncomp(s))
    lib().orc_sys_flux(C.byref(s), _p(u), _p(f))
    return f


def sys_eig(s: Scheme, u):
    """(eigenvalues, R, L = R^-1) of the flux Jacobian at the conserved state u."""
    D = ncomp(s)
    u = np.ascontiguousarray(u, dtype=np.float64)
    lam, R, L = np.zeros(D), np.zeros((D, D)), np.zeros((D, D))
    lib().orc_sys_eig(C.byref(s), _p(u), _p(lam), _p(R), _p(L))
    return lam, R, L


def sys_roe_eig(s: Scheme, uL, uR):
    D = ncomp(s)
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    lam, R, L = np.zeros(D), np.zeros((D, D)), np.zeros((D, D))
    lib().orc_sys_roe_eig(C.byref(s), _p(uL), _p(uR), _p(lam), _p(R), _p(L))
    return lam, R, L


def sys_roe_flux(s: Scheme, uL, uR):
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    F = np.zeros(ncomp(s))
    lib().orc_sys_roe_flux(C.byref(s), _p(uL), _p(uR), _p(F))
    return F


def sys_recon(s: Scheme, u):
    """(um, up) with um[d, i] = u^-_{i+1/2} and up[d, i] = u^+_{i-1/2} of cell i."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    um, up = np.zeros(u.size), np.zeros(u.size)
    lib().orc_sys_recon(C.byref(s), _p(u), _p(um), _p(up))
    return um.reshape(ncomp(s), s.nx), up.reshape(ncomp(s), s.nx)


def weno_tables(k):
    """(c [k+1, k+1], d [k+1], B [k+1, k+1, k+1]) of degree k, computed from
    their definitions (eq C, B, D)."""
    n1 = k + 1
    c, d, B = np.zeros((n1, n1)), np.zeros(n1), np.zeros((n1, n1, n1))
    lib().orc_weno_tables(k, _p(c), _p(d), _p(B))
    return c, d, B


def weno_left(k, v, eps=1e-6):
    """u^-_{i+1/2} of degree k from v = u_{i-k} .. u_{i+k}."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.size == 2 * k + 1
    return lib().orc_weno_left(k, _p(v), eps)


def roe_flux(s: Scheme, um, up):
    """Roe flux with the Harten-Hyman fix at one interface (eq roeflux)."""
    return lib().orc_roe_flux(C.byref(s), float(um), float(up))


def spatial_operator(s: Scheme, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    A = np.zeros_like(u)
    assert u.size == line_len(s)
    alpha = lib().orc_spatial_operator(C.byref(s), _p(u), _p(A))
    return A, alpha


def phi(s: Scheme, dt, u):
    """Phi applied to every row of ``u`` (shape [..., nx])."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    nlines = u.size // line_len(s)
    lib().orc_phi_lines(C.byref(s), dt, _p(u), _p(out), nlines)
    return out


def psi(s: Scheme, order, M, dt, u):
    """Coarse integrator matching M fine steps of eq fineLF (fine step dt),
    order 0 (eq coarseLFord0) or 1 (eq coarseLFord1, eq fineLFxM)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    lib().orc_psi(C.byref(s), order, M, dt, _p(u), _p(out))
    return out


def serial(s: Scheme, dt, nt, u0):
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    traj = np.zeros((nt + 1, line_len(s)))
    lib().orc_serial(C.byref(s), dt, nt, _p(u0), _p(traj))
    return traj


def mgrit(s: Scheme, p: Params, u0, u_init=None):
    """Run FAS-MGRIT; returns (u [(nt+1) x nx], residual history, cycles applied, status)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    u = np.zeros((p.nt + 1, line_len(s)))
    if u_init is not None:
        u[...] = u_init
    hist = np.full(p.max_iter + 1, np.nan)
    iters = C.c_int32(0)
    st = lib().orc_mgrit(C.byref(s), C.byref(p), _p(u0), _p(u), _p(hist), C.byref(iters))
    n = iters.value
    return u, hist[: n + 1] if p.levels > 1 else hist[:1], n, st


def mgrit_levels(schemes, p: Params, u0, u_init=None):
    """FAS-MGRIT with schemes[l] on level l; returns as :func:`mgrit`."""
    assert len(schemes) == p.levels
    arr = (Scheme * len(schemes))(*schemes)
    nx = line_len(schemes[0])
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    u = np.zeros((p.nt + 1, nx))
    if u_init is not None:
        u[...] = u_init
    hist = np.full(p.max_iter + 1, np.nan)
    iters = C.c_int32(0)
    st = lib().orc_mgrit_levels(arr, C.byref(p), _p(u0), _p(u), _p(hist), C.byref(iters))
    n = iters.value
    return u, hist[: n + 1] if p.levels > 1 else hist[:1], n, st


def weno5_left_grad(v, eps=1e-6):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(5)
    lib().orc_weno5_left_grad(_p(v), eps, _p(out))
    return out


def spatial_operator_vjp(s: Scheme, u, v):
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros_like(u)
    lib().orc_spatial_operator_vjp(C.byref(s), _p(u), _p(v), _p(out))
    return out


def phi_vjp(s: Scheme, dt, u, lam):
    """(dPhi/du(u))^T lam for one step."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros_like(u)
    lib().orc_phi_vjp(C.byref(s), dt, _p(u), _p(lam), _p(out))
    return out


def serial_adjoint(s: Scheme, dt, nt, u0, u_target):
    """(J, dJ/du0) for J = 1/2 ||u(T) - u_target||^2 with serial time stepping."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    ut = np.ascontiguousarray(u_target, dtype=np.float64)
    g = np.zeros_like(u0)
    J = lib().orc_serial_adjoint(C.byref(s), dt, nt, _p(u0), _p(ut), _p(g))
    return J, g
