"""Seeded synthetic workloads (initial data, grids and MGRIT settings).

This module generates inputs only: exact cell averages of Fourier modes on a
periodic grid, seeded noise and the per-workload grid/MGRIT parameters.  It
holds none of the method's arithmetic (no reconstruction, flux, time stepping
or MGRIT step), so the GPU path and the reference implementation can both be
fed from it.

Every array comes from ``numpy.random.Generator(PCG64(seed))`` with
``seed = 210409404 + workload index``; the same call always returns the same
bits.

The paper's experiments use analytic initial conditions on [0, L) with L = 1
(sec 4); the workloads below are synthetic stand-ins of the same kind, with the
sizes of the five benchmark configurations:

  W0  burgers_k0_fe_nx64        first-order LF + forward Euler, two-level F-relaxation
  W1  burgers_weno5_nx1024      WENO5 + SSPRK3, 3-level FCF V-cycle (benchmark workload)
  W2  burgers_weno5_nx65536     WENO5 + SSPRK3, 4-level FCF V-cycle, large single problem
  W3  batched_512               512 independent Burgers / advection problems
  W4  adjoint_nx4096            WENO5 + SSPRK3 forward for the discrete adjoint

and the settings of the paper's own high-order experiment (Fig. MGRITweno):

  E4  e4_burgers_s{1,3,5,7}_{lf,roe}  N_x = 64, N_T = 400, 3-level V-cycle, m = 2
      e4_{sw,euler}_s{1,3,5,7}_{lf,roe}  the same for shallow water and Euler

A system's line holds its D components one after the other (D x N_x values).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 210409404

FLUX_BURGERS = 0
FLUX_ADVECTION = 1
FLUX_SHALLOW_WATER = 2
FLUX_EULER = 3


@dataclasses.dataclass
class Problem:
    """One conservation-law problem plus its MGRIT settings."""

    name: str
    flux: int              # 0 Burgers, 1 linear advection, 2 shallow water, 3 Euler
    k: int                 # WENO degree, order s = 2k+1 (0 first order, 2 WENO5)
    stepper: int           # 1 FE, 2 SSPRK2, 3 SSPRK3
    nx: int
    nt: int
    dt: float
    m: int
    levels: int
    relax: int             # 0 F, 1 FCF
    u0: np.ndarray
    a: float = 1.0         # advection speed, g (shallow water) or gamma (Euler)
    eps: float = 1e-6
    L: float = 1.0
    tol: float = 1e-10
    max_iter: int = 100
    cfl: Optional[float] = None
    numflux: int = 0       # 0 Lax-Friedrichs, 1 Roe with the Harten-Hyman fix
    lf_dx_dt: int = 0      # 1: the LF coefficient is dx/dt (the scheme of eq fineLF)
    coarse_integrator: int = 0  # 0 rediscretisation, 1/2 zeroth/first-order fine-integrator matching
    cycle: int = 0         # 0 V-cycle, 1 F-cycle
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def dx(self) -> float:
        return self.L / self.nx

    @property
    def T(self) -> float:
        return self.nt * self.dt

    def level_steps(self) -> List[int]:
        return [self.nt // self.m ** l for l in range(self.levels)]


def rng(index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index))


def cell_edges(nx: int, L: float = 1.0) -> np.ndarray:
    """Cell interfaces x_{i-1/2} = i*dx, i = 0..nx."""
    return np.arange(nx + 1, dtype=np.float64) * (L / nx)


def cell_average_sin(nx: int, kwave: int, phase: float, L: float = 1.0) -> np.ndarray:
    """Exact cell averages of sin(2 pi k x / L + phase) over each cell."""
    x = cell_edges(nx, L)
    w = 2.0 * math.pi * kwave / L
    c = np.cos(w * x + phase)
    return (c[:-1] - c[1:]) / (w * (L / nx))


def fourier_data(g: np.random.Generator, nx: int, nmodes: int, kmax: int, amp_max: float = 0.2,
                 mean: float = 0.5, L: float = 1.0) -> np.ndarray:
    """mean + sum of ``nmodes`` modes with distinct wave numbers in 1..kmax,
    amplitudes U(0, amp_max) and phases U(0, 2 pi)."""
    ks = g.choice(np.arange(1, kmax + 1), size=nmodes, replace=False)
    amps = g.uniform(0.0, amp_max, size=nmodes)
    phases = g.uniform(0.0, 2.0 * math.pi, size=nmodes)
    u = np.full(nx, mean, dtype=np.float64)
    for kw, a, ph in zip(ks, amps, phases):
        u += a * cell_average_sin(nx, int(kw), float(ph), L)
    return u


def dt_for_cfl(cfl: float, dx: float, speed: float) -> float:
    """Time step giving Courant number ``cfl`` for wave speed ``speed``."""
    return cfl * dx / speed


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def w0_burgers_k0(cfl_variant: bool = False) -> Problem:
    """N_x=64, N_T=256, T=0.25, first-order LF + FE, two-level, m=4, F-relaxation.
    u0 = 0.5 + 0.25 sin(2 pi x) + U(-1e-3, 1e-3) noise per cell.  With
    ``cfl_variant`` the step is set by CFL 0.5 instead of T = 0.25."""
    g = rng(0)
    nx, nt = 64, 256
    u0 = 0.5 + 0.25 * cell_average_sin(nx, 1, 0.0) + g.uniform(-1e-3, 1e-3, size=nx)
    dx = 1.0 / nx
    if cfl_variant:
        dt = dt_for_cfl(0.5, dx, float(np.max(np.abs(u0))))
    else:
        dt = 0.25 / nt
    return Problem("burgers_k0_fe_nx64", FLUX_BURGERS, 0, 1, nx, nt, dt, 4, 2, 0, u0,
                   max_iter=64, cfl=float(np.max(np.abs(u0))) * dt / dx)


def w1_burgers_weno5(nx: int = 1024, nt: int = 4096, m: int = 8, levels: int = 3) -> Problem:
    """WENO5-JS + SSPRK3 at CFL 0.8, 3-level FCF V-cycle, m=8.
    u0 = 0.5 + 4 Fourier modes, k distinct in 1..8, amplitudes U(0, 0.2)."""
    g = rng(1)
    u0 = fourier_data(g, nx, 4, 8)
    dx = 1.0 / nx
    dt = dt_for_cfl(0.8, dx, float(np.max(np.abs(u0))))
    return Problem("burgers_weno5_nx%d" % nx, FLUX_BURGERS, 2, 3, nx, nt, dt, m, levels, 1, u0,
                   max_iter=nt // m, cfl=0.8)


def w2_burgers_weno5_large(nx: int = 65536, nt: int = 16384, m: int = 16, levels: int = 4) -> Problem:
    """Large single problem: WENO5 + SSPRK3, CFL 0.8, 4-level FCF V-cycle, m=16,
    u0 = 0.5 + 16 modes with k distinct in 1..64."""
    g = rng(2)
    u0 = fourier_data(g, nx, 16, 64)
    dx = 1.0 / nx
    dt = dt_for_cfl(0.8, dx, float(np.max(np.abs(u0))))
    return Problem("burgers_weno5_nx%d" % nx, FLUX_BURGERS, 2, 3, nx, nt, dt, m, levels, 1, u0,
                   max_iter=nt // m, cfl=0.8)


def w3_batched(count: int = 512, nx_min: int = 256, nx_max: int = 8192) -> List[Problem]:
    """``count`` independent problems, alternately Burgers and linear advection
    (speed U(0.5, 1.5)); N_x log-uniform in [nx_min, nx_max] rounded to an even
    integer; N_T = 4 N_x; WENO5 + SSPRK3 at CFL U(0.3, 0.9); 2-level FCF, m=8."""
    g = rng(3)
    out = []
    for b in range(count):
        nx = int(round(math.exp(g.uniform(math.log(nx_min), math.log(nx_max))) / 2.0)) * 2
        nx = max(nx, 8)
        flux = FLUX_BURGERS if b % 2 == 0 else FLUX_ADVECTION
        a = float(g.uniform(0.5, 1.5)) if flux == FLUX_ADVECTION else 1.0
        cfl = float(g.uniform(0.3, 0.9))
        u0 = fourier_data(g, nx, 4, 8)
        speed = float(np.max(np.abs(u0))) if flux == FLUX_BURGERS else abs(a)
        dt = dt_for_cfl(cfl, 1.0 / nx, speed)
        out.append(Problem("batched_%03d" % b, flux, 2, 3, nx, 4 * nx, dt, 8, 2, 1, u0, a=a,
                           max_iter=nx // 2, cfl=cfl))
    return out


def w4_adjoint(nx: int = 4096, nt: int = 2048, ndirs: int = 16) -> Problem:
    """Adjoint workload: WENO5 + SSPRK3 at CFL 0.8, N_x=4096, N_T=2048, 3-level FCF, m=8.
    J = 0.5 ||u(T) - u_target||^2 with u_target = u0 + delta, delta = two seeded modes
    (k in 1..8, amplitude 0.02); 16 unit-norm Gaussian test directions."""
    g = rng(4)
    u0 = fourier_data(g, nx, 4, 8)
    delta = fourier_data(g, nx, 2, 8, amp_max=0.02, mean=0.0)
    dx = 1.0 / nx
    dt = dt_for_cfl(0.8, dx, float(np.max(np.abs(u0))))
    gd = rng(104)
    dirs = gd.standard_normal((ndirs, nx))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    p = Problem("adjoint_nx%d" % nx, FLUX_BURGERS, 2, 3, nx, nt, dt, 8, 3, 1, u0, max_iter=nt // 8,
                cfl=0.8)
    p.extra["u_target"] = u0 + delta
    p.extra["directions"] = dirs
    p.extra["checkpoint_every"] = 32
    return p


def e4_high_order(k: int = 2, numflux: int = 0, stepper: int = 3, max_iter: int = 20) -> Problem:
    """The high-order experiment of Fig. MGRITweno for Burgers: L = 1, T = 0.5,
    N_x = 64, N_T = 400 fine steps, 3-level V-cycle with F-relaxation and m = 2
    (N_t = 400, 200, 100 per level), u0 = (4/3) sin(2 pi x) as exact cell
    averages; the coarsest level runs at CFL (4/3)(4 dt)/dx = 0.43.  WENO degree
    k (order s = 2k+1) and the numerical flux (0 LF, 1 Roe) are the
    experiment's variables."""
    nx, nt = 64, 400
    u0 = (4.0 / 3.0) * cell_average_sin(nx, 1, 0.0)
    dt = 0.5 / nt
    name = "e4_burgers_s%d_%s" % (2 * k + 1, "roe" if numflux else "lf")
    return Problem(name, FLUX_BURGERS, k, stepper, nx, nt, dt, 2, 3, 0, u0, max_iter=max_iter,
                   tol=-1.0, cfl=(4.0 / 3.0) * dt * nx, numflux=numflux)


def e4_system(system: str, k: int = 2, numflux: int = 0, stepper: int = 3, max_iter: int = 20) -> Problem:
    """Fig. MGRITweno for a system, settings as e4_high_order: shallow water
    (g = 9.81) from h = (1 + sin(2 pi x)/2)/11, hu = 0; Euler (gamma = 5/3)
    from rho = 1, rho u = 0, E = 1 + sin(2 pi x)/2 (exact cell averages)."""
    nx, nt = 64, 400
    sn = cell_average_sin(nx, 1, 0.0)
    if system == "sw":
        u0 = np.concatenate([(1.0 + 0.5 * sn) / 11.0, np.zeros(nx)])
        flux, a, speed = FLUX_SHALLOW_WATER, 9.81, math.sqrt(9.81 * 1.5 / 11.0)
    else:
        u0 = np.concatenate([np.ones(nx), np.zeros(nx), 1.0 + 0.5 * sn])
        flux, a, speed = FLUX_EULER, 5.0 / 3.0, math.sqrt(5.0 / 3.0 * (2.0 / 3.0) * 1.5)
    dt = 0.5 / nt
    name = "e4_%s_s%d_%s" % (system, 2 * k + 1, "roe" if numflux else "lf")
    return Problem(name, flux, k, stepper, nx, nt, dt, 2, 3, 0, u0, a=a, max_iter=max_iter, tol=-1.0,
                   cfl=speed * 4 * dt * nx, numflux=numflux)


def e1_fine_matching(nx: int = 1024, nt: int = 8192, moving: bool = True, order: int = 1,
                     cycle: int = 0) -> Problem:
    """The fine-integrator-matching experiment of sec 4 (Fig. MGRITfineMatch)
    at its largest grid by default: Burgers with the first-order scheme of
    eq fineLF (LF with alpha = dx/dt, forward Euler), L = 1, T = 0.475,
    5 levels, m = 2, F-relaxation, coarse integrators matching the fine one
    to first (order 1) or zeroth order; u0 = (1 + sin 2 pi x)/2 (moving
    shock) or sin 2 pi x (stationary shock) as exact cell averages."""
    base = cell_average_sin(nx, 1, 0.0)
    u0 = 0.5 * (1.0 + base) if moving else base
    dt = 0.475 / nt
    name = "e1_matching%d_%s_nx%d" % (order, "moving" if moving else "stationary", nx)
    return Problem(name, FLUX_BURGERS, 0, 1, nx, nt, dt, 2, 5, 0, u0, max_iter=nt // 2,
                   cfl=float(np.max(np.abs(u0))) * dt * nx, lf_dx_dt=1, coarse_integrator=order + 1,
                   cycle=cycle)


def w1_stable_coarse(nx: int = 1024, nt: int = 4096, m: int = 4, levels: int = 3,
                     coarse_cfl: float = 0.8) -> Problem:
    """The 1024-cell WENO5 + SSPRK3 problem (u0 of w1_burgers_weno5) with a
    step small enough that the coarsest level runs at CFL ``coarse_cfl``:
    level 0 at coarse_cfl / m^(levels-1), so that MGRIT converges (sec 4
    finds that the coarse CFL decides convergence)."""
    pb = w1_burgers_weno5(nx=nx, nt=nt, m=m, levels=levels)
    cfl0 = coarse_cfl / float(m ** (levels - 1))
    dt = dt_for_cfl(cfl0, 1.0 / nx, float(np.max(np.abs(pb.u0))))
    return Problem("burgers_weno5_nx%d_coarse_cfl%.1f" % (nx, coarse_cfl), FLUX_BURGERS, 2, 3, nx, nt, dt, m,
                   levels, 1, pb.u0, max_iter=nt // m, cfl=cfl0)


def w2_stable_coarse(nx: int = 65536, nt: int = 16384, m: int = 16, levels: int = 3,
                     coarse_cfl: float = 0.8) -> Problem:
    """The 65536-cell problem (u0 of w2_burgers_weno5_large, N_T and m of the
    benchmark) with 3 levels and a step that puts the coarsest level at CFL
    ``coarse_cfl`` (level 0 at coarse_cfl / m^(levels-1)), so that MGRIT
    converges."""
    pb = w2_burgers_weno5_large(nx=nx, nt=nt, m=m, levels=levels)
    cfl0 = coarse_cfl / float(m ** (levels - 1))
    dt = dt_for_cfl(cfl0, 1.0 / nx, float(np.max(np.abs(pb.u0))))
    return Problem("burgers_weno5_nx%d_coarse_cfl%.1f" % (nx, coarse_cfl), FLUX_BURGERS, 2, 3, nx, nt, dt, m,
                   levels, 1, pb.u0, max_iter=nt // m, cfl=cfl0)


def w4_stable_coarse(coarse_cfl: float = 0.8) -> Problem:
    """The adjoint workload's problem (4096 cells, 2048 steps, u0 and u_target
    of w4_adjoint) with m = 4 and 3 levels and a step that puts the coarsest
    level at CFL ``coarse_cfl``, so that the MGRIT forward converges."""
    pb = w4_adjoint()
    m, levels = 4, 3
    cfl0 = coarse_cfl / float(m ** (levels - 1))
    dt = dt_for_cfl(cfl0, 1.0 / pb.nx, float(np.max(np.abs(pb.u0))))
    q = Problem("adjoint_nx%d_coarse_cfl%.1f" % (pb.nx, coarse_cfl), FLUX_BURGERS, 2, 3, pb.nx, pb.nt, dt, m,
                levels, 1, pb.u0, max_iter=pb.nt // m, cfl=cfl0)
    q.extra = dict(pb.extra)
    return q


def random_lines(index: int, nlines: int, nx: int, mean: float = 0.5, amp: float = 0.3) -> np.ndarray:
    """Independent smooth random lines (for per-line operator checks):
    mean + 4 Fourier modes per line with amplitudes up to ``amp``."""
    g = rng(1000 + index)
    out = np.empty((nlines, nx))
    for b in range(nlines):
        kmax = min(8, max(1, nx // 4))
        out[b] = fourier_data(g, nx, min(4, kmax), kmax, amp_max=amp / 2, mean=mean)
    return out


def shock_lines(index: int, nlines: int, nx: int) -> np.ndarray:
    """Lines with jumps (piecewise constant states plus noise), to exercise the
    non-smooth branch of the nonlinear weights."""
    g = rng(2000 + index)
    out = np.empty((nlines, nx))
    for b in range(nlines):
        nj = int(g.integers(1, 5))
        cuts = np.sort(g.choice(np.arange(1, nx), size=min(nj, nx - 1), replace=False))
        vals = g.uniform(-1.0, 1.5, size=len(cuts) + 1)
        line = np.empty(nx)
        start = 0
        for c, v in zip(list(cuts) + [nx], vals):
            line[start:c] = v
            start = c
        out[b] = line + g.uniform(-1e-3, 1e-3, size=nx)
    return out
