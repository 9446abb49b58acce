"""Python binding of ``libmgrit.so`` (include/mgrit.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Arrays are torch tensors on the GPU (float64,
contiguous); work is enqueued on torch's current stream.  There is no CPU
fallback: importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgrit.so")

MGRIT_OK = 0
MGRIT_NOT_CONVERGED = 1
MGRIT_EINVAL = -1
MGRIT_EHIP = -2
MGRIT_EUNSUPPORTED = -4

KERNEL_CLASSES = ["phi", "relax_fc_l0", "relax_fr_l0", "relax_fc_coarse", "relax_fr_coarse", "interp",
                  "coarse_solve", "aux", "adjoint", "adjoint_recompute"]

EXPORTED = ["mgrit_phi", "mgrit_serial", "mgrit_relax", "mgrit_residual", "mgrit_workspace_bytes",
            "mgrit_cycle", "mgrit_last_error", "mgrit_set_profiling", "mgrit_get_profile",
            "mgrit_kernel_config", "mgrit_set_kernel_config", "mgrit_phi_vjp", "mgrit_checkpoints",
            "mgrit_adjoint_workspace_bytes", "mgrit_adjoint", "mgrit_tiled_config", "mgrit_set_tiled_config",
            "mgrit_batched_workspace_bytes", "mgrit_cycle_batched", "mgrit_cycle_levels",
            "mgrit_set_profiling_mask", "mgrit_autotune_scratch_bytes", "mgrit_autotune",
            "mgrit_cycle_noalloc", "mgrit_set_tiled_intervals", "mgrit_tiled_intervals", "mgrit_autotune_tiled",
            "mgrit_set_sys_tiles", "mgrit_sys_tiles", "mgrit_tiled_launch_config"]

# size of the library's static workspace of mgrit_cycle_noalloc (MGRIT_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class MgritError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libmgrit error %d: %s" % (code, msg))
        self.code = code


class Scheme(C.Structure):
    """Mirror of ``mgrit_scheme``."""

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
    """Mirror of ``mgrit_params``."""

    _fields_ = [
        ("nt", C.c_int32),
        ("m", C.c_int32),
        ("levels", C.c_int32),
        ("relax", C.c_int32),
        ("cycle", C.c_int32),
        ("max_iter", C.c_int32),
        ("init", C.c_int32),
        ("coarse_guess", C.c_int32),
        ("storage", C.c_int32),
        ("sync_every", C.c_int32),
        ("dt", C.c_double),
        ("tol", C.c_double),
        ("coarse_integrator", C.c_int32),
        ("pad2_", C.c_int32),
    ]


class Problem(C.Structure):
    """Mirror of ``mgrit_problem`` (one problem of a batch)."""

    _fields_ = [
        ("scheme", Scheme),
        ("nt", C.c_int32),
        ("pad_", C.c_int32),
        ("dt", C.c_double),
        ("u0", C.c_void_p),
        ("u", C.c_void_p),
    ]


class ProfileEntry(C.Structure):
    _fields_ = [
        ("launches", C.c_int64),
        ("ms", C.c_double),
        ("phi_lines", C.c_double),
        ("cell_steps", C.c_double),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libmgrit.so not found at %s: build it with "
                          "`python -m paper_2104_09404_amd.build`" % path)
    L = C.CDLL(path)
    vp, dp, i32, i64 = C.c_void_p, C.c_void_p, C.c_int32, C.c_int64
    S, P = C.POINTER(Scheme), C.POINTER(Params)
    L.mgrit_phi.argtypes = [S, C.c_double, dp, dp, i64, vp]
    L.mgrit_serial.argtypes = [S, C.c_double, i32, dp, dp, vp]
    L.mgrit_relax.argtypes = [S, C.c_double, i32, i32, dp, dp, i32, vp]
    L.mgrit_residual.argtypes = [S, C.c_double, i32, dp, dp, i32, i32, dp, dp, dp, dp, vp]
    L.mgrit_workspace_bytes.argtypes = [S, P]
    L.mgrit_workspace_bytes.restype = C.c_size_t
    L.mgrit_cycle.argtypes = [S, P, dp, dp, vp, C.c_size_t, C.POINTER(C.c_double), C.POINTER(C.c_int32), vp]
    L.mgrit_cycle_levels.argtypes = [S, P, dp, dp, vp, C.c_size_t, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     vp]
    L.mgrit_cycle_noalloc.argtypes = [S, P, dp, dp, C.POINTER(C.c_double), C.POINTER(C.c_int32), vp]
    L.mgrit_last_error.restype = C.c_char_p
    L.mgrit_set_profiling.argtypes = [C.c_int]
    L.mgrit_autotune_scratch_bytes.argtypes = [i32, i32]
    L.mgrit_autotune_scratch_bytes.restype = C.c_size_t
    L.mgrit_autotune.argtypes = [S, i32, i32, vp, C.c_size_t, i32, C.POINTER(i32), C.POINTER(i32),
                                 C.POINTER(C.c_float), vp]
    L.mgrit_autotune_tiled.argtypes = [S, i32, i32, vp, C.c_size_t, i32, C.POINTER(i32), C.POINTER(i32),
                                       C.POINTER(i32), C.POINTER(C.c_float), vp]
    L.mgrit_set_profiling_mask.argtypes = [C.c_uint32]
    L.mgrit_set_profiling_mask.restype = None
    L.mgrit_get_profile.argtypes = [C.POINTER(ProfileEntry), C.c_int]
    L.mgrit_kernel_config.argtypes = [i32, i32, C.POINTER(i32), C.POINTER(i32)]
    L.mgrit_set_kernel_config.argtypes = [i32, i32, i32, i32, i32]
    L.mgrit_tiled_launch_config.argtypes = [i32, i64, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.mgrit_set_sys_tiles.argtypes = [i32, i32, i32]
    L.mgrit_sys_tiles.argtypes = [S, C.POINTER(i32)]
    L.mgrit_phi_vjp.argtypes = [S, C.c_double, dp, dp, dp, i64, vp]
    L.mgrit_checkpoints.argtypes = [S, C.c_double, i32, i32, dp, dp, vp]
    L.mgrit_adjoint_workspace_bytes.argtypes = [S, i32, i32, i32]
    L.mgrit_adjoint_workspace_bytes.restype = C.c_size_t
    L.mgrit_adjoint.argtypes = [S, C.c_double, i32, i32, i32, dp, dp, dp, vp, C.c_size_t, vp]
    PR = C.POINTER(Problem)
    L.mgrit_batched_workspace_bytes.argtypes = [PR, i32, P]
    L.mgrit_batched_workspace_bytes.restype = C.c_size_t
    L.mgrit_cycle_batched.argtypes = [PR, i32, P, vp, C.c_size_t, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), vp]
    for name in EXPORTED:
        if name in ("mgrit_last_error", "mgrit_set_profiling", "mgrit_set_profiling_mask", "mgrit_workspace_bytes",
                    "mgrit_autotune_scratch_bytes",
                    "mgrit_adjoint_workspace_bytes", "mgrit_batched_workspace_bytes"):
            continue
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, allow=(MGRIT_OK,)):
    if rc not in allow:
        raise MgritError(rc, load().mgrit_last_error().decode())
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("arrays must be contiguous float64 tensors on the GPU")
    return t.data_ptr()


def _stream(stream=None) -> Optional[int]:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def scheme(nx: int, flux: int = 0, k: int = 2, stepper: int = 3, a: float = 1.0, eps: float = 1e-6,
           L: float = 1.0, alpha_fixed: float = 0.0, lf_dx_dt: int = 0, numflux: int = 0) -> Scheme:
    """k: WENO degree (order 2k+1, 0..3); numflux 0 Lax-Friedrichs, 1 Roe with
    the Harten-Hyman fix."""
    return Scheme(flux=flux, k=k, stepper=stepper, nx=nx, a=a, eps=eps, L=L, alpha_fixed=alpha_fixed,
                  lf_dx_dt=lf_dx_dt, numflux=numflux)


def shallow_water_scheme(nx: int, g: float = 9.81, **kw) -> Scheme:
    """Shallow water (flux 2, D = 2 components h, hu)."""
    return scheme(nx, flux=2, a=g, **kw)


def euler_scheme(nx: int, gamma: float = 5.0 / 3.0, **kw) -> Scheme:
    """Euler equations of an ideal gas (flux 3, D = 3 components rho, rho u, E)."""
    return scheme(nx, flux=3, a=gamma, **kw)


def ncomp(s: Scheme) -> int:
    return {2: 2, 3: 3}.get(s.flux, 1)


def line_len(s: Scheme) -> int:
    """Doubles per line or time node: the D components one after the other."""
    return ncomp(s) * s.nx


def fine_lf_scheme(nx: int, flux: int = 0, a: float = 1.0, L: float = 1.0) -> Scheme:
    """The scheme of eq fineLF: first order, forward Euler, alpha_LF = dx/dt."""
    return scheme(nx, flux=flux, k=0, stepper=1, a=a, L=L, lf_dx_dt=1)


def params(nt: int, dt: float, m: int, levels: int, relax: int = 1, cycle: int = 0, max_iter: int = 100,
           tol: float = 1e-10, init: int = 0, coarse_guess: int = 0, storage: int = 0,
           sync_every: int = 1, coarse_integrator: int = 0) -> Params:
    """coarse_integrator: 0 rediscretisation; 1 / 2 zeroth- / first-order matching
    of the fine scheme of eq fineLF on levels >= 1 (sec 3.3.1)."""
    return Params(nt=nt, m=m, levels=levels, relax=relax, cycle=cycle, max_iter=max_iter, init=init,
                  coarse_guess=coarse_guess, storage=storage, sync_every=sync_every, dt=dt, tol=tol,
                  coarse_integrator=coarse_integrator, pad2_=0)


def scheme_from_problem(pb) -> Scheme:
    return scheme(pb.nx, flux=pb.flux, k=pb.k, stepper=pb.stepper, a=pb.a, eps=pb.eps, L=pb.L,
                  numflux=getattr(pb, "numflux", 0), lf_dx_dt=getattr(pb, "lf_dx_dt", 0))


def phi(s: Scheme, dt: float, u_in, u_out, stream=None):
    """u_out[b] = Phi(u_in[b]) for every line b."""
    nlines = u_in.numel() // line_len(s)
    _check(load().mgrit_phi(C.byref(s), dt, _ptr(u_in), _ptr(u_out), nlines, _stream(stream)))


def serial(s: Scheme, dt: float, nt: int, u0, traj, stream=None):
    _check(load().mgrit_serial(C.byref(s), dt, nt, _ptr(u0), _ptr(traj), _stream(stream)))


def relax(s: Scheme, dt: float, m: int, kind: int, u, g, n: int, stream=None):
    _check(load().mgrit_relax(C.byref(s), dt, m, kind, _ptr(u), _ptr(g), n, _stream(stream)))


def residual(s: Scheme, dt: float, m: int, u, g, n: int, coarse_guess: int = 0, r=None, u_coarse=None,
             g_coarse=None, norm=None, stream=None):
    _check(load().mgrit_residual(C.byref(s), dt, m, _ptr(u), _ptr(g), n, coarse_guess, _ptr(r), _ptr(u_coarse),
                                 _ptr(g_coarse), _ptr(norm), _stream(stream)))


def workspace_bytes(s: Scheme, p: Params) -> int:
    n = load().mgrit_workspace_bytes(C.byref(s), C.byref(p))
    if n == 0:
        # surface the validation message
        raise MgritError(MGRIT_EINVAL, load().mgrit_last_error().decode())
    return n


def alloc_workspace(s: Scheme, p: Params):
    import torch

    nbytes = workspace_bytes(s, p)
    return torch.empty((nbytes + 7) // 8, dtype=torch.float64, device="cuda")


def cycle(s: Scheme, p: Params, u0, u, workspace=None, stream=None):
    """Run MGRIT; returns (status, residual history list, cycles applied)."""
    if workspace is None:
        workspace = alloc_workspace(s, p)
    hist = (C.c_double * (p.max_iter + 1))()
    iters = C.c_int32(0)
    rc = load().mgrit_cycle(C.byref(s), C.byref(p), _ptr(u0), _ptr(u), C.c_void_p(workspace.data_ptr()),
                            workspace.numel() * 8, hist, C.byref(iters), _stream(stream))
    _check(rc, allow=(MGRIT_OK, MGRIT_NOT_CONVERGED))
    n = iters.value
    nres = 1 if p.levels == 1 else n + 1
    return rc, [hist[i] for i in range(nres)], n


def cycle_noalloc(s: Scheme, p: Params, u0, u, stream=None):
    """mgrit_cycle on the library's static workspace (no allocation in the
    call); returns (status, residual history list, cycles applied)."""
    hist = (C.c_double * (p.max_iter + 1))()
    iters = C.c_int32(0)
    rc = load().mgrit_cycle_noalloc(C.byref(s), C.byref(p), _ptr(u0), _ptr(u), hist, C.byref(iters),
                                    _stream(stream))
    _check(rc, allow=(MGRIT_OK, MGRIT_NOT_CONVERGED))
    n = iters.value
    nres = 1 if p.levels == 1 else n + 1
    return rc, [hist[i] for i in range(nres)], n


def cycle_levels(schemes, p: Params, u0, u, workspace=None, stream=None):
    """MGRIT with schemes[l] on level l; returns as :func:`cycle`."""
    assert len(schemes) == p.levels
    arr = (Scheme * len(schemes))(*schemes)
    if workspace is None:
        workspace = alloc_workspace(schemes[0], p)
    hist = (C.c_double * (p.max_iter + 1))()
    iters = C.c_int32(0)
    rc = load().mgrit_cycle_levels(arr, C.byref(p), _ptr(u0), _ptr(u), C.c_void_p(workspace.data_ptr()),
                                   workspace.numel() * 8, hist, C.byref(iters), _stream(stream))
    _check(rc, allow=(MGRIT_OK, MGRIT_NOT_CONVERGED))
    n = iters.value
    nres = 1 if p.levels == 1 else n + 1
    return rc, [hist[i] for i in range(nres)], n


def autotune(s: Scheme, nlines: int, nsteps: int = 8, install: bool = True, stream=None):
    """Time every compiled one-workgroup launch shape for lines of s.nx cells
    (nlines lines, nsteps steps of Phi) and return (cells_per_thread, waves,
    ms) of the fastest; with ``install`` it becomes the override for that line
    length in the regime of ``nlines``."""
    import torch

    n = load().mgrit_autotune_scratch_bytes(s.nx, nlines)
    if n == 0:
        raise MgritError(MGRIT_EINVAL, "nx and nlines must be positive")
    scratch = torch.empty((n + 7) // 8, dtype=torch.float64, device="cuda")
    cpt, nw, ms = C.c_int32(0), C.c_int32(0), C.c_float(0.0)
    _check(load().mgrit_autotune(C.byref(s), nlines, nsteps, C.c_void_p(scratch.data_ptr()), n, 1 if install else 0,
                                 C.byref(cpt), C.byref(nw), C.byref(ms), _stream(stream)))
    return cpt.value, nw.value, ms.value


def autotune_tiled(s: Scheme, nlines: int, nsteps: int = 4, install: bool = True, stream=None):
    """Time every compiled split-line shape (cells per thread, waves, intervals
    per workgroup) on nlines lines of s.nx cells and (install) make the
    fastest the setting for that line length; returns (cpt, waves,
    intervals, ms)."""
    import torch

    nbytes = load().mgrit_autotune_scratch_bytes(s.nx, nlines)
    scratch = torch.empty(nbytes // 8 + 1, dtype=torch.float64, device="cuda")
    c, w, iv, ms = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_float(0.0)
    _check(load().mgrit_autotune_tiled(C.byref(s), nlines, nsteps, C.c_void_p(scratch.data_ptr()), nbytes,
                                       1 if install else 0, C.byref(c), C.byref(w), C.byref(iv), C.byref(ms),
                                       _stream(stream)))
    return c.value, w.value, iv.value, ms.value


def autotune_batch(problems, nsteps: int = 8, stream=None) -> dict:
    """Tune the launch shape of every distinct (nx, k, stepper) of a batch of
    (scheme, nt, dt, u0, u) problems in the throughput regime (a batch launch
    holds many lines) and install the choices; returns {nx: (cpt, waves, ms)}."""
    out = {}
    for sch, nt, dt, u0, u in problems:
        key = sch.nx
        if key in out or sch.nx > 4096:
            continue
        out[key] = autotune(sch, 512, nsteps, install=True, stream=stream)
    return out


def set_profiling(on: bool, classes=None):
    """Kernel timing on/off.  ``classes``: names from KERNEL_CLASSES whose
    launches get HIP events (default: all); the others are counted only."""
    mask = 0xFFFFFFFF if classes is None else sum(1 << KERNEL_CLASSES.index(c) for c in classes)
    load().mgrit_set_profiling_mask(mask)
    load().mgrit_set_profiling(1 if on else 0)


def get_profile() -> dict:
    arr = (ProfileEntry * len(KERNEL_CLASSES))()
    n = load().mgrit_get_profile(arr, len(KERNEL_CLASSES))
    _check(0 if n > 0 else n)
    return {KERNEL_CLASSES[i]: dict(launches=arr[i].launches, ms=arr[i].ms, phi_lines=arr[i].phi_lines,
                                    cell_steps=arr[i].cell_steps) for i in range(len(KERNEL_CLASSES))}


def kernel_config(nx: int, nlines: int = 1 << 20):
    c, w = C.c_int32(0), C.c_int32(0)
    _check(load().mgrit_kernel_config(nx, nlines, C.byref(c), C.byref(w)))
    return c.value, w.value


def set_kernel_config(nx_lo: int, nx_hi: int, cpt: int, waves: int, latency: bool = False):
    _check(load().mgrit_set_kernel_config(nx_lo, nx_hi, 1 if latency else 0, cpt, waves))


def clear_kernel_config():
    _check(load().mgrit_set_kernel_config(0, 0, 0, 0, 0))


def problem_table(problems):
    """ctypes array of mgrit_problem from (scheme, nt, dt, u0, u) tuples
    (u0, u: float64 GPU tensors)."""
    arr = (Problem * len(problems))()
    for i, (sch, nt, dt, u0, u) in enumerate(problems):
        arr[i].scheme = sch
        arr[i].nt = nt
        arr[i].dt = dt
        arr[i].u0 = _ptr(u0)
        arr[i].u = _ptr(u)
    return arr


def batched_workspace_bytes(problems, p: Params) -> int:
    arr = problems if isinstance(problems, C.Array) else problem_table(problems)
    n = load().mgrit_batched_workspace_bytes(arr, len(arr), C.byref(p))
    if n == 0:
        raise MgritError(MGRIT_EINVAL, load().mgrit_last_error().decode())
    return n


def cycle_batched(problems, p: Params, workspace=None, stream=None):
    """FAS-MGRIT on a batch of problems; returns (histories, iters, status),
    histories[i] the residual norms r_0..r_{iters[i]} of problem i."""
    import torch

    arr = problems if isinstance(problems, C.Array) else problem_table(problems)
    count = len(arr)
    if workspace is None:
        nbytes = batched_workspace_bytes(arr, p)
        workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    H = p.max_iter + 1
    hist = (C.c_double * (count * H))()
    iters = (C.c_int32 * count)()
    status = (C.c_int32 * count)()
    _check(load().mgrit_cycle_batched(arr, count, C.byref(p), C.c_void_p(workspace.data_ptr()),
                                      workspace.numel() * workspace.element_size(), hist, iters, status,
                                      _stream(stream)))
    hs = [list(hist[i * H:i * H + iters[i] + 1]) for i in range(count)]
    return hs, list(iters), list(status)


def tiled_config(nx: int):
    """(cells per thread, waves, tiles) of split lines of nx cells; tiles == 1
    when a line runs on one workgroup."""
    c, w, t = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    _check(load().mgrit_tiled_config(nx, C.byref(c), C.byref(w), C.byref(t)))
    return c.value, w.value, t.value


def tiled_launch_config(nx: int, nchunks: int, residual: bool = False):
    """(cells per thread, waves, tiles) of one split-line launch over nchunks
    chunks of lines of nx cells: launches of few chunks that form no residual
    take 1024-cell tiles (latency bound), others the tiled_config shape."""
    c, w, t = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    _check(load().mgrit_tiled_launch_config(nx, nchunks, 1 if residual else 0, C.byref(c), C.byref(w),
                                            C.byref(t)))
    return c.value, w.value, t.value


def set_tiled_config(nx_lo: int, nx_hi: int, cpt: int, waves: int):
    """Split lines of nx_lo..nx_hi cells into tiles of at most 64*waves*cpt cells."""
    _check(load().mgrit_set_tiled_config(nx_lo, nx_hi, cpt, waves))


def set_tiled_intervals(nx_lo: int, nx_hi: int, cpt: int, waves: int, intervals: int):
    """Split lines of nx_lo..nx_hi cells into tiles of (cpt, waves), each
    workgroup advancing ``intervals`` chunks (1 or 2) together."""
    _check(load().mgrit_set_tiled_intervals(nx_lo, nx_hi, cpt, waves, intervals))


def tiled_intervals(nx: int) -> int:
    n = C.c_int32(0)
    _check(load().mgrit_tiled_intervals(nx, C.byref(n)))
    return n.value


def clear_tiled_config():
    _check(load().mgrit_set_tiled_config(0, 0, 0, 0))


def set_sys_tiles(nx_lo: int, nx_hi: int, tiles: int):
    """Run system lines of nx_lo..nx_hi cells on ``tiles`` workgroups each."""
    _check(load().mgrit_set_sys_tiles(nx_lo, nx_hi, tiles))


def clear_sys_tiles():
    _check(load().mgrit_set_sys_tiles(0, 0, 0))


def sys_tiles(s: Scheme) -> int:
    """Workgroups per line of system scheme s (1: one workgroup)."""
    t = C.c_int32(0)
    _check(load().mgrit_sys_tiles(C.byref(s), C.byref(t)))
    return t.value


def phi_vjp(s: Scheme, dt: float, u, lam_in, lam_out, stream=None):
    """lam_out[b] = (dPhi/du(u[b]))^T lam_in[b] for every line b."""
    nlines = u.numel() // s.nx
    _check(load().mgrit_phi_vjp(C.byref(s), dt, _ptr(u), _ptr(lam_in), _ptr(lam_out), nlines, _stream(stream)))


def checkpoints(s: Scheme, dt: float, nt: int, every: int, u0, ckpt, stream=None):
    """Serial forward keeping nodes 0, every, ..., nt in ckpt [(nt/every)+1, nx]."""
    _check(load().mgrit_checkpoints(C.byref(s), dt, nt, every, _ptr(u0), _ptr(ckpt), _stream(stream)))


def adjoint_workspace_bytes(s: Scheme, nt: int, every: int, parallel_segments: int) -> int:
    n = load().mgrit_adjoint_workspace_bytes(C.byref(s), nt, every, parallel_segments)
    if n == 0:
        raise MgritError(MGRIT_EINVAL, load().mgrit_last_error().decode())
    return n


def adjoint(s: Scheme, dt: float, nt: int, every: int, ckpt, lambda_T, lambda_0, parallel_segments: int = 0,
            workspace=None, stream=None):
    """lambda_0 = (du^{nt}/du^0)^T lambda_T from checkpoints (reverse sweep on the GPU).
    parallel_segments = 0 recomputes all segments in one launch."""
    import torch

    nseg = nt // every
    P = parallel_segments if parallel_segments > 0 else nseg
    if workspace is None:
        nbytes = adjoint_workspace_bytes(s, nt, every, P)
        workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
    _check(load().mgrit_adjoint(C.byref(s), dt, nt, every, P, _ptr(ckpt), _ptr(lambda_T), _ptr(lambda_0),
                                C.c_void_p(workspace.data_ptr()), workspace.numel() * 8, _stream(stream)))
