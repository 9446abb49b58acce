/*
 * mgrit.h -- C ABI of the MI355X (gfx950) MGRIT library for non-linear 1D
 * scalar conservation laws (Danieli & MacLachlan, "Multigrid Reduction in
 * Time for non-linear hyperbolic equations", arXiv 2104.09404).
 *
 * Problem (sec 2, eq consLaw): u_t + f(u)_x = 0 on [0, L), periodic, N_x
 * cells of width dx = L/N_x holding cell averages (sec 2.1); N_T fine time
 * steps of size dt, nodes n = 0..N_T, node 0 the initial condition.
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers to contiguous FP64 data owned by
 *     the caller (e.g. torch tensors).  The library never allocates or frees
 *     caller memory, and allocates no device memory of its own: split lines
 *     outside a workspace-taking call synchronise through a static 10.5 MB
 *     device array (one per device, held while the library is loaded;
 *     concurrent split-line calls on one device share it, so they must not
 *     overlap).
 *   - Line length.  Lines of up to 4096 cells run on one workgroup each.
 *     Longer lines (or any range chosen with mgrit_set_tiled_config) are split
 *     into tiles of balanced length, one workgroup per tile, which exchange
 *     alpha_LF and their edge fluxes once per Runge-Kutta stage through
 *     device memory; their launches are
 *     cooperative (all workgroups of a line resident at once).  The tile
 *     shape follows the line length (mgrit_tiled_config) and, for launches
 *     of few chunks, the launch (mgrit_tiled_launch_config).  Results are
 *     bitwise the same as with one workgroup per line.  Split-line calls
 *     outside mgrit_cycle that overlap in time on one device (different
 *     streams or threads) share that device's synchronisation buffer and must
 *     not run concurrently.
 *   - A "line" is N_x consecutive doubles (one spatial grid function).  A
 *     level array holds lines for nodes 0..N, node n at offset n*N_x: the
 *     space-time iterate is stored time-major, contiguous in x.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on that stream and returns, except where stated.
 *   - Return codes: MGRIT_OK (0); MGRIT_NOT_CONVERGED (1, mgrit_cycle only);
 *     MGRIT_EINVAL (-1) invalid argument, nothing enqueued; MGRIT_EHIP (-2) a
 *     HIP runtime error; MGRIT_EUNSUPPORTED (-4) valid but not supported
 *     (e.g. a line longer than the largest kernel configuration).  The
 *     message of the last failure on the calling thread is returned by
 *     mgrit_last_error().
 *   - Arithmetic is IEEE FP64 throughout.  max() ignores NaN, so a line that
 *     overflows (an unstable coarse integrator) never poisons alpha_LF of
 *     another line; non-finite residual norms count as "not converged".
 *   - Calls are not thread safe with respect to mgrit_set_profiling /
 *     mgrit_get_profile; everything else is reentrant.
 */
#ifndef MGRIT_H
#define MGRIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MGRIT_OK = 0,
    MGRIT_NOT_CONVERGED = 1,
    MGRIT_EINVAL = -1,
    MGRIT_EHIP = -2,
    MGRIT_EUNSUPPORTED = -4
};

/*
 * The fine propagator Phi (sec 2.1 - 2.2).
 *   flux     0: Burgers f(u) = u^2/2, lambda = u (eq burgers);
 *            1: linear advection f(u) = a u, lambda = a;
 *            2: shallow water (eq shallowWater), D = 2 components (h, hu),
 *               gravitational constant a;
 *            3: Euler (eq Euler), D = 3 components (rho, rho u, E), ideal gas
 *               with ratio of specific heats a (the paper uses 5/3).
 *            A system's time node is D x nx doubles, its components one after
 *            the other (component d of cell i at d nx + i); every array of
 *            the calls below then has D nx doubles per line or node.  Systems
 *            reconstruct characteristic-wise on the eigenvectors of the
 *            central cell's state (sec 2.1.1), take alpha_LF as the largest
 *            |lambda_k| (eq eigs) and, with the Roe flux, Roe averages
 *            (sec 2.1.3; u and H weighted by sqrt(h) or sqrt(rho)) and
 *            alpha_k = l_k . (u+ - u-) with the left eigenvectors.  Lines
 *            of up to 512 cells run on one workgroup, longer ones (up to
 *            65536 cells) on split lines of at most 510 cells per tile, with
 *            bitwise the same results (mgrit_set_sys_tiles); batches, the
 *            adjoint, the autotuner and fine-integrator matching cover scalar
 *            laws only (MGRIT_EUNSUPPORTED / MGRIT_EINVAL).
 *   k        WENO polynomial degree (sec 2.1.1), order s = 2k+1: 0 = piecewise
 *            constant (u^-_{i+1/2} = u_i, u^+_{i+1/2} = u_{i+1}); 1 = WENO3;
 *            2 = WENO5-JS with the printed k = 2 tables; 3 = WENO7.  Stencil
 *            r = {i-r, ..., i-r+k}; for k = 1 and 3 the tables of eq C, B and D
 *            are those their definitions give (the paper prints k = 2 only).
 *            Split lines keep k + 1 ghost cells per tile side for k = 3
 *            (3 otherwise).
 *   stepper  1: forward Euler (eq SSPRK1); 2: SSPRK2; 3: SSPRK3 (eq SSPRK3).
 *   nx       number of cells N_x >= 8.
 *   a        flux parameter: advection speed (flux 1), g (flux 2), gamma (flux 3).
 *   eps      WENO epsilon of eq omega (> 0; the paper uses 1e-6).
 *   L        domain length (> 0); dx = L/nx.
 *   lf_dx_dt 1: the Lax-Friedrichs coefficient is dx/dt of the step being
 *            taken (with k = 0 and forward Euler this is the scheme of eq
 *            fineLF, and rediscretised on a coarse level eq coarseLF);
 *            overrides alpha_fixed.  0: see alpha_fixed.
 *   alpha_fixed  > 0: use this Lax-Friedrichs coefficient; 0: the global
 *            alpha_LF = max over all interfaces and both sides of
 *            |lambda(u^{+-})| of eq eigs, recomputed at every RK stage of every
 *            line.  The LF flux is F = (f(u^-)+f(u^+))/2 - alpha (u^+ - u^-)/2
 *            (eq LFflux with the dissipative sign that makes it the
 *            Lax-Friedrichs scheme of eq fineLF).
 *   numflux  0: Lax-Friedrichs (eq LFflux).  1: Roe with the Harten-Hyman
 *            entropy fix (sec 2.1.3, eq roeflux):
 *            F = (f(u^-)+f(u^+))/2 - q_H(lh) (u^+ - u^-)/2 with the Roe speed
 *            lh = (f(u^+)-f(u^-))/(u^+-u^-) (u_hat = (u^-+u^+)/2 for Burgers,
 *            a for advection), q_H = (lh^2/delta + delta)/2 when |lh| < delta
 *            and |lh| otherwise, delta = max(0, lh - lambda(u^-),
 *            lambda(u^+) - lh).  With 1, alpha_fixed and lf_dx_dt must be 0.
 */
typedef struct {
    int32_t flux;
    int32_t k;
    int32_t stepper;
    int32_t nx;
    double a;
    double eps;
    double L;
    double alpha_fixed;
    int32_t lf_dx_dt;
    int32_t numflux;
} mgrit_scheme;

/*
 * MGRIT settings (sec 3.2, Alg. 1).
 *   nt        number of fine steps N_T >= 1.
 *   m         coarsening factor >= 2; N_T must be divisible by m^(levels-1).
 *   levels    1..16.  Level l has N_l = N_T/m^l steps of size m^l dt; the
 *             coarse integrators are the same scheme with that step
 *             (rediscretisation).  levels == 1 is serial time stepping.
 *   relax     0: F-relaxation; 1: FCF-relaxation (eq relaxation).
 *   cycle     0: V-cycle (Alg. 1); 1: F-cycle (Fig. MGcycles).
 *   max_iter  maximum number of cycles (>= 0).
 *   init      0: the initial iterate is u^n = u0 at every node;
 *             1: the caller's u is the initial iterate (resume).
 *   coarse_guess 0: coarse initial guess of eq restriction::u;
 *             1: plain injection.
 *   storage   0: u holds every level-0 node, (nt+1) lines;
 *             1: u holds the level-0 C-points only, (nt/m+1) lines.
 *   sync_every  check convergence on the host every this many cycles
 *             (>= 1; work enqueued after convergence is skipped on the GPU).
 *   dt        fine step (> 0, finite).
 *   tol       stop when the residual norm is < tol; tol < 0 runs exactly
 *             max_iter cycles.
 *   coarse_integrator  integrator of the levels l >= 1 (sec 3.3): 0
 *             rediscretisation (the scheme with step m^l dt); 1 zeroth-order
 *             (eq coarseLFord0) or 2 first-order (eq coarseLFord1) matching of
 *             M = m^l steps of the fine scheme (eq fineLFxM), for the fine
 *             scheme of eq fineLF only (k = 0, stepper 1, lf_dx_dt = 1); on
 *             split lines each application of the average or the difference
 *             exchanges the tiles' edge cells.
 */
typedef struct {
    int32_t nt;
    int32_t m;
    int32_t levels;
    int32_t relax;
    int32_t cycle;
    int32_t max_iter;
    int32_t init;
    int32_t coarse_guess;
    int32_t storage;
    int32_t sync_every;
    double dt;
    double tol;
    int32_t coarse_integrator;
    int32_t pad2_;
} mgrit_params;

/*
 * mgrit_phi -- one application of the fine propagator to independent lines
 * (sec 2.2; Phi of eq monolithicSystem):  u_out[b] = Phi(u_in[b]) with step
 * dt, for b = 0..nlines-1.  u_in, u_out: nlines x nx, may not overlap.
 * nlines == 0 is a no-op.  Errors: EINVAL on a bad scheme, dt <= 0, a null
 * pointer with nlines > 0, or nlines > 2^31-1.
 */
int mgrit_phi(const mgrit_scheme* s, double dt, const double* u_in, double* u_out,
              int64_t nlines, void* stream);

/*
 * mgrit_serial -- serial time stepping, the forward block substitution of
 * eq monolithicSystem: traj[0] = u0, traj[n+1] = Phi(traj[n]), n < nt.
 * u0: nx; traj: (nt+1) x nx.  One workgroup steps the line.
 */
int mgrit_serial(const mgrit_scheme* s, double dt, int32_t nt, const double* u0, double* traj,
                 void* stream);

/*
 * mgrit_relax -- relaxation on one level (eq relaxation, sec 3.2):
 *   kind 0 (F): for every chunk c, u^{cm+j} = Phi(u^{cm+j-1}) + g^{cm+j}, j = 1..m-1;
 *   kind 1 (C): u^{cm} = Phi(u^{cm-1}) + g^{cm}, c = 1..n/m;
 *   kind 2 (FCF): F, then C, then F.
 * u: (n+1) x nx level array, updated in place; g: (n+1) x nx right-hand side
 * of the level, or NULL for g^j = 0 (level 0, j >= 1; g^0 is never read).
 * dt is the step of this level; n % m == 0.  All chunks run concurrently.
 */
int mgrit_relax(const mgrit_scheme* s, double dt, int32_t m, int32_t kind, double* u,
                const double* g, int32_t n, void* stream);

/*
 * mgrit_residual -- C-point residual and FAS restriction of one level
 * (rows of eq monolithicSystem; eq restrictionOperator, FAScorrection,
 * restriction::rhs, restriction::u).  For i = 1..n/m:
 *   t_i   = Phi_l(u^{mi-1}) + g^{mi}                      (step dt)
 *   r_i   = t_i - u^{mi}                                  -> r[i-1]      (optional)
 *   u_c^i = t_i  (coarse_guess 0) or u^{mi} (coarse_guess 1) -> u_coarse[i] (optional)
 *   g_c^i = t_i - Phi_{l+1}(u^{m(i-1)})                   -> g_coarse[i] (optional, step m*dt)
 * and u_coarse[0] = u^0, g_coarse[0] = g^0 (g^0 = u^0 when g is NULL).
 * u: (n+1) x nx with its F-points relaxed; g: as in mgrit_relax.
 * r: (n/m) x nx; u_coarse, g_coarse: (n/m+1) x nx; each may be NULL.
 * norm: DEVICE scalar, if non-NULL receives ||r||_2 over all C-points and
 * cells (requires r); the sum is taken in a fixed order, so repeated calls
 * give identical bits.  No synchronisation.
 */
int mgrit_residual(const mgrit_scheme* s, double dt, int32_t m, const double* u, const double* g,
                   int32_t n, int32_t coarse_guess, double* r, double* u_coarse, double* g_coarse,
                   double* norm, void* stream);

/*
 * mgrit_workspace_bytes -- device workspace needed by mgrit_cycle: the
 * coarse level arrays u_l, g_l (l >= 1), a side buffer for the concurrent
 * C-relaxation, residual partial sums and the on-device residual history.
 * Returns 0 for invalid arguments.
 */
size_t mgrit_workspace_bytes(const mgrit_scheme* s, const mgrit_params* p);

/*
 * mgrit_cycle -- FAS-MGRIT iterations (sec 3.2, Alg. 1) to ||r|| < tol or
 * max_iter cycles.  For k = 0, 1, ...: the first level-0 sweep of the next
 * cycle F-relaxes the current iterate and yields r_k, the residual
 * Phi_0(u^{mi-1}) - u^{mi} over all level-0 C-points; if ||r_k|| < tol or
 * k == max_iter the iteration stops (the returned iterate then has its
 * F-points relaxed from its C-points), otherwise the cycle is completed
 * (restriction, coarse levels, coarsest serial solve, ideal interpolation).
 * The level-0 F-relaxation of interpolation is left to the next cycle's
 * first sweep (sec 3.2 notes it is redundant before pre-relaxation).
 *   u0        nx, the initial condition (g^0 of eq monolithicSystem).
 *   u         level-0 iterate, layout per p->storage; in/out.
 *   workspace device scratch of at least mgrit_workspace_bytes(s, p) bytes,
 *             256-byte aligned, owned by the caller, not shared by
 *             concurrent calls.
 *   res_hist  HOST array of max_iter+1 doubles: ||r_0||, ..., ||r_iters||.
 *   iters     HOST: number of cycles applied.
 * Synchronises the stream every p->sync_every cycles and at the end.
 * Returns MGRIT_OK if converged, MGRIT_NOT_CONVERGED otherwise.
 */
int mgrit_cycle(const mgrit_scheme* s, const mgrit_params* p, const double* u0, double* u,
                void* workspace, size_t ws_bytes, double* res_hist, int32_t* iters, void* stream);

/*
 * mgrit_cycle_noalloc -- mgrit_cycle for callers that cannot allocate device
 * or pinned host memory (serving loops, harnesses that forbid hipMalloc).
 * The workspace is a static device array of MGRIT_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that the library holds on every device it runs on until the
 * process ends; the call allocates nothing: no hipMalloc, no pinned host
 * buffer (the stop flag is read into host stack memory), no profiling events
 * (with profiling on, its launches are counted without timing).  Arguments,
 * synchronisation, iterates and return codes are those of mgrit_cycle with
 * the workspace argument dropped.  Problems whose mgrit_workspace_bytes(s, p)
 * exceeds MGRIT_NOALLOC_SCRATCH_BYTES return MGRIT_EINVAL before any device
 * work.  Every call on one device shares that device's array, which keeps
 * the last call's contents (the call clears what must start at zero):
 * calls that overlap in time on one device race and must not be issued.
 */
#define MGRIT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mgrit_cycle_noalloc(const mgrit_scheme* s, const mgrit_params* p, const double* u0, double* u,
                        double* res_hist, int32_t* iters, void* stream);

/*
 * mgrit_cycle_levels -- mgrit_cycle with the scheme schemes[l] on level l
 * (sec 4, Fig. MGRITweno_diffOrd: the WENO degree k and the Runge-Kutta
 * scheme may rise or fall across levels; the numerical flux and eps may
 * change too).  Level l still steps with m^l dt; the FAS restriction from
 * level l applies Phi_{l+1} with schemes[l+1].
 *   schemes   HOST array of p->levels schemes with the same nx, L and flux
 *             (and a, for advection).  Lines of more than 4096 cells need
 *             the same scheme on every level (else MGRIT_EUNSUPPORTED).
 *   p         as for mgrit_cycle; coarse_integrator must be 0.
 *   workspace at least mgrit_workspace_bytes(&schemes[0], p) bytes.
 * Other arguments, synchronisation and return codes as for mgrit_cycle.
 * With the same scheme on every level the iterates equal mgrit_cycle's bit
 * for bit.
 */
int mgrit_cycle_levels(const mgrit_scheme* schemes, const mgrit_params* p, const double* u0, double* u,
                       void* workspace, size_t ws_bytes, double* res_hist, int32_t* iters, void* stream);

/*
 * Discrete adjoint (the derivative of Phi written by hand; not in the paper).
 *
 * mgrit_phi_vjp -- lam_out[b] = (dPhi/du(u[b]))^T lam_in[b] for independent
 * lines: the Runge-Kutta stages of eq SSPRK1/2/3 in reverse, each applying the
 * transpose of the Jacobian of A (eq spaceDisc, eq LFflux) including the
 * subgradient of the global alpha_LF (all weight on the first maximising
 * interface/side, interfaces in increasing order, u^- before u^+).  Arrays are
 * nlines x nx.  The line must be a multiple of the cells per thread of the
 * adjoint kernel (any nx <= 512, even nx <= 1024); else MGRIT_EUNSUPPORTED.
 * The adjoint covers the Lax-Friedrichs flux with k = 0 or 2; other schemes
 * return MGRIT_EUNSUPPORTED here and in mgrit_adjoint (and 0 from
 * mgrit_adjoint_workspace_bytes).
 */
int mgrit_phi_vjp(const mgrit_scheme* s, double dt, const double* u, const double* lam_in, double* lam_out,
                  int64_t nlines, void* stream);

/*
 * mgrit_checkpoints -- serial forward stepping that keeps every `every`-th
 * node: ckpt[i] = u^{i*every}, i = 0..nt/every (so ckpt[nt/every] = u(T)).
 */
int mgrit_checkpoints(const mgrit_scheme* s, double dt, int32_t nt, int32_t every, const double* u0, double* ckpt,
                      void* stream);

/*
 * mgrit_adjoint -- reverse sweep of serial time stepping from checkpoints:
 * lambda_0 = (d u^{nt} / d u^0)^T lambda_T.  ckpt holds u at nodes 0, every,
 * 2 every, ..., nt (mgrit_checkpoints, or the level-0 C-points of a converged
 * mgrit_cycle with storage 1 and every = m).  Segments of `every` steps are
 * recomputed `parallel_segments` at a time (in parallel, keeping every stage
 * input), then swept backwards.  Memory: mgrit_adjoint_workspace_bytes =
 * parallel_segments * every * stages * nx doubles plus one line.  For
 * J = 1/2 ||u(T) - u_target||^2, lambda_T = u(T) - u_target and lambda_0 =
 * dJ/du0.  lambda_0 may not alias lambda_T.
 */
size_t mgrit_adjoint_workspace_bytes(const mgrit_scheme* s, int32_t nt, int32_t every, int32_t parallel_segments);
int mgrit_adjoint(const mgrit_scheme* s, double dt, int32_t nt, int32_t every, int32_t parallel_segments,
                  const double* ckpt, const double* lambda_T, double* lambda_0, void* workspace, size_t ws_bytes,
                  void* stream);

/* message of the last failure on this thread ("" if none) */
const char* mgrit_last_error(void);

/*
 * Kernel timing.  With profiling on, the library brackets every kernel it
 * launches with HIP events on the launch stream and accumulates, per kernel
 * class, the number of launches, the summed event time (ms), the number of
 * Phi line applications and the number of cell steps (Phi applications x
 * nx).  mgrit_get_profile synchronises the device and fills up to `cap`
 * entries; it returns the number of classes.  mgrit_set_profiling(1) clears
 * the counters.  Class ids: see MGRIT_KC_*.
 */
enum {
    MGRIT_KC_PHI = 0,        /* mgrit_phi / mgrit_serial                        */
    MGRIT_KC_RELAX_FC = 1,   /* fused F + C sweep (FCF first half), level 0      */
    MGRIT_KC_RELAX_FR = 2,   /* fused F + FAS restriction sweep, level 0         */
    MGRIT_KC_RELAX_FC_C = 3, /* fused F + C sweep, levels >= 1                   */
    MGRIT_KC_RELAX_FR_C = 4, /* fused F + restriction sweep, levels >= 1         */
    MGRIT_KC_INTERP = 5,     /* injection + F-relaxation (ideal interpolation)   */
    MGRIT_KC_COARSE = 6,     /* serial solve on the coarsest level               */
    MGRIT_KC_AUX = 7,        /* norms, copies, flags                             */
    MGRIT_KC_ADJOINT = 8,    /* reverse sweeps / single-step VJPs                */
    MGRIT_KC_ADJOINT_RECOMPUTE = 9, /* segment recomputation keeping stage inputs */
    MGRIT_KC_COUNT = 10
};

typedef struct {
    int64_t launches;
    double ms;
    double phi_lines;
    double cell_steps;
} mgrit_profile_entry;

void mgrit_set_profiling(int on);
int mgrit_get_profile(mgrit_profile_entry* out, int cap);

/* With profiling on, bracket only the launches of the kernel classes whose
   bit (1 << MGRIT_KC_*) is set in `classes` with events; the other classes
   still count launches, Phi lines and cell steps, with ms = 0.  Each event
   pair costs stream time between kernels, so a timing run keeps the events
   to the kernel it measures.  Default: every class.  Not thread safe. */
void mgrit_set_profiling_mask(uint32_t classes);

/* kernel configuration chosen for `nlines` lines of `nx` cells in one launch
   (one workgroup per line): cells per thread and waves per line.  Launches of
   fewer than 256 lines count as latency bound and get more threads per line.
   Returns MGRIT_EUNSUPPORTED if no compiled configuration covers the line. */
int mgrit_kernel_config(int32_t nx, int32_t nlines, int32_t* cells_per_thread, int32_t* waves);

/* split-line configuration for lines of nx cells in launches of many chunks:
   cells per thread, waves per tile and number of tiles; *tiles == 1 (and
   zeros) when the line runs on one workgroup. */
int mgrit_tiled_config(int32_t nx, int32_t* cells_per_thread, int32_t* waves, int32_t* tiles);

/* split-line configuration of one launch over `nchunks` chunks (time
   intervals, or lines for mgrit_phi; 1 for mgrit_serial and the coarsest
   solve) of lines of nx cells; `residual` != 0 for a launch that also forms
   the C-point residual (level-0 relaxation with a residual).  Launches whose
   mgrit_tiled_config shape would occupy fewer than 256 workgroups (chunks x
   tiles), write no residual and have no mgrit_set_tiled_config setting for
   nx take tiles of 1024 cells (2 cells per thread, 8 waves) when nx is even
   and at most 131072: a stage of such a launch is bound by latency, and
   smaller tiles shorten it.  Results are bitwise the same for every shape.
   Outputs as mgrit_tiled_config; MGRIT_EINVAL if nchunks < 0.  Allocates
   nothing and launches nothing. */
int mgrit_tiled_launch_config(int32_t nx, int64_t nchunks, int32_t residual, int32_t* cells_per_thread,
                              int32_t* waves, int32_t* tiles);

/* split lines of nx_lo..nx_hi cells into tiles of at most
   64 * waves * cells_per_thread cells (balanced lengths), with a compiled
   split-line pair: (1,4), (2,4), (2,8), (2,16), (4,4), (4,8), (4,16), (16,8).
   cells_per_thread == 0 clears every such setting.  Lines must give tiles of
   at least 4 cells.  Scalar laws only (systems: mgrit_set_sys_tiles).  Not
   thread safe. */
int mgrit_set_tiled_config(int32_t nx_lo, int32_t nx_hi, int32_t cells_per_thread, int32_t waves);

/* Systems (flux 2, 3) on split lines (sec 2.1.1 per tile): lines of
   nx_lo..nx_hi cells run on `tiles` workgroups, one cell per thread, the
   line cut into tiles of balanced length, each of 4..510 cells (else
   MGRIT_EINVAL); each tile keeps k + 1 ghost cells per side and exchanges
   alpha_LF and its edge faces' flux parts with the other tiles once per
   Runge-Kutta stage, so results are bitwise those of one workgroup per line.
   Lines of more than 512 cells split by default into the fewest tiles of at
   most 510 cells.  tiles == 0 clears every such setting.  Not thread safe. */
int mgrit_set_sys_tiles(int32_t nx_lo, int32_t nx_hi, int32_t tiles);

/* tiles per line of system scheme s (1: one workgroup) */
int mgrit_sys_tiles(const mgrit_scheme* s, int32_t* tiles);

/* the same with the number of time intervals (chunks) each workgroup of a
   split line advances together: 1, or 2 (the two chunks run half a
   Runge-Kutta stage apart, so that one chunk's exchange with the other tiles
   overlaps the other chunk's reconstruction; results are bitwise those of
   one chunk per workgroup).  Two intervals are compiled for (4, 8), whose
   workgroup then keeps up to 256 VGPRs (2 waves per SIMD).  The setting is
   cleared with the others by
   mgrit_set_tiled_config(.., 0, ..).  Not thread safe. */
int mgrit_set_tiled_intervals(int32_t nx_lo, int32_t nx_hi, int32_t cells_per_thread, int32_t waves,
                              int32_t intervals);

/* intervals per workgroup of the split-line configuration for lines of nx
   cells (1 when such a line runs on one workgroup) */
int mgrit_tiled_intervals(int32_t nx, int32_t* intervals);

/* override the configuration for line lengths nx_lo..nx_hi in latency-bound
   (latency != 0) or throughput launches (mgrit_autotune installs its choice
   this way); the pair must be compiled and cover nx_hi.  cells_per_thread ==
   0 clears every override.  Batches keep to the pairs compiled for them and
   take the measured default when an override names another.  Not thread
   safe. */
int mgrit_set_kernel_config(int32_t nx_lo, int32_t nx_hi, int32_t latency, int32_t cells_per_thread,
                            int32_t waves);

/*
 * Autotuner of the launch shape (not in the paper): times nsteps applications
 * of Phi with scheme s on nlines independent lines, one workgroup per line,
 * for every compiled (cells per thread, waves) pair whose workgroup covers
 * the line without being more than 4x larger, and picks the fastest (median
 * of three launches after one warm-up, HIP events on `stream`).  With
 * install != 0 the choice becomes the override for lines of exactly s->nx
 * cells in the regime of nlines (latency bound below 256 lines, else
 * throughput), as mgrit_set_kernel_config would set it.
 *   scratch  device, at least mgrit_autotune_scratch_bytes(s->nx, nlines)
 *            bytes, caller-owned; overwritten with smooth test lines.
 *   cells_per_thread, waves, ms_best  HOST outputs (each may be NULL).
 * Synchronises the stream.  Lines longer than one workgroup holds return
 * MGRIT_EUNSUPPORTED.  Not thread safe when installing.
 */
size_t mgrit_autotune_scratch_bytes(int32_t nx, int32_t nlines);
int mgrit_autotune(const mgrit_scheme* s, int32_t nlines, int32_t nsteps, void* scratch, size_t scratch_bytes,
                   int32_t install, int32_t* cells_per_thread, int32_t* waves, float* ms_best, void* stream);

/*
 * Split-line autotuner (not in the paper): times nsteps applications of Phi
 * on nlines lines of s->nx cells for every compiled split-line shape (cells
 * per thread, waves per tile, and intervals per workgroup: one chunk, or two
 * chunks advanced half a stage apart) whose balanced tiles hold the line and
 * can all be resident at once, and picks the fastest (median of three
 * launches after one warm-up, HIP events on `stream`).  With install != 0 the
 * choice becomes the split-line setting for lines of exactly s->nx cells, as
 * mgrit_set_tiled_intervals would set it.  Every shape evaluates the same
 * per-cell operations, so results do not depend on the choice.
 *   scratch  device, at least mgrit_autotune_scratch_bytes(s->nx, nlines)
 *            bytes, caller-owned; overwritten with smooth test lines.
 *   cells_per_thread, waves, intervals, ms_best  HOST outputs (may be NULL).
 * Synchronises the stream; uses the device's static split-line
 * synchronisation array.  Systems return MGRIT_EUNSUPPORTED.
 * Not thread safe when installing.
 */
int mgrit_autotune_tiled(const mgrit_scheme* s, int32_t nlines, int32_t nsteps, void* scratch, size_t scratch_bytes,
                         int32_t install, int32_t* cells_per_thread, int32_t* waves, int32_t* intervals,
                         float* ms_best, void* stream);

/*
 * Batches of independent problems (many initial-value problems solved by
 * MGRIT together; not in the paper).  Every problem has its own scheme
 * constants (flux, advection speed, nx, eps, L, alpha_fixed), fine step count
 * and step; k and stepper are common.  The MGRIT settings (m, levels >= 2,
 * relax, cycle, max_iter, init, coarse_guess, storage, sync_every, tol) are
 * common; the nt and dt fields of the params are ignored.
 *   u0   device, nx doubles: the problem's initial condition;
 *   u    device, the problem's level-0 iterate, (nt+1) x nx (storage 0) or
 *        (nt/m+1) x nx (storage 1), as for mgrit_cycle.
 * One launch per phase of the cycle covers the chunks of every problem that
 * shares a kernel configuration (lines longer than 4096 cells run their own
 * split-line launches).  Each problem stops doing work once its residual
 * norm is below tol (its chunks retire); the call returns when every
 * problem has converged or after max_iter cycles.  Every problem's iterates
 * are bitwise those of mgrit_cycle on that problem alone.
 */
typedef struct {
    mgrit_scheme scheme;
    int32_t nt;
    int32_t pad_;
    double dt;
    const double* u0;
    double* u;
} mgrit_problem;

/* workspace bytes of mgrit_cycle_batched (0 on invalid input) */
size_t mgrit_batched_workspace_bytes(const mgrit_problem* probs, int32_t count, const mgrit_params* p);

/*
 * mgrit_cycle_batched -- FAS-MGRIT on `count` problems (host array probs).
 * workspace: device, >= mgrit_batched_workspace_bytes, 256-byte aligned.
 * res_hist: host, count x (max_iter+1) doubles: problem i's residual norms
 * r_0 .. r_{iters[i]} at res_hist[i*(max_iter+1) + k], zeros after;
 * iters: host, count (cycles applied to each problem); status: host, count
 * (MGRIT_OK: converged, MGRIT_NOT_CONVERGED).  Synchronises the stream every
 * sync_every cycles and at the end.  Returns MGRIT_OK unless an error
 * occurred (per-problem convergence is in status).
 */
int mgrit_cycle_batched(const mgrit_problem* probs, int32_t count, const mgrit_params* p, void* workspace,
                        size_t ws_bytes, double* res_hist, int32_t* iters, int32_t* status, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MGRIT_H */
