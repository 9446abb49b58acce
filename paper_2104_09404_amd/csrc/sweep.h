// sweep.h -- internal interface between the C-ABI layer and the sweep kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mgk {

// Constants of Phi for one scheme: f(u) = u (fa u + fb), lambda(u) = 2 fa u + fb
// (Burgers: fa = 1/2, fb = 0; linear advection: fa = 0, fb = a).
struct PhiConst {
    double fa, fb;
    double half_inv_dx;  // 1/(2 dx): the flux difference uses twice the flux
    double eps;
    double alpha_fixed;  // > 0 replaces the global alpha_LF
    int roe;             // 1: Roe flux with the Harten-Hyman fix instead of LF
    int pad_;
};

enum EndMode : int {
    END_NONE = 0,      // stop after the F-steps
    END_CSTEP = 1,     // one more step to the chunk's end C-point -> side_out[c+1]
    END_RESTRICT = 2,  // one more step t, then FAS restriction: uc_out, gc_out
    END_PHI = 3,       // one more step (no rhs), stored at side_out[c]
};

// One launch = nchunks workgroups, chunk c handled by workgroup c.
// Chunk c starts from line `ustart + c*ustart_stride*nx` (or from side_in[c]
// for c >= 1 when side_in is set), optionally commits that start value to
// `ucommit + c*ucommit_stride*nx`, then takes `nsteps` steps
//   x <- Phi(x) + g^{cm+j}   (g == nullptr: no right-hand side)
// storing node cm+j at fout + (cm+j)*nx when fout is set, and finishes per end_mode.
struct SweepArgs {
    int nx;
    int nchunks;
    int m;
    int nsteps;
    int end_mode;
    int inject_last;       // chunk nchunks-1 also copies ustart[nchunks] -> ucommit[nchunks]
    int coarse_injection;  // END_RESTRICT: coarse guess by injection instead of eq restriction::u
    int coarse_split;      // END_RESTRICT: store g_c = t only; Phi_{l+1} of the chunk start is
                           // subtracted by a separate END_PHI launch (gc_sub) with the scheme of level l+1
    double dt;
    double dt_next;        // step of the next-coarser level (END_RESTRICT)
    PhiConst pc;
    const double* ustart;
    int64_t ustart_stride;
    const double* side_in;
    double* ucommit;
    int64_t ucommit_stride;
    double* fout;
    int fout_every;         // > 1: store only nodes n with n % fout_every == 0, at fout + (n/fout_every)*nx
    const double* g;
    double* side_out;
    const double* cref;     // current value of the chunk's end C-point: cref + (c+1)*cref_stride*nx
    int64_t cref_stride;
    const double* ystart;   // END_RESTRICT: source of the coarse step Phi_{l+1}; nullptr = the chunk start
    int64_t ystart_stride;
    double* r_out;          // residual t - u^{(c+1)m} stored at r_out + c*nx (nullable)
    double* resid_partial;  // per-chunk sum of squared C-point residuals (nullable)
    double* uc_out;
    double* gc_out;
    double* gc_sub;         // END_PHI: gc_sub[(c+1)*nx ..] -= Phi(x) instead of storing at side_out[c]
    const int* flag;        // if non-null and *flag != 0 the launch does nothing
    // fine-integrator matching (first order, forward Euler kernels only): the
    // steps of this launch apply Psi of order psi_order - 1 matching psi_M fine
    // steps of size dt_fine instead of Phi (psi_M == 0: Phi), the coarse step
    // of END_RESTRICT matching psi_M_next steps
    int psi_order;
    int psi_M;
    int psi_M_next;
    int ncomp;              // components per cell: 1, or D for a system (nx is then D x cells)
    double dt_fine;
    double alpha_next;      // > 0: LF coefficient of the coarse step of END_RESTRICT
    // lines split over several workgroups (tiled_impl.h)
    int tiles;              // workgroups per line (0: one workgroup per line)
    int groups;             // line groups resident at once (set by the launcher)
    unsigned long long* tile_sync;  // [0] error word, [kTileCounterStride * (1 + group)] arrival counters
    double* tile_pub;       // published edge data: groups x tiles x 2 x kTileSlot
};

// One batched launch: workgroup b runs chunk b - offset[i] of problem
// problem[i], i the last bucket entry with offset[i] <= b, with the arguments
// args[problem[i]] (device memory).
// A split-line batch launch reads the same table as (problem, chunk) work
// items: line groups of `tiles` workgroups take items grp, grp + groups, ...
// and synchronise through tile_sync / tile_pub.
struct BatchLaunch {
    const SweepArgs* args;
    const int* offset;   // nprob entries, ascending, offset[0] = 0
    const int* problem;  // nprob entries
    int nprob;
    int nblocks;         // work items (chunks of all problems of the launch)
    int end_mode;        // END_NONE, END_CSTEP or END_RESTRICT (every entry of args has it)
    int ragged;          // some problem's line is not a multiple of the cells per thread
    int roe;             // every problem of the launch uses the Roe flux (else LF)
    int tiles;           // split lines: workgroups per line (else 1)
    unsigned long long* tile_sync;  // split lines: error word
    double* tile_pub;               // split lines: published slots
    int groups;          // split lines: line groups of the launch (set at launch)
    int pad_;
};

// per-problem residual reduction of a batch
struct BatchNorm {
    const double* partial;  // n per-chunk partial sums
    int n;
    int pad_;
    double* hist;
    int* counter;
    int* flag;
};

// tiled lines: doubles per published slot, words between arrival counters
// (one 128-byte line each, so that groups do not contend for a line), and the
// largest resident grid the synchronisation scratch is sized for
constexpr int kTileSlot = 24;  // at least 1 + 4 x (ghost cells per side)
// systems on split lines: at least 1 + 4 x (ghost cells per side) x components
constexpr int kSysTileSlot = 56;
constexpr int kTileCounterStride = 16;
constexpr int kTileMaxWorkgroups = 8192;
// forward split-line sweeps publish into a ring of 3 slots per tile (the
// adjoint uses 2, by parity)
constexpr int kTileRing = 3;
// bit pattern of an empty slot value: a negative signalling NaN, which no
// arithmetic result can be (results are quiet NaNs at most)
constexpr unsigned long long kSlotEmpty = 0xFFF7DEADBEEF0001ull;
constexpr size_t kTileSyncBytes = sizeof(unsigned long long) * kTileCounterStride * (size_t)(kTileMaxWorkgroups + 1);
// two chunks per workgroup at most
constexpr size_t kTileScratchBytes = kTileSyncBytes + sizeof(double) * (size_t)kTileMaxWorkgroups * 2 * kTileRing * kTileSlot;
inline size_t tile_sync_bytes() { return kTileSyncBytes; }
inline size_t tile_scratch_bytes() { return kTileScratchBytes; }

// Adjoint launches (adjoint_impl.h): one workgroup per line b.
struct AdjArgs {
    int nx;
    int nlines;
    int nsteps;
    int stored;             // stage inputs read from traj (else recomputed from u, nsteps == 1)
    double dt;
    PhiConst pc;
    const double* u;        // start (stage_store) / state u^n (recompute) of line b at u + b*u_stride*nx
    int64_t u_stride;
    const double* traj;     // stage inputs of step n: traj + b*traj_stride + (n*ST + s)*nx
    double* traj_out;       // the same layout, written by the stage-store kernel
    int64_t traj_stride;
    const double* lam_in;   // adjoint at the end of the stretch, line b at lam_in + b*nx
    double* lam_out;        // adjoint at its start
    // lines split over several workgroups (tiled_adjoint_impl.h), as in SweepArgs
    int tiles;
    int groups;
    unsigned long long* tile_sync;
    double* tile_pub;
};

struct KernelCfg {
    int cpt;            // cells per thread
    int nw;             // waves per workgroup (= per line)
    int intervals = 1;  // split lines: chunks a workgroup advances together (1 or 2)
};

// compiled (cells per thread, waves) pairs.  Many-line launches use few
// threads per line with several cells each (instruction-level parallelism,
// registers); launches with few lines (coarse levels, the serial coarsest
// solve) use more threads per line to shorten each step.
#define MGK_CFG_LIST(X) \
    X(1, 1)             \
    X(2, 1)             \
    X(4, 1)             \
    X(1, 2)             \
    X(2, 2)             \
    X(4, 2)             \
    X(1, 4)             \
    X(2, 4)             \
    X(4, 4)             \
    X(8, 4)             \
    X(1, 8)             \
    X(2, 8)             \
    X(4, 8)             \
    X(8, 8)             \
    X(1, 16)            \
    X(2, 16)

// (cells per thread, waves) pairs compiled for batches of problems (the ones
// the configuration choice makes for throughput and latency launches)
#define MGK_BATCH_CFG_LIST(X) \
    X(1, 1)                   \
    X(2, 1)                   \
    X(4, 1)                   \
    X(1, 2)                   \
    X(2, 2)                   \
    X(4, 2)                   \
    X(2, 4)                   \
    X(4, 4)                   \
    X(2, 8)                   \
    X(4, 8)                   \
    X(8, 8)

// (cells per thread, waves) pairs compiled for the adjoint; the line must be a
// multiple of the cells per thread
#define MGK_ADJ_CFG_LIST(X) \
    X(1, 1)                 \
    X(1, 2)                 \
    X(1, 4)                 \
    X(1, 8)                 \
    X(2, 4)                 \
    X(2, 8)

// (cells per thread, waves) pairs compiled for tiled lines; a tile holds at
// most 64 * waves * cells per thread cells
// (cells per thread, waves) pairs compiled for split lines with two chunks
// per workgroup (two chunks' state needs up to 256 VGPRs, hence 8 waves)
#define MGK_TILED_PAIR_CFG_LIST(X) \
    X(4, 8)

// split-line shapes compiled for batches (the default choices of split lines)
#define MGK_TILED_BATCH_CFG_LIST(X) \
    X(4, 16)                        \
    X(2, 16)                        \
    X(4, 8)

// one-workgroup shapes of batches for lines of 4097..8192 cells (wide_impl.h):
// (cells per thread, waves, virtual threads per thread), the line a multiple
// of the cells per thread
#define MGK_WIDE_CFG_LIST(X) \
    X(4, 16, 2)              \
    X(4, 8, 4)               \
    X(2, 8, 8)

#define MGK_TILED_CFG_LIST(X) \
    X(1, 4)                   \
    X(2, 4)                   \
    X(2, 8)                   \
    X(2, 16)                  \
    X(4, 4)                   \
    X(4, 8)                   \
    X(4, 16)                  \
    X(16, 8)

// (cells per thread, waves) pairs compiled for the adjoint of split lines;
// every tile must be a whole number of threads
#define MGK_TADJ_CFG_LIST(X) \
    X(1, 4)                  \
    X(2, 4)                  \
    X(1, 8)                  \
    X(2, 8)

// Split lines: G tiles balanced in whole threads (TGeo) of at least 4 and at
// most 64 nw cpt cells each.  The shortest tile holds cpt floor(U/G) cells and
// the longest cpt ceil(U/G) + nx mod cpt, U = floor(nx / cpt).
inline bool tiles_fit(int64_t nx, int64_t G, int cpt, int nw)
{
    if (G < 1 || cpt < 1) return false;
    const int64_t U = nx / cpt;
    const int64_t shortest = (int64_t)cpt * (U / G);
    const int64_t longest = (int64_t)cpt * ((U + G - 1) / G) + nx % cpt;
    return shortest >= 4 && longest <= 64 * (int64_t)nw * cpt;
}

inline size_t tiled_smem_bytes(int cpt, int nw)
{
    // tile + 4 ghost cells per side and a scratch slot (degree 3; fewer ghosts otherwise)
    return sizeof(double) * (64 * (size_t)nw * (size_t)cpt + 9 + 2 * 64 * (size_t)nw + (size_t)nw + 2 * 40);
}

inline size_t smem_bytes(int cpt, int nw)
{
    return sizeof(double) * (64 * (size_t)nw * (size_t)cpt + 2 * 64 * (size_t)nw + 3 * (size_t)nw);
}

hipError_t launch_sweep(const SweepArgs& a, const KernelCfg& cfg, int k, int stepper, hipStream_t s);
hipError_t launch_tiled(const SweepArgs& a, const KernelCfg& cfg, int k, int stepper, hipStream_t s);
hipError_t launch_batch(const BatchLaunch& t, const KernelCfg& cfg, int k, int stepper, hipStream_t s);
hipError_t launch_tiled_batch(const BatchLaunch& t, const KernelCfg& cfg, int k, int stepper, hipStream_t s);
// one workgroup per line of up to cfg.intervals x 64 cfg.nw x cfg.cpt cells (wide_impl.h)
hipError_t launch_wide_batch(const BatchLaunch& t, const KernelCfg& cfg, int k, int stepper, hipStream_t s);
bool tiled_batch_compiled(const KernelCfg& cfg);
hipError_t launch_reduce_norm_batch(const BatchNorm* tab, int count, double tol, int* converged, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& a, const KernelCfg& cfg, int k, int stepper, int store_mode, hipStream_t s);
hipError_t launch_tiled_adjoint(const AdjArgs& a, const KernelCfg& cfg, int k, int stepper, int store_mode,
                                hipStream_t s);
hipError_t launch_broadcast(const double* src, double* dst, int64_t nx, int64_t nlines, hipStream_t s);
hipError_t launch_fill_wave(double* u, int64_t nx, int64_t nlines, hipStream_t s);
// systems (flux 2: shallow water, 3: Euler): one workgroup of `threads` per line
hipError_t launch_sys(const SweepArgs& a, int threads, int flux, int k, int stepper, hipStream_t s);
// systems on split lines: a.tiles workgroups of `threads` per line (sys_tiled_impl.h)
hipError_t launch_sys_tiled(const SweepArgs& a, int threads, int flux, int k, int stepper, hipStream_t s);
hipError_t launch_clear_ints(int* p, int n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long value, int64_t n, hipStream_t s);
hipError_t launch_sumsq_norm(const double* r, int64_t n, double* out, hipStream_t s);
hipError_t launch_reduce_norm(const double* partial, int n, double* hist, int* counter, int* flag, double tol,
                              hipStream_t s);

}  // namespace mgk
