// sweep_impl.h -- gfx950 kernels for the MGRIT hot path (included by the
// sweep_k*_s*.hip translation units, one per reconstruction degree and
// Runge-Kutta scheme, so that they compile in parallel).
//
// One workgroup owns one line (one time chunk at one level, or one independent
// line) and steps it through several applications of the propagator Phi,
// entirely on chip: every thread keeps CPT consecutive cells of the line in
// registers, the line is mirrored into LDS once per Runge-Kutta stage so that
// threads can read their 3-cell halo (periodic wrap by index), and the global
// Lax-Friedrichs coefficient alpha_LF of the stage is a workgroup max
// reduction (DPP within each wave, then one LDS slot per wave).
//
// Per RK stage (sec 2.2) a thread:
//   1. writes its cells to LDS, barrier;
//   2. reads its halo and reconstructs u^-_{j+1/2} and u^+_{j-1/2} for each of
//      its cells (sec 2.1.1; the per-cell arithmetic is in cell_math.h), takes
//      the local max of |lambda|, publishes its two boundary reconstructions,
//      barrier;
//   3. reads alpha_LF and its neighbours' boundary reconstructions, forms the
//      LF fluxes of its CPT+1 interfaces (eq LFflux) and the stage update.
// The interface shared by two threads is evaluated by both from the same
// operands with the same operations, so the flux difference telescopes
// exactly and the sum of u is conserved to round-off.
//
// Arithmetic is FP64 only; no MFMA (this is stencil work, not a contraction).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cell_math.h"
#include "sweep.h"

namespace mgk {

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Max over the 64 lanes of a wave, returned uniformly (NaN-ignoring like fmax).
// DPP moves within quads, half-rows and rows, then the row broadcasts of lanes
// 15 and 31 leave the maximum in lane 63, which is read back as a scalar.
// Full-mask moves take no "old" operand; the two row broadcasts keep the old
// value in the rows they do not write.
template <int CTRL>
__device__ __forceinline__ double dpp_all(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __double2loint(v);
    const int hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false);
    const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_all<0xb1>(v));         // quad_perm [1,0,3,2]
    v = fmax(v, dpp_all<0x4e>(v));         // quad_perm [2,3,0,1]
    v = fmax(v, dpp_all<0x141>(v));        // row_half_mirror
    v = fmax(v, dpp_all<0x140>(v));        // row_mirror
    v = fmax(v, dpp_move<0x142, 0xa>(v));  // row_bcast:15 into rows 1 and 3
    v = fmax(v, dpp_move<0x143, 0xc>(v));  // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// Geometry of one thread inside its line.  Thread t owns cells
// j0 = t*CPT .. j0+CPT-1; threads past the end of the line (and the cells past
// nx of the last, ragged thread) compute on scratch values that are never
// stored and never enter alpha_LF.
template <int CPT, int NW>
struct Geo {
    int nx;
    int t;        // thread index in the line
    int j0;       // first cell
    int nvalid;   // cells owned inside the line (CPT, fewer for the ragged thread, 0 past the end)
    int left;     // thread owning the cell before j0 (periodic)
    int right;    // thread owning the cell after the last owned one (periodic)
    bool active;  // owns at least one cell
    bool ragged;  // owns fewer than CPT cells
    int halo[6];  // LDS slots of window positions 0,1,2 and CPT+3..CPT+5

    // LDS slot of cell c: the line is stored transposed, cell c at
    // (c mod CPT) * threads + c / CPT, so that the q-th cells of consecutive
    // threads (and every window position) are consecutive doubles: no bank
    // conflicts for any cells per thread
    static __device__ __forceinline__ int slot(int c) { return (c % CPT) * (64 * NW) + c / CPT; }
    __device__ __forceinline__ int own(int q) const { return q * (64 * NW) + t; }

    __device__ __forceinline__ void init(int nx_)
    {
        nx = nx_;
        t = threadIdx.x;
        const int nact = (nx + CPT - 1) / CPT;
        active = t < nact;
        j0 = t * CPT;
        nvalid = active ? min(CPT, nx - j0) : 0;
        ragged = active && nvalid < CPT;
        left = active ? ((t == 0) ? nact - 1 : t - 1) : t;
        right = active ? ((t == nact - 1) ? 0 : t + 1) : t;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            halo[p] = slot(wrapi(j0 - 3 + p, nx));
            halo[3 + p] = slot(wrapi(j0 + CPT + p, nx));
        }
    }
};

// Shared-memory layout: line[64*NW*CPT] | bm[64*NW] | bp[64*NW] | wred[NW] | amax[2*NW].
// The line array (transposed, see Geo::slot) covers every thread's cells, so stage values are written
// without predicates; slots nx.. are scratch.  amax holds the per-wave maxima
// of the alpha_LF reduction, double-buffered by stage parity.
template <int CPT, int NW>
struct Smem {
    double* line;
    double* bm;
    double* bp;
    double* wred;
    double* amax;
    __device__ __forceinline__ void init(double* base)
    {
        line = base;
        bm = base + 64 * NW * CPT;
        bp = bm + 64 * NW;
        wred = bp + 64 * NW;
        amax = wred + NW;
    }
};

// WENO reconstructions of the thread's cells from its window w[p] = cell
// j0 - 3 + p (p = 0..CPT+5): um[q] = u^-_{j+1/2}, up[q] = u^+_{j-1/2} of cell
// j = j0 + q, for degree K = 0 (piecewise constant), 1, 2 or 3 (s = 1, 3, 5, 7).
template <int CPT, int K>
__device__ __forceinline__ void reconstruct(const double (&w)[CPT + 6], double eps, double (&um)[CPT],
                                            double (&up)[CPT])
{
    if constexpr (K == 0) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            um[q] = w[3 + q];
            up[q] = w[3 + q];
        }
    } else if constexpr (K == 1) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) weno3_cell(w[q + 2], w[q + 3], w[q + 4], eps, um[q], up[q]);
    } else if constexpr (K == 2) {
        double E[CPT + 6];
#pragma unroll
        for (int p = 2; p <= CPT + 3; ++p) E[p] = weno5_e(w[p - 1], w[p], w[p + 1], eps);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int p = q + 3;
            weno5_cell(w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], E[p - 1], E[p], E[p + 1], um[q], up[q]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            weno7_cell(w[q], w[q + 1], w[q + 2], w[q + 3], w[q + 4], w[q + 5], w[q + 6], eps, um[q], up[q]);
    }
}

// A(V) for the thread's cells: eq spaceDisc with the LF flux (eq LFflux) or,
// with ROE, the Roe flux with the Harten-Hyman fix (eq roeflux), and a WENO
// reconstruction of degree K.
// RAG: the line length is not a multiple of CPT, so one thread is ragged.
// par selects the alpha_LF slots of this stage (the other half is still read
// by slow waves of the previous stage until the first barrier).  The Roe flux
// is local to its interface: no reduction.  The flux is a compile-time choice:
// a run-time one lets the compiler duplicate whole step loops per flux.
template <int CPT, int NW, int K, bool RAG, bool ROE = false>
__device__ __forceinline__ void op_A(const double (&V)[CPT], double (&A)[CPT], const Geo<CPT, NW>& g,
                                     const Smem<CPT, NW>& sm, const PhiConst& pc, int& par)
{
#pragma unroll
    for (int q = 0; q < CPT; ++q) sm.line[g.own(q)] = V[q];
    __syncthreads();

    // window w[p] = cell j0 - 3 + p, p = 0..CPT+5
    double w[CPT + 6];
#pragma unroll
    for (int q = 0; q < CPT; ++q) w[3 + q] = V[q];
    if (RAG && g.ragged) {
        // positions past the end of the line wrap around to its first cells
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (q >= g.nvalid) w[3 + q] = sm.line[g.slot(wrapi(g.j0 + q, g.nx))];
    }
    if constexpr (K > 0) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            w[p] = sm.line[g.halo[p]];
            w[CPT + 3 + p] = sm.line[g.halo[3 + p]];
        }
    }
    double um[CPT], up[CPT];
    reconstruct<CPT, K>(w, pc.eps, um, up);
    double last = um[CPT - 1];
    if (RAG && g.ragged) {
#pragma unroll
        for (int q = 0; q < CPT - 1; ++q)
            if (q == g.nvalid - 1) last = um[q];
    }
    sm.bm[g.t] = last;
    sm.bp[g.t] = up[0];
    double F[CPT + 1];
    if constexpr (ROE) {
        __syncthreads();
        const double uml = sm.bm[g.left];
        const double upr = sm.bp[g.right];
#pragma unroll
        for (int q = 0; q <= CPT; ++q) {
            const double uL = (q == 0) ? uml : um[q - 1];
            const double uR = (q == CPT) ? upr : up[q];
            F[q] = roe_flux2(uL, uR, pc.fa, pc.fb);
        }
    } else {
        double lmax = 0.0;
#pragma unroll
        for (int q = 0; q < CPT; ++q) lmax = fmax(lmax, fmax(fabs(um[q]), fabs(up[q])));
        // alpha_LF: max|u^{+-}| over the line (exact, order independent): wave max,
        // then one slot per wave (double-buffered by stage parity)
        if (!g.active) lmax = 0.0;
        lmax = wave_max(lmax);
        if (NW > 1 && (threadIdx.x & 63) == 0) sm.amax[par * NW + (threadIdx.x >> 6)] = lmax;
        __syncthreads();

        double alpha = pc.alpha_fixed;
        if (!(alpha > 0.0)) {
            if (NW > 1) {
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) lmax = fmax(lmax, sm.amax[par * NW + w2]);
            }
            alpha = lf_alpha(lmax, pc.fa, pc.fb);
        }
        par ^= 1;
        const double uml = sm.bm[g.left];
        const double upr = sm.bp[g.right];
#pragma unroll
        for (int q = 0; q <= CPT; ++q) {
            const double uL = (q == 0) ? uml : um[q - 1];
            const double uR = (q == CPT) ? upr : up[q];
            F[q] = lf_flux2(uL, uR, pc.fa, pc.fb, alpha);
        }
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) A[q] = (F[q] - F[q + 1]) * pc.half_inv_dx;
}

// x <- Phi(x) with step dt (eq SSPRK1/2/3)
template <int CPT, int NW, int K, int ST, bool RAG, bool ROE = false>
__device__ __forceinline__ void phi(double (&x)[CPT], double dt, const Geo<CPT, NW>& g, const Smem<CPT, NW>& sm,
                                    const PhiConst& pc, int& par)
{
    double A[CPT];
    if (ST == 1) {
        op_A<CPT, NW, K, RAG, ROE>(x, A, g, sm, pc, par);
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = rk_first(x[q], A[q], dt);
    } else if (ST == 2) {
        double v[CPT];
        op_A<CPT, NW, K, RAG, ROE>(x, A, g, sm, pc, par);
#pragma unroll
        for (int q = 0; q < CPT; ++q) v[q] = rk_first(x[q], A[q], dt);
        op_A<CPT, NW, K, RAG, ROE>(v, A, g, sm, pc, par);
        const double hdt = 0.5 * dt;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = rk2_second(x[q], v[q], A[q], hdt);
    } else {
        double v[CPT];
        op_A<CPT, NW, K, RAG, ROE>(x, A, g, sm, pc, par);
#pragma unroll
        for (int q = 0; q < CPT; ++q) v[q] = rk_first(x[q], A[q], dt);
        op_A<CPT, NW, K, RAG, ROE>(v, A, g, sm, pc, par);
        const double qdt = 0.25 * dt;
#pragma unroll
        for (int q = 0; q < CPT; ++q) v[q] = rk3_second(x[q], v[q], A[q], qdt);
        op_A<CPT, NW, K, RAG, ROE>(v, A, g, sm, pc, par);
        const double tdt = (2.0 / 3.0) * dt;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = rk3_third(x[q], v[q], A[q], tdt);
    }
}

// ---------------------------------------------------------------------------
// fine-integrator matching (sec 3.3.1) for the fine scheme of eq fineLF:
// average E(v)_i = (v_{i+1} + v_{i-1})/2 and central difference
// D(v)_i = (v_{i+1} - v_{i-1})/(2 dx) through the LDS line
// ---------------------------------------------------------------------------
template <int CPT, int NW, bool RAG>
__device__ __forceinline__ void lds_neighbours(const double (&v)[CPT], double& nl, double& nr, const Geo<CPT, NW>& g,
                                               const Smem<CPT, NW>& sm)
{
    __syncthreads();  // earlier readers of the line are done
#pragma unroll
    for (int q = 0; q < CPT; ++q) sm.line[g.own(q)] = v[q];
    __syncthreads();
    nl = sm.line[g.halo[2]];  // cell j0 - 1
    nr = (RAG && g.ragged) ? sm.line[g.slot(wrapi(g.j0 + g.nvalid, g.nx))] : sm.line[g.halo[3]];
}

// out = E(v) (avg) or D(v) (diff); out may alias v
template <int CPT, int NW, bool RAG, bool DIFF>
__device__ __forceinline__ void ed_op(const double (&v)[CPT], double (&out)[CPT], const Geo<CPT, NW>& g,
                                      const Smem<CPT, NW>& sm, const PhiConst& pc)
{
    double nl, nr;
    lds_neighbours<CPT, NW, RAG>(v, nl, nr, g, sm);
    const int last = RAG ? g.nvalid - 1 : CPT - 1;
    double r[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const double left = (q == 0) ? nl : v[q - 1];
        const double right = (q == last) ? nr : ((q + 1 < CPT) ? v[q + 1] : nr);
        r[q] = DIFF ? (right - left) * pc.half_inv_dx : 0.5 * (right + left);
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) out[q] = r[q];
}

// x <- Psi(x): the coarse integrator matching M steps of eq fineLF with fine
// step dt (order 0: eq coarseLFord0, E^M u - M dt D f(u); order 1: eq
// coarseLFord1 / eq fineLFxM, E^M u - dt sum_{i=1}^{M} E^{i-1} D f(E^{M-i} u),
// the sum accumulated as T_0 = D f(u), T_k = E T_{k-1} + D f(E^k u))
template <int CPT, int NW, bool RAG>
__device__ __forceinline__ void psi(double (&x)[CPT], int order, int M, double dt, const Geo<CPT, NW>& g,
                                    const Smem<CPT, NW>& sm, const PhiConst& pc)
{
    double f[CPT], T[CPT], v[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        v[q] = x[q];
        f[q] = flux_f(x[q], pc.fa, pc.fb);
    }
    ed_op<CPT, NW, RAG, true>(f, T, g, sm, pc);
    if (order == 0) {
        for (int r = 0; r < M; ++r) ed_op<CPT, NW, RAG, false>(v, v, g, sm, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = v[q] - (double)M * dt * T[q];
        return;
    }
    for (int k = 1; k < M; ++k) {
        ed_op<CPT, NW, RAG, false>(v, v, g, sm, pc);
        ed_op<CPT, NW, RAG, false>(T, T, g, sm, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) f[q] = flux_f(v[q], pc.fa, pc.fb);
        double Df[CPT];
        ed_op<CPT, NW, RAG, true>(f, Df, g, sm, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) T[q] = T[q] + Df[q];
    }
    ed_op<CPT, NW, RAG, false>(v, v, g, sm, pc);
#pragma unroll
    for (int q = 0; q < CPT; ++q) x[q] = v[q] - dt * T[q];
}

// one step of the level: Phi, or the matching coarse integrator of M fine steps
template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__device__ __forceinline__ void level_step(double (&x)[CPT], double dt, int M, const SweepArgs& a,
                                           const Geo<CPT, NW>& g, const Smem<CPT, NW>& sm, const PhiConst& pc,
                                           int& par)
{
    if constexpr (K == 0 && ST == 1) {
        if (a.psi_order != 0 && M > 0) {
            psi<CPT, NW, RAG>(x, a.psi_order - 1, M, a.dt_fine, g, sm, pc);
            return;
        }
    }
    phi<CPT, NW, K, ST, RAG, ROE>(x, dt, g, sm, pc, par);
}

// Reads the thread's cells of a line into t without using them, so that the
// loads stay in flight until the values are needed.  Every lane reads in
// bounds and without a branch: a lane that owns no cell reads the line's
// first cells, and (RAG) the ragged lane its last cell in place of the
// missing ones; without RAG every active lane owns CPT cells and the line
// holds at least CPT.  (A load under its own per-cell predicate would be
// waited for before the next one is issued: one memory round trip per cell.)
// Only t[q] with q < nvalid is meaningful.
template <int CPT, int NW, bool RAG = true>
__device__ __forceinline__ void fetch_line(double (&t)[CPT], const double* src, const Geo<CPT, NW>& g)
{
    // 32-bit cell indices off the (wave-uniform) line pointer
    const int j0 = g.active ? g.j0 : 0;
    if constexpr (RAG) {
        const int last = g.active ? g.nvalid - 1 : 0;
#pragma unroll
        for (int q = 0; q < CPT; ++q) t[q] = src[j0 + (q < last ? q : last)];
    } else {
#pragma unroll
        for (int q = 0; q < CPT; ++q) t[q] = src[j0 + q];
    }
}

// The thread's cells of a line, 0 where it owns none.
template <int CPT, int NW, bool RAG = true>
__device__ __forceinline__ void load_line(double (&x)[CPT], const double* src, const Geo<CPT, NW>& g)
{
    double t[CPT];
    fetch_line<CPT, NW, RAG>(t, src, g);
#pragma unroll
    for (int q = 0; q < CPT; ++q) x[q] = (q < g.nvalid) ? t[q] : 0.0;
}

// Waits for every outstanding vector memory operation of the thread (loads
// and stores).  Placed before a step loop where loads or stores are pending:
// the compiler otherwise carries them into the loop's entry and waits at the
// top of every step, which then also waits for the previous step's stores.
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// How a step loop gets the right-hand side g of each step, as a compile-time
// tag for a generic lambda (one compiled loop per mode):
//   RHS_NONE:  no right-hand side (level 0);
//   RHS_AHEAD: g of the next step is read while the current one runs;
//   RHS_LATE:  g is read after the step's stages, if there is one (run-time
//              test; for kernels whose registers cannot hold g across stages).
enum RhsMode { RHS_NONE = 0, RHS_AHEAD = 1, RHS_LATE = 2 };
template <int M>
struct RhsTag {
    static constexpr int value = M;
};

template <int CPT, int NW>
__device__ __forceinline__ void store_line(const double (&x)[CPT], double* dst, const Geo<CPT, NW>& g)
{
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (q < g.nvalid) dst[g.j0 + q] = x[q];
    }
}

// x += t on every cell slot of the thread.  The slots it does not own (past
// the line end) carry values that no owned cell's arithmetic reads: the
// stage code takes those window positions from the wrapped line in LDS and
// leaves inactive lanes out of the alpha reduction, and stores skip them.
// Without a per-cell select the stored registers are x itself, not
// temporaries that the next step would reuse while the stores are pending
// (which would make it wait for them).
template <int CPT>
__device__ __forceinline__ void add_line(double (&x)[CPT], const double (&t)[CPT])
{
#pragma unroll
    for (int q = 0; q < CPT; ++q) x[q] = x[q] + t[q];
}

template <int CPT, int NW, bool RAG = true>
__device__ __forceinline__ void copy_line(const double* src, double* dst, const Geo<CPT, NW>& g)
{
    double t[CPT];
    fetch_line<CPT, NW, RAG>(t, src, g);
    store_line(t, dst, g);
}

// sum of squares of (a - b) over the line, in a fixed order; valid in thread 0
template <int CPT, int NW, bool RAG = true>
__device__ __forceinline__ double line_sqdiff(const double (&a)[CPT], const double* b, const Geo<CPT, NW>& g,
                                              const Smem<CPT, NW>& sm)
{
    double s = 0.0;
    if (g.active) {
        double t[CPT];
        fetch_line<CPT, NW, RAG>(t, b, g);
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (q < g.nvalid) {
                const double d = a[q] - t[q];
                s = fma(d, d, s);
            }
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sm.wred[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NW; ++w) tot += sm.wred[w];
    }
    return tot;
}

// One chunk (one line) per workgroup.  See SweepArgs for the roles; END is
// the compile-time end mode, ROE the numerical flux.
template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE>
__device__ __forceinline__ void sweep_body_t(const SweepArgs& a, const int c)
{
    if (a.flag != nullptr && *a.flag != 0) return;
    extern __shared__ double smem_raw[];
    Smem<CPT, NW> sm;
    sm.init(smem_raw);
    Geo<CPT, NW> g;
    g.init(a.nx);
    int par = 0;
    const int64_t nx = a.nx;

    const double* src = (a.side_in != nullptr && c > 0) ? a.side_in + (int64_t)c * nx
                                                        : a.ustart + (int64_t)c * a.ustart_stride * nx;
    double x[CPT];
    load_line<CPT, NW, RAG>(x, src, g);
    wait_loads();
    if (a.ucommit != nullptr) store_line(x, a.ucommit + (int64_t)c * a.ucommit_stride * nx, g);
    if (a.inject_last && c == a.nchunks - 1) {
        // the level's final C-point is committed / injected as well
        const double* last = (a.side_in != nullptr) ? a.side_in + (int64_t)a.nchunks * nx
                                                    : a.ustart + (int64_t)a.nchunks * a.ustart_stride * nx;
        copy_line<CPT, NW, RAG>(last, a.ucommit + (int64_t)a.nchunks * a.ucommit_stride * nx, g);
        // (the copies' registers are reused in the step loop, which would
        // otherwise wait at every step for these stores)
        wait_loads();
    }
    // the chunk's starting C-point (the source of the coarse step of END_RESTRICT)
    const double* cstart = (a.ystart != nullptr) ? a.ystart + (int64_t)c * a.ystart_stride * nx : src;
    if (END == END_RESTRICT && c == 0) {
        // coarse node 0: u_c^0 = u^0, g_c^0 = g^0 (= u^0 at level 0)
        copy_line<CPT, NW, RAG>(cstart, a.uc_out, g);
        copy_line<CPT, NW, RAG>(a.g != nullptr ? a.g : cstart, a.gc_out, g);
        wait_loads();
    }

    // Step j of the loop ends at node n0 + j; the C-step after it (END_CSTEP,
    // END_RESTRICT) at n1 = n0 + m.  With up to 4 cells per thread the
    // right-hand side of the next step is read one step ahead, so that its
    // loads are in flight during the stages, and the loop is compiled once
    // with and once without a right-hand side (level 0 has none), so that
    // neither version carries the other's loads, adds or waits.  With 8 cells
    // per thread the registers that would hold g across the stages cost more
    // than the wait, and one loop reads g after each step's stages.
    constexpr bool AHEAD = CPT <= 4;
    const int64_t n0 = (int64_t)c * a.m;
    const int64_t n1 = n0 + a.m;
    constexpr bool cend = (END == END_CSTEP || END == END_RESTRICT);
    const int nrhs = a.nsteps + (cend ? 1 : 0);
    const bool hg = a.g != nullptr;
    auto rhs_node = [&](int j) -> int64_t { return j <= a.nsteps ? n0 + j : n1; };
    double gn[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) gn[q] = 0.0;
    if (AHEAD && hg && nrhs >= 1) fetch_line<CPT, NW, RAG>(gn, a.g + rhs_node(1) * nx, g);
    auto steps = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        // strided trajectory: position of node n0 + j among the stored nodes
        const int every = a.fout_every > 1 ? a.fout_every : 1;
        int frem = (int)((n0 + 1) % every);
        int64_t fidx = (n0 + 1) / every;
        for (int j = 1; j <= a.nsteps; ++j) {
            level_step<CPT, NW, K, ST, RAG, ROE>(x, a.dt, a.psi_M, a, g, sm, a.pc, par);
            if constexpr (M == RHS_AHEAD) {
                add_line(x, gn);
            } else if constexpr (M == RHS_LATE) {
                if (hg) {
                    fetch_line<CPT, NW, RAG>(gn, a.g + rhs_node(j) * nx, g);
                    add_line(x, gn);
                }
            }
            if (a.fout != nullptr && frem == 0) store_line(x, a.fout + fidx * nx, g);
            if constexpr (M == RHS_AHEAD) {
                if (j < nrhs) fetch_line<CPT, NW, RAG>(gn, a.g + rhs_node(j + 1) * nx, g);
            }
            if (++frem == every) {
                frem = 0;
                ++fidx;
            }
        }
    };
    if constexpr (AHEAD) {
        if (hg) steps(RhsTag<RHS_AHEAD>{});
        else steps(RhsTag<RHS_NONE>{});
    } else {
        steps(RhsTag<RHS_LATE>{});
    }

    if constexpr (END == END_NONE) return;
    if constexpr (END == END_PHI) {
        level_step<CPT, NW, K, ST, RAG, ROE>(x, a.dt, a.psi_M, a, g, sm, a.pc, par);
        if (a.gc_sub != nullptr) {
            // the second half of a split FAS restriction: g_c = t - Phi_{l+1}(chunk start)
            double* out = a.gc_sub + (int64_t)(c + 1) * nx;
            double t[CPT];
            fetch_line<CPT, NW, RAG>(t, out, g);
            if (g.active) {
#pragma unroll
                for (int q = 0; q < CPT; ++q)
                    if (q < g.nvalid) out[g.j0 + q] = t[q] - x[q];
            }
            return;
        }
        store_line(x, a.side_out + (int64_t)c * nx, g);
        return;
    }
    // one more step to the chunk's end C-point n1
    level_step<CPT, NW, K, ST, RAG, ROE>(x, a.dt, a.psi_M, a, g, sm, a.pc, par);
    if (hg) {
        if constexpr (!AHEAD) fetch_line<CPT, NW, RAG>(gn, a.g + n1 * nx, g);
        add_line(x, gn);
    }
    // the current value at that C-point
    const double* cnext = a.cref + (int64_t)(c + 1) * a.cref_stride * nx;
    if (a.resid_partial != nullptr) {
        const double s = line_sqdiff<CPT, NW, RAG>(x, cnext, g, sm);
        if (threadIdx.x == 0) a.resid_partial[c] = s;
    }
    if (a.r_out != nullptr && g.active) {
        double t[CPT];
        fetch_line<CPT, NW, RAG>(t, cnext, g);
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (q < g.nvalid) a.r_out[(int64_t)c * nx + g.j0 + q] = x[q] - t[q];
    }
    if constexpr (END == END_CSTEP) {
        if (a.side_out != nullptr) store_line(x, a.side_out + (int64_t)(c + 1) * nx, g);
        return;
    }
    // END_RESTRICT: t = x; coarse guess and FAS right-hand side
    if (a.coarse_injection) copy_line<CPT, NW, RAG>(cnext, a.uc_out + (int64_t)(c + 1) * nx, g);
    else store_line(x, a.uc_out + (int64_t)(c + 1) * nx, g);
    if (a.coarse_split) {
        store_line(x, a.gc_out + (int64_t)(c + 1) * nx, g);
        return;
    }
    double y[CPT];
    load_line<CPT, NW, RAG>(y, cstart, g);
    PhiConst pcn = a.pc;
    if (a.alpha_next > 0.0) pcn.alpha_fixed = a.alpha_next;
    level_step<CPT, NW, K, ST, RAG, ROE>(y, a.dt_next, a.psi_M_next, a, g, sm, pcn, par);
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) y[q] = x[q] - y[q];
    }
    store_line(y, a.gc_out + (int64_t)(c + 1) * nx, g);
}


// The four roles as separately named kernels (so that profiles tell them
// apart); ROE (the numerical flux) is a kernel parameter, so that each flux
// gets its own code and register allocation
template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void relax_f_kernel(SweepArgs a)
{
    sweep_body_t<CPT, NW, K, ST, RAG, END_NONE, ROE>(a, blockIdx.x);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void relax_fc_kernel(SweepArgs a)
{
    sweep_body_t<CPT, NW, K, ST, RAG, END_CSTEP, ROE>(a, blockIdx.x);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void relax_fr_kernel(SweepArgs a)
{
    sweep_body_t<CPT, NW, K, ST, RAG, END_RESTRICT, ROE>(a, blockIdx.x);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void phi_kernel(SweepArgs a)
{
    sweep_body_t<CPT, NW, K, ST, RAG, END_PHI, ROE>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// batches of independent problems: one launch covers the chunks of every
// problem of a bucket (problems sharing a configuration and a numerical
// flux); workgroup b finds its problem by binary search over the bucket's
// chunk offsets and takes that problem's arguments from a device table
// ---------------------------------------------------------------------------
template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE>
__device__ __forceinline__ void batch_body(const BatchLaunch& t)
{
    const int b = blockIdx.x;
    int lo = 0, hi = t.nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.offset[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const SweepArgs a = t.args[t.problem[lo]];
    sweep_body_t<CPT, NW, K, ST, RAG, END, ROE>(a, b - t.offset[lo]);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void batch_f_kernel(BatchLaunch t)
{
    batch_body<CPT, NW, K, ST, RAG, END_NONE, ROE>(t);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void batch_fc_kernel(BatchLaunch t)
{
    batch_body<CPT, NW, K, ST, RAG, END_CSTEP, ROE>(t);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void batch_fr_kernel(BatchLaunch t)
{
    batch_body<CPT, NW, K, ST, RAG, END_RESTRICT, ROE>(t);
}
template <class Fn>
static hipError_t launch_batch_fn(Fn fn, const BatchLaunch& t, int nw, size_t shmem, hipStream_t s)
{
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(t.nblocks), dim3(64 * nw), shmem, s, t);
    return hipGetLastError();
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
static hipError_t launch_batch_role_f(const BatchLaunch& t, hipStream_t s)
{
    const size_t shmem = smem_bytes(CPT, NW);
    switch (t.end_mode) {
    case END_NONE: return launch_batch_fn(batch_f_kernel<CPT, NW, K, ST, RAG, ROE>, t, NW, shmem, s);
    case END_CSTEP: return launch_batch_fn(batch_fc_kernel<CPT, NW, K, ST, RAG, ROE>, t, NW, shmem, s);
    case END_RESTRICT: return launch_batch_fn(batch_fr_kernel<CPT, NW, K, ST, RAG, ROE>, t, NW, shmem, s);
    default: return hipErrorInvalidValue;
    }
}

template <int CPT, int NW, int K, int ST, bool RAG>
static hipError_t launch_batch_role(const BatchLaunch& t, hipStream_t s)
{
    if (t.roe) return launch_batch_role_f<CPT, NW, K, ST, RAG, true>(t, s);
    return launch_batch_role_f<CPT, NW, K, ST, RAG, false>(t, s);
}

template <int K, int ST>
hipError_t launch_batch_ks(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s)
{
    if (t.nblocks <= 0) return hipSuccess;
    if (cfg.cpt == 8 && cfg.nw == 16) {
        // serial solves of lines up to 8192 cells (F-steps only: the other
        // roles spill registers at this size)
        if (t.end_mode != END_NONE) return hipErrorInvalidValue;
        const size_t shmem = smem_bytes(8, 16);
        if (t.roe) {
            if (t.ragged) return launch_batch_fn(batch_f_kernel<8, 16, K, ST, true, true>, t, 16, shmem, s);
            return launch_batch_fn(batch_f_kernel<8, 16, K, ST, false, true>, t, 16, shmem, s);
        }
        if (t.ragged) return launch_batch_fn(batch_f_kernel<8, 16, K, ST, true, false>, t, 16, shmem, s);
        return launch_batch_fn(batch_f_kernel<8, 16, K, ST, false, false>, t, 16, shmem, s);
    }
#define MGK_CASE(C, W)                                                                  \
    if (cfg.cpt == C && cfg.nw == W) {                                                  \
        if (C > 1 && t.ragged) return launch_batch_role<C, W, K, ST, C == 1 ? false : true>(t, s); \
        return launch_batch_role<C, W, K, ST, false>(t, s);                             \
    }
    MGK_BATCH_CFG_LIST(MGK_CASE)
#undef MGK_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// launch over the compiled configurations
// ---------------------------------------------------------------------------
template <class Fn>
static hipError_t launch_fn(Fn fn, const SweepArgs& a, int nw, size_t shmem, hipStream_t s)
{
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(a.nchunks), dim3(64 * nw), shmem, s, a);
    return hipGetLastError();
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
static hipError_t launch_role_f(const SweepArgs& a, hipStream_t s)
{
    const size_t shmem = smem_bytes(CPT, NW);
    switch (a.end_mode) {
    case END_NONE: return launch_fn(relax_f_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    case END_CSTEP: return launch_fn(relax_fc_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    case END_RESTRICT: return launch_fn(relax_fr_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    case END_PHI: return launch_fn(phi_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    default: return hipErrorInvalidValue;
    }
}

template <int CPT, int NW, int K, int ST, bool RAG>
static hipError_t launch_role(const SweepArgs& a, hipStream_t s)
{
    if (a.pc.roe) return launch_role_f<CPT, NW, K, ST, RAG, true>(a, s);
    return launch_role_f<CPT, NW, K, ST, RAG, false>(a, s);
}

template <int CPT, int NW, int K, int ST>
static hipError_t launch_cfg(const SweepArgs& a, hipStream_t s)
{
    if constexpr (CPT > 1) {
        if (a.nx % CPT != 0) return launch_role<CPT, NW, K, ST, true>(a, s);
    }
    return launch_role<CPT, NW, K, ST, false>(a, s);
}

template <int K, int ST>
hipError_t launch_sweep_ks(const SweepArgs& a, const KernelCfg& cfg, hipStream_t s)
{
#define MGK_CASE(C, W) \
    if (cfg.cpt == C && cfg.nw == W) return launch_cfg<C, W, K, ST>(a, s);
    MGK_CFG_LIST(MGK_CASE)
#undef MGK_CASE
    return hipErrorInvalidValue;
}

}  // namespace mgk
