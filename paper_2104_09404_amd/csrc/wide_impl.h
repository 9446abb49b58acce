// wide_impl.h -- one workgroup per line for lines longer than its threads
// hold at CPT cells each (included by the wide_k*_s*.hip translation units).
//
// Used by batches for lines of 4097..8192 cells: with many lines in flight a
// line costs least on one compute unit, without the per-stage exchange of a
// split line.  Each thread runs SB "virtual threads": virtual thread
// v = s * 64 NW + t (s < SB) owns cells v CPT .. v CPT + CPT - 1, exactly the
// cells thread v would own in a workgroup of SB x 64 NW threads, and runs
// that thread's operations (reconstruct, the LF / Roe flux, the Runge-Kutta
// combination of sweep_impl.h), so results are bitwise those of every other
// arrangement.  The whole line lives in LDS (transposed: cell c at
// (c mod CPT) * SB * 64 NW + c / CPT), alpha_LF is one workgroup reduction
// per stage, and the line length must be a multiple of CPT.
#pragma once
#include "sweep_impl.h"

namespace mgk {

template <int CPT, int NW, int SB>
struct WGeo {
    static constexpr int NT = 64 * NW;     // threads
    static constexpr int NVMAX = SB * NT;  // virtual threads
    int nx;                                // cells
    int nv;                                // virtual threads that own cells (nx / CPT)
    int t;
    __device__ __forceinline__ void init(int nx_)
    {
        nx = nx_;
        nv = nx_ / CPT;
        t = threadIdx.x;
    }
    __device__ __forceinline__ int v(int s) const { return s * NT + t; }
    __device__ __forceinline__ bool active(int s) const { return v(s) < nv; }
    static __device__ __forceinline__ int slot(int c) { return (c % CPT) * NVMAX + c / CPT; }
    __device__ __forceinline__ int own(int s, int q) const { return q * NVMAX + v(s); }
};

// LDS: line[NVMAX CPT] | bm[NVMAX] | bp[NVMAX] | wred[NW] | amax[2 NW]
template <int CPT, int NW, int SB>
struct WSmem {
    double *line, *bm, *bp, *wred, *amax;
    __device__ __forceinline__ void init(double* base)
    {
        constexpr int NVMAX = WGeo<CPT, NW, SB>::NVMAX;
        line = base;
        bm = line + NVMAX * CPT;
        bp = bm + NVMAX;
        wred = bp + NVMAX;
        amax = wred + NW;
    }
};

inline size_t wide_smem_bytes(int cpt, int nw, int sb)
{
    const size_t nvmax = (size_t)sb * 64 * nw;
    return sizeof(double) * (nvmax * cpt + 2 * nvmax + 3 * (size_t)nw);
}

// A(V) of every virtual thread's cells (the operations of op_A)
template <int CPT, int NW, int SB, int K, bool ROE>
__device__ __forceinline__ void op_A_w(const double (&V)[SB][CPT], double (&A)[SB][CPT], const WGeo<CPT, NW, SB>& g,
                                       const WSmem<CPT, NW, SB>& sm, const PhiConst& pc, int& par)
{
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
        for (int q = 0; q < CPT; ++q) sm.line[g.own(s, q)] = V[s][q];
    __syncthreads();

    double um[SB][CPT], up[SB][CPT];
    double lmax = 0.0;
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        // (a virtual thread past the line's end works on the line's first cells)
        const int j0 = g.active(s) ? g.v(s) * CPT : 0;
        double w[CPT + 6];
#pragma unroll
        for (int q = 0; q < CPT; ++q) w[3 + q] = V[s][q];
        if constexpr (K > 0) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                int cl = j0 - 3 + p, cr = j0 + CPT + p;  // periodic: only the line's end cells wrap
                if (cl < 0) cl += g.nx;
                if (cr >= g.nx) cr -= g.nx;
                w[p] = sm.line[g.slot(cl)];
                w[CPT + 3 + p] = sm.line[g.slot(cr)];
            }
        }
        reconstruct<CPT, K>(w, pc.eps, um[s], up[s]);
        sm.bm[g.v(s)] = um[s][CPT - 1];
        sm.bp[g.v(s)] = up[s][0];
        if constexpr (!ROE) {
            if (g.active(s)) {
#pragma unroll
                for (int q = 0; q < CPT; ++q) lmax = fmax(lmax, fmax(fabs(um[s][q]), fabs(up[s][q])));
            }
        }
    }
    double alpha = 0.0;
    if constexpr (ROE) {
        __syncthreads();
    } else {
        lmax = wave_max(lmax);
        if ((threadIdx.x & 63) == 0) sm.amax[par * NW + (threadIdx.x >> 6)] = lmax;
        __syncthreads();
        alpha = pc.alpha_fixed;
        if (!(alpha > 0.0)) {
#pragma unroll
            for (int w2 = 0; w2 < NW; ++w2) lmax = fmax(lmax, sm.amax[par * NW + w2]);
            alpha = lf_alpha(lmax, pc.fa, pc.fb);
        }
        par ^= 1;
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        const int v = g.v(s);
        const int left = (v == 0) ? g.nv - 1 : v - 1;
        const int right = (v == g.nv - 1) ? 0 : v + 1;
        const int lv = g.active(s) ? left : v, rv = g.active(s) ? right : v;
        const double uml = sm.bm[lv];
        const double upr = sm.bp[rv];
        double F[CPT + 1];
#pragma unroll
        for (int q = 0; q <= CPT; ++q) {
            const double uL = (q == 0) ? uml : um[s][q - 1];
            const double uR = (q == CPT) ? upr : up[s][q];
            if constexpr (ROE) F[q] = roe_flux2(uL, uR, pc.fa, pc.fb);
            else F[q] = lf_flux2(uL, uR, pc.fa, pc.fb, alpha);
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q) A[s][q] = (F[q] - F[q + 1]) * pc.half_inv_dx;
    }
}

// x <- Phi(x) with step dt (the operations of phi)
template <int CPT, int NW, int SB, int K, int ST, bool ROE>
__device__ __forceinline__ void phi_w(double (&x)[SB][CPT], double dt, const WGeo<CPT, NW, SB>& g,
                                      const WSmem<CPT, NW, SB>& sm, const PhiConst& pc, int& par)
{
    double A[SB][CPT];
    if constexpr (ST == 1) {
        op_A_w<CPT, NW, SB, K, ROE>(x, A, g, sm, pc, par);
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int q = 0; q < CPT; ++q) x[s][q] = rk_first(x[s][q], A[s][q], dt);
    } else if constexpr (ST == 2) {
        double v[SB][CPT];
        op_A_w<CPT, NW, SB, K, ROE>(x, A, g, sm, pc, par);
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int q = 0; q < CPT; ++q) v[s][q] = rk_first(x[s][q], A[s][q], dt);
        op_A_w<CPT, NW, SB, K, ROE>(v, A, g, sm, pc, par);
        const double hdt = 0.5 * dt;
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int q = 0; q < CPT; ++q) x[s][q] = rk2_second(x[s][q], v[s][q], A[s][q], hdt);
    } else {
        double v[SB][CPT];
        op_A_w<CPT, NW, SB, K, ROE>(x, A, g, sm, pc, par);
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int q = 0; q < CPT; ++q) v[s][q] = rk_first(x[s][q], A[s][q], dt);
        op_A_w<CPT, NW, SB, K, ROE>(v, A, g, sm, pc, par);
        const double qdt = 0.25 * dt;
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int q = 0; q < CPT; ++q) v[s][q] = rk3_second(x[s][q], v[s][q], A[s][q], qdt);
        op_A_w<CPT, NW, SB, K, ROE>(v, A, g, sm, pc, par);
        const double tdt = (2.0 / 3.0) * dt;
#pragma unroll
        for (int s = 0; s < SB; ++s)
#pragma unroll
            for (int q = 0; q < CPT; ++q) x[s][q] = rk3_third(x[s][q], v[s][q], A[s][q], tdt);
    }
}

// line transfers of the thread's cells (virtual threads past the line's end
// read cell 0 and store nothing)
template <int CPT, int NW, int SB>
__device__ __forceinline__ void w_load(double (&x)[SB][CPT], const double* src, const WGeo<CPT, NW, SB>& g)
{
#pragma unroll
    for (int s = 0; s < SB; ++s) {
        const int j0 = g.active(s) ? g.v(s) * CPT : 0;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[s][q] = src[j0 + q];
    }
}

template <int CPT, int NW, int SB>
__device__ __forceinline__ void w_store(const double (&x)[SB][CPT], double* dst, const WGeo<CPT, NW, SB>& g)
{
#pragma unroll
    for (int s = 0; s < SB; ++s)
        if (g.active(s)) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) dst[g.v(s) * CPT + q] = x[s][q];
        }
}

template <int CPT, int NW, int SB>
__device__ __forceinline__ void w_add(double (&x)[SB][CPT], const double* src, const WGeo<CPT, NW, SB>& g)
{
    double t[SB][CPT];
    w_load(t, src, g);
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[s][q] = x[s][q] + t[s][q];
}

template <int CPT, int NW, int SB>
__device__ __forceinline__ void w_copy(const double* src, double* dst, const WGeo<CPT, NW, SB>& g)
{
    double t[SB][CPT];
    w_load(t, src, g);
    w_store(t, dst, g);
}

// sum over the line of (x - b)^2 in a fixed order; valid in thread 0
template <int CPT, int NW, int SB>
__device__ __forceinline__ double w_sqdiff(const double (&x)[SB][CPT], const double* b, const WGeo<CPT, NW, SB>& g,
                                           const WSmem<CPT, NW, SB>& sm)
{
    double t[SB][CPT];
    w_load(t, b, g);
    double sum = 0.0;
#pragma unroll
    for (int s = 0; s < SB; ++s)
        if (g.active(s)) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const double d = x[s][q] - t[s][q];
                sum = fma(d, d, sum);
            }
        }
    sum = wave_sum(sum);
    if ((threadIdx.x & 63) == 0) sm.wred[threadIdx.x >> 6] = sum;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NW; ++w) tot += sm.wred[w];
    }
    return tot;
}

// One chunk of one line (the roles END_NONE, END_CSTEP and END_RESTRICT of
// sweep_body_t, Phi steps only).  The chunk's residual partial goes to
// resid_partial[c * P], the other P - 1 entries of the chunk (P = a.tiles,
// the partials per chunk of the problem's layout) are zero.
template <int CPT, int NW, int SB, int K, int ST, int END, bool ROE>
__device__ __forceinline__ void wide_body(const SweepArgs& a, const int c)
{
    if (a.flag != nullptr && *a.flag != 0) return;
    extern __shared__ double smem_raw[];
    WSmem<CPT, NW, SB> sm;
    sm.init(smem_raw);
    WGeo<CPT, NW, SB> g;
    g.init(a.nx);
    int par = 0;
    const int64_t nx = a.nx;

    const double* src = (a.side_in != nullptr && c > 0) ? a.side_in + (int64_t)c * nx
                                                        : a.ustart + (int64_t)c * a.ustart_stride * nx;
    double x[SB][CPT];
    w_load(x, src, g);
    if (a.ucommit != nullptr) w_store(x, a.ucommit + (int64_t)c * a.ucommit_stride * nx, g);
    if (a.inject_last && c == a.nchunks - 1) {
        const double* last = (a.side_in != nullptr) ? a.side_in + (int64_t)a.nchunks * nx
                                                    : a.ustart + (int64_t)a.nchunks * a.ustart_stride * nx;
        w_copy(last, a.ucommit + (int64_t)a.nchunks * a.ucommit_stride * nx, g);
    }
    const double* cstart = (a.ystart != nullptr) ? a.ystart + (int64_t)c * a.ystart_stride * nx : src;
    if (END == END_RESTRICT && c == 0) {
        w_copy(cstart, a.uc_out, g);
        w_copy(a.g != nullptr ? a.g : cstart, a.gc_out, g);
    }
    wait_loads();

    const int64_t n0 = (int64_t)c * a.m;
    const int64_t n1 = n0 + a.m;
    const int every = a.fout_every > 1 ? a.fout_every : 1;
    for (int j = 1; j <= a.nsteps; ++j) {
        phi_w<CPT, NW, SB, K, ST, ROE>(x, a.dt, g, sm, a.pc, par);
        if (a.g != nullptr) w_add(x, a.g + (n0 + j) * nx, g);
        if (a.fout != nullptr && (n0 + j) % every == 0) w_store(x, a.fout + ((n0 + j) / every) * nx, g);
    }
    if constexpr (END == END_NONE) return;

    phi_w<CPT, NW, SB, K, ST, ROE>(x, a.dt, g, sm, a.pc, par);
    if (a.g != nullptr) w_add(x, a.g + n1 * nx, g);
    const double* cnext = a.cref + (int64_t)(c + 1) * a.cref_stride * nx;
    if (a.resid_partial != nullptr) {
        const double sq = w_sqdiff(x, cnext, g, sm);
        const int P = a.tiles > 1 ? a.tiles : 1;
        if (threadIdx.x < P) a.resid_partial[(int64_t)c * P + threadIdx.x] = (threadIdx.x == 0) ? sq : 0.0;
    }
    if (a.r_out != nullptr) {
        double t[SB][CPT];
        w_load(t, cnext, g);
#pragma unroll
        for (int s = 0; s < SB; ++s)
            if (g.active(s)) {
#pragma unroll
                for (int q = 0; q < CPT; ++q) a.r_out[(int64_t)c * nx + g.v(s) * CPT + q] = x[s][q] - t[s][q];
            }
    }
    if constexpr (END == END_CSTEP) {
        if (a.side_out != nullptr) w_store(x, a.side_out + (int64_t)(c + 1) * nx, g);
        return;
    }
    if (a.coarse_injection) w_copy(cnext, a.uc_out + (int64_t)(c + 1) * nx, g);
    else w_store(x, a.uc_out + (int64_t)(c + 1) * nx, g);
    double y[SB][CPT];
    w_load(y, cstart, g);
    PhiConst pcn = a.pc;
    if (a.alpha_next > 0.0) pcn.alpha_fixed = a.alpha_next;
    phi_w<CPT, NW, SB, K, ST, ROE>(y, a.dt_next, g, sm, pcn, par);
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
        for (int q = 0; q < CPT; ++q) y[s][q] = x[s][q] - y[s][q];
    w_store(y, a.gc_out + (int64_t)(c + 1) * nx, g);
}

template <int CPT, int NW, int SB, int K, int ST, int END, bool ROE>
__device__ __forceinline__ void wide_batch_body(const BatchLaunch& t)
{
    const int b = blockIdx.x;
    int lo = 0, hi = t.nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.offset[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const SweepArgs a = t.args[t.problem[lo]];
    wide_body<CPT, NW, SB, K, ST, END, ROE>(a, b - t.offset[lo]);
}

template <int CPT, int NW, int SB, int K, int ST, bool ROE>
__global__ __launch_bounds__(64 * NW) void wide_batch_f_kernel(BatchLaunch t)
{
    wide_batch_body<CPT, NW, SB, K, ST, END_NONE, ROE>(t);
}
template <int CPT, int NW, int SB, int K, int ST, bool ROE>
__global__ __launch_bounds__(64 * NW) void wide_batch_fc_kernel(BatchLaunch t)
{
    wide_batch_body<CPT, NW, SB, K, ST, END_CSTEP, ROE>(t);
}
template <int CPT, int NW, int SB, int K, int ST, bool ROE>
__global__ __launch_bounds__(64 * NW) void wide_batch_fr_kernel(BatchLaunch t)
{
    wide_batch_body<CPT, NW, SB, K, ST, END_RESTRICT, ROE>(t);
}

template <int CPT, int NW, int SB, int K, int ST, bool ROE>
static hipError_t launch_wide_role(const BatchLaunch& t, hipStream_t s)
{
    const size_t shmem = wide_smem_bytes(CPT, NW, SB);
    switch (t.end_mode) {
    case END_NONE: return launch_batch_fn(wide_batch_f_kernel<CPT, NW, SB, K, ST, ROE>, t, NW, shmem, s);
    case END_CSTEP: return launch_batch_fn(wide_batch_fc_kernel<CPT, NW, SB, K, ST, ROE>, t, NW, shmem, s);
    case END_RESTRICT: return launch_batch_fn(wide_batch_fr_kernel<CPT, NW, SB, K, ST, ROE>, t, NW, shmem, s);
    default: return hipErrorInvalidValue;
    }
}

// wide batch launch of shape (cfg.cpt, cfg.nw) with cfg.intervals sub-blocks
template <int K, int ST>
hipError_t launch_wide_batch_ks(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s)
{
    if (t.nblocks <= 0) return hipSuccess;
    // with the Roe flux or ragged lines these kernels spill registers: such
    // lines stay split
    if (t.ragged || t.roe) return hipErrorInvalidValue;
    // WENO7 spills registers here as well (the batch keeps its lines split)
    if constexpr (K == 3) return hipErrorInvalidValue;
#define MGK_CASE(C, W, B)                                                   \
    if (cfg.cpt == C && cfg.nw == W && cfg.intervals == B) return launch_wide_role<C, W, B, K, ST, false>(t, s);
    MGK_WIDE_CFG_LIST(MGK_CASE)
#undef MGK_CASE
    return hipErrorInvalidValue;
}

}  // namespace mgk
