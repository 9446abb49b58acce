// adjoint_impl.h -- gfx950 kernels of the discrete adjoint of Phi (included by
// the adjoint_k*_s*.hip translation units).
//
// One workgroup per line.  The adjoint lambda stays in registers while the
// kernel walks backwards over the steps of a stretch of trajectory; for each
// step it runs the Runge-Kutta stages in reverse (eq SSPRK1/2/3 transposed),
// and each stage applies J_A(v)^T mu, the transpose of the Jacobian of the
// semi-discrete operator (eq spaceDisc with eq LFflux), in four phases:
//   1. the stage state v goes to LDS (for the 3-cell halo) and every thread
//      publishes the first and last mu of its cells; barrier;
//   2. per cell j: reconstructions u^-_{j+1/2}, u^+_{j-1/2}, the adjoints of the
//      two fluxes touching it, g_j = (mu_{j+1} - mu_j)/dx and g_{j-1}, the
//      candidate for the alpha_LF maximum (value, key) and the cell's share of
//      the adjoint of alpha_LF; wave reductions, one slot per wave; barrier;
//   3. alpha_LF, the key of the first maximising (interface, side) and the
//      adjoint of alpha_LF; reverse of the flux and of the WENO5 arithmetic of
//      the cell (cell_math.h); contributions to cells owned by neighbouring
//      threads go to target-indexed LDS slots (each slot has exactly one
//      writer); barrier;
//   4. every thread adds the slots of its own cells.
// Lines must be a multiple of the cells per thread (no ragged thread).
#pragma once
#include "sweep_impl.h"

namespace mgk {

// LDS of J_A^T: lineV[cap] | MF[NT] | ML[NT] | SP[nsp][cap] | slots[3 NW]
template <int CPT, int NW>
struct SmemAdj {
    static constexpr int NT = 64 * NW;
    static constexpr int CAP = NT * CPT;
    static constexpr int NSP = (CPT == 1) ? 4 : 2;
    double* lineV;
    double* MF;
    double* ML;
    double* SP[4];
    double* slots;
    __device__ __forceinline__ void init(double* base)
    {
        lineV = base;
        MF = lineV + CAP;
        ML = MF + NT;
        double* p = ML + NT;
        for (int i = 0; i < 4; ++i) {
            SP[i] = p;
            if (i < NSP) p += CAP;
        }
        slots = p;
    }
};

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// out = J_A(v)^T mu for the thread's cells
template <int CPT, int NW, int K>
__device__ __forceinline__ void op_AT(const double (&v)[CPT], const double (&mu)[CPT], double (&out)[CPT],
                                      const Geo<CPT, NW>& g, const SmemAdj<CPT, NW>& sa, const PhiConst& pc)
{
    // phase 1
#pragma unroll
    for (int q = 0; q < CPT; ++q) sa.lineV[g.own(q)] = v[q];
    sa.MF[g.t] = mu[0];
    sa.ML[g.t] = mu[CPT - 1];
    __syncthreads();

    // phase 2
    double w[CPT + 6];
#pragma unroll
    for (int q = 0; q < CPT; ++q) w[3 + q] = v[q];
    double um[CPT], up[CPT];
    if (K == 0) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            um[q] = w[3 + q];
            up[q] = w[3 + q];
        }
    } else {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            w[p] = sa.lineV[g.halo[p]];
            w[CPT + 3 + p] = sa.lineV[g.halo[3 + p]];
        }
        double E[CPT + 6];
#pragma unroll
        for (int p = 2; p <= CPT + 3; ++p) E[p] = weno5_e(w[p - 1], w[p], w[p + 1], pc.eps);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int p = q + 3;
            weno5_cell(w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], E[p - 1], E[p], E[p + 1], um[q], up[q]);
        }
    }
    const double mu_l = sa.ML[g.left];
    const double mu_r = sa.MF[g.right];
    const double inv_dx = 2.0 * pc.half_inv_dx;
    double gr[CPT], gl[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const double mn = (q + 1 < CPT) ? mu[q + 1] : mu_r;
        const double mp = (q > 0) ? mu[q - 1] : mu_l;
        gr[q] = (mn - mu[q]) * inv_dx;
        gl[q] = (mu[q] - mp) * inv_dx;
    }
    // alpha_LF candidates: u^-_k has key 2k, u^+_k (the left face of cell k+1) key 2k+1;
    // the oracle's scan order makes the smallest key win a tie
    double bv = -1.0, bk = 0.0, ab = 0.0;
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int j = g.j0 + q;
            const double km = 2.0 * (double)j;
            const double kp = 2.0 * (double)(j == 0 ? g.nx - 1 : j - 1) + 1.0;
            const double am = fabs(um[q]), ap = fabs(up[q]);
            if (am > bv || (am == bv && km < bk)) {
                bv = am;
                bk = km;
            }
            if (ap > bv || (ap == bv && kp < bk)) {
                bv = ap;
                bk = kp;
            }
            ab = fma(0.5 * gr[q], um[q], ab);
            ab = fma(-0.5 * gl[q], up[q], ab);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const double ok = __shfl_xor(bk, o, 64);
        if (ov > bv || (ov == bv && ok < bk)) {
            bv = ov;
            bk = ok;
        }
        ab = ab + __shfl_xor(ab, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        const int wv = threadIdx.x >> 6;
        sa.slots[3 * wv] = bv;
        sa.slots[3 * wv + 1] = bk;
        sa.slots[3 * wv + 2] = ab;
    }
    __syncthreads();

    // phase 3
    double mv = sa.slots[0], mk = sa.slots[1], abar = sa.slots[2];
#pragma unroll
    for (int wv = 1; wv < NW; ++wv) {
        const double ov = sa.slots[3 * wv], ok = sa.slots[3 * wv + 1];
        if (ov > mv || (ov == mv && ok < mk)) {
            mv = ov;
            mk = ok;
        }
        abar = abar + sa.slots[3 * wv + 2];
    }
    double alpha, csub;
    if (pc.alpha_fixed > 0.0) {
        alpha = pc.alpha_fixed;
        csub = 0.0;
    } else {
        alpha = lf_alpha(mv, pc.fa, pc.fb);
        csub = abar * 2.0 * fabs(pc.fa);  // d alpha / d u* = 2|fa| sign(u*)
    }
    double acc[CPT + 4];
#pragma unroll
    for (int i = 0; i < CPT + 4; ++i) acc[i] = 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int j = g.j0 + q;
        const double km = 2.0 * (double)j;
        const double kp = 2.0 * (double)(j == 0 ? g.nx - 1 : j - 1) + 1.0;
        const double cm = (km == mk) ? csub : 0.0;
        const double cp = (kp == mk) ? csub : 0.0;
        const double grq = gr[q], glq = gl[q];
        auto adj = [&](double um_, double up_, double& umb, double& upb) {
            umb = fma(cm, sgn(um_), grq * fma(0.5, flux_fprime(um_, pc.fa, pc.fb), 0.5 * alpha));
            upb = fma(cp, sgn(up_), glq * fma(0.5, flux_fprime(up_, pc.fa, pc.fb), -0.5 * alpha));
        };
        if (K == 0) {
            double umb, upb;
            adj(w[3 + q], w[3 + q], umb, upb);
            acc[q + 2] += umb + upb;
        } else {
            const int p = q + 3;
            weno5_cell_vjp_f(w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], pc.eps, adj, &acc[q]);
        }
        // one cell at a time: keeps the live intermediates of the reverse pass bounded
        __builtin_amdgcn_sched_barrier(0);
    }
    if (g.active) {
        if (CPT == 1) {
            sa.SP[0][wrapi(g.j0 - 1, g.nx)] = acc[1];
            sa.SP[2][wrapi(g.j0 - 2, g.nx)] = acc[0];
            sa.SP[1][wrapi(g.j0 + 1, g.nx)] = acc[3];
            sa.SP[3][wrapi(g.j0 + 2, g.nx)] = acc[4];
        } else {
            sa.SP[0][wrapi(g.j0 - 1, g.nx)] = acc[1];
            sa.SP[0][wrapi(g.j0 - 2, g.nx)] = acc[0];
            sa.SP[1][wrapi(g.j0 + CPT, g.nx)] = acc[CPT + 2];
            sa.SP[1][wrapi(g.j0 + CPT + 1, g.nx)] = acc[CPT + 3];
        }
    }
    __syncthreads();

    // phase 4
    if (CPT == 1) {
        out[0] = acc[2] + sa.SP[0][g.j0] + sa.SP[1][g.j0] + sa.SP[2][g.j0] + sa.SP[3][g.j0];
    } else {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            double o = acc[q + 2];
            if (q >= CPT - 2) o += sa.SP[0][g.j0 + q];
            if (q <= 1) o += sa.SP[1][g.j0 + q];
            out[q] = o;
        }
    }
}

// Forward stages of one step, keeping the stage inputs: s0 = u, s1, s2 (eq SSPRK).
template <int CPT, int NW, int K, int ST>
__device__ __forceinline__ void fwd_stages(const double (&u)[CPT], double (&s1)[CPT], double (&s2)[CPT], double dt,
                                           const Geo<CPT, NW>& g, const Smem<CPT, NW>& sm, const PhiConst& pc,
                                           int& par)
{
    if (ST == 1) return;
    double A[CPT];
    op_A<CPT, NW, K, false>(u, A, g, sm, pc, par);
#pragma unroll
    for (int q = 0; q < CPT; ++q) s1[q] = rk_first(u[q], A[q], dt);
    if (ST == 3) {
        op_A<CPT, NW, K, false>(s1, A, g, sm, pc, par);
#pragma unroll
        for (int q = 0; q < CPT; ++q) s2[q] = rk3_second(u[q], s1[q], A[q], 0.25 * dt);
    }
}

// lam <- (dPhi/du)^T lam; stage(s, v) fills v with the input of stage s of the step
template <int CPT, int NW, int K, int ST, class Stage>
__device__ __forceinline__ void rev_step(double (&lam)[CPT], Stage&& stage, double dt, const Geo<CPT, NW>& g,
                                         const SmemAdj<CPT, NW>& sa, const PhiConst& pc)
{
    double t[CPT], v[CPT];
    if (ST == 1) {
        // y = u + dt A(u)
        stage(0, v);
        op_AT<CPT, NW, K>(v, lam, t, g, sa, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) lam[q] = fma(dt, t[q], lam[q]);
    } else if (ST == 2) {
        // y = u/2 + s1/2 + dt/2 A(s1), s1 = u + dt A(u)
        double l1[CPT];
        stage(1, v);
        op_AT<CPT, NW, K>(v, lam, t, g, sa, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) l1[q] = fma(0.5 * dt, t[q], 0.5 * lam[q]);
        stage(0, v);
        op_AT<CPT, NW, K>(v, l1, t, g, sa, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) lam[q] = fma(dt, t[q], fma(0.5, lam[q], l1[q]));
    } else {
        // y = u/3 + 2 s2/3 + 2dt/3 A(s2); s2 = 3u/4 + s1/4 + dt/4 A(s1); s1 = u + dt A(u)
        double l1[CPT], l2[CPT];
        stage(2, v);
        op_AT<CPT, NW, K>(v, lam, t, g, sa, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            l2[q] = fma((2.0 / 3.0) * dt, t[q], (2.0 / 3.0) * lam[q]);
            lam[q] = (1.0 / 3.0) * lam[q];
        }
        stage(1, v);
        op_AT<CPT, NW, K>(v, l2, t, g, sa, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            l1[q] = fma(0.25 * dt, t[q], 0.25 * l2[q]);
            lam[q] = fma(0.75, l2[q], lam[q]);
        }
        stage(0, v);
        op_AT<CPT, NW, K>(v, l1, t, g, sa, pc);
#pragma unroll
        for (int q = 0; q < CPT; ++q) lam[q] = fma(dt, t[q], lam[q] + l1[q]);
    }
}

template <int CPT, int NW>
constexpr size_t adj_smem_bytes(bool stored)
{
    return sizeof(double) * ((stored ? 0 : (size_t)64 * NW * CPT + 2 * 64 * NW + 3 * NW) +              // forward op_A
                             (size_t)64 * NW * CPT + 2 * 64 * NW + (CPT == 1 ? 4 : 2) * 64 * NW * CPT +  // J_A^T
                             3 * NW);
}

// Reverse sweep over nsteps steps of line b.  STORED: the stage inputs of step
// n are read from traj + b*traj_stride + (n*ST + s)*nx; otherwise nsteps == 1
// and they are recomputed from u + b*nx.
template <int CPT, int NW, int K, int ST, bool STORED>
__global__ __launch_bounds__(64 * NW) void adjoint_kernel(AdjArgs a)
{
    extern __shared__ double smem_raw[];
    SmemAdj<CPT, NW> sa;
    sa.init(smem_raw + (STORED ? 0 : 64 * NW * CPT + 2 * 64 * NW + 3 * NW));
    Geo<CPT, NW> g;
    g.init(a.nx);
    const int64_t nx = a.nx;
    const int64_t b = blockIdx.x;
    double lam[CPT];
    load_line(lam, a.lam_in + b * nx, g);
    if constexpr (STORED) {
        for (int n = a.nsteps - 1; n >= 0; --n) {
            const double* base = a.traj + b * a.traj_stride + (int64_t)n * ST * nx;
            rev_step<CPT, NW, K, ST>(
                lam, [&](int st, double(&v)[CPT]) { load_line(v, base + st * nx, g); }, a.dt, g, sa, a.pc);
        }
    } else {
        Smem<CPT, NW> sm;
        sm.init(smem_raw);
        int par = 0;
        double u[CPT], s1[CPT], s2[CPT];
        load_line(u, a.u + b * nx, g);
        fwd_stages<CPT, NW, K, ST>(u, s1, s2, a.dt, g, sm, a.pc, par);
        rev_step<CPT, NW, K, ST>(
            lam,
            [&](int st, double(&v)[CPT]) {
#pragma unroll
                for (int q = 0; q < CPT; ++q) v[q] = st == 0 ? u[q] : (st == 1 ? s1[q] : s2[q]);
            },
            a.dt, g, sa, a.pc);
    }
    store_line(lam, a.lam_out + b * nx, g);
}

// Forward steps storing the stage inputs: line b starts from u0 + b*u0_stride*nx
// and writes step n's stage inputs to traj + b*traj_stride + (n*ST + s)*nx.
template <int CPT, int NW, int K, int ST>
__global__ __launch_bounds__(64 * NW) void stage_store_kernel(AdjArgs a)
{
    extern __shared__ double smem_raw[];
    Smem<CPT, NW> sm;
    sm.init(smem_raw);
    Geo<CPT, NW> g;
    g.init(a.nx);
    int par = 0;
    const int64_t nx = a.nx;
    const int64_t b = blockIdx.x;
    double x[CPT];
    load_line(x, a.u + b * a.u_stride * nx, g);
    for (int n = 0; n < a.nsteps; ++n) {
        double* base = a.traj_out + b * a.traj_stride + (int64_t)n * ST * nx;
        double s1[CPT], s2[CPT];
        store_line(x, base, g);
        fwd_stages<CPT, NW, K, ST>(x, s1, s2, a.dt, g, sm, a.pc, par);
        if (ST >= 2) store_line(s1, base + nx, g);
        if (ST == 3) store_line(s2, base + 2 * nx, g);
        // finish the step
        double A[CPT];
        if (ST == 1) {
            op_A<CPT, NW, K, false>(x, A, g, sm, a.pc, par);
#pragma unroll
            for (int q = 0; q < CPT; ++q) x[q] = rk_first(x[q], A[q], a.dt);
        } else if (ST == 2) {
            op_A<CPT, NW, K, false>(s1, A, g, sm, a.pc, par);
#pragma unroll
            for (int q = 0; q < CPT; ++q) x[q] = rk2_second(x[q], s1[q], A[q], 0.5 * a.dt);
        } else {
            op_A<CPT, NW, K, false>(s2, A, g, sm, a.pc, par);
#pragma unroll
            for (int q = 0; q < CPT; ++q) x[q] = rk3_third(x[q], s2[q], A[q], (2.0 / 3.0) * a.dt);
        }
    }
}

template <class Fn>
static hipError_t launch_adj_fn(Fn fn, const AdjArgs& a, int nw, size_t shmem, hipStream_t s)
{
    if (shmem > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(a.nlines), dim3(64 * nw), shmem, s, a);
    return hipGetLastError();
}

template <int K, int ST>
hipError_t launch_adjoint_ks(const AdjArgs& a, const KernelCfg& cfg, int store_mode, hipStream_t s)
{
#define MGK_ADJ_CASE(C, W)                                                                                  \
    if (cfg.cpt == C && cfg.nw == W) {                                                                      \
        if (store_mode) return launch_adj_fn(stage_store_kernel<C, W, K, ST>, a, W, smem_bytes(C, W), s);        \
        if (a.stored) return launch_adj_fn(adjoint_kernel<C, W, K, ST, true>, a, W, adj_smem_bytes<C, W>(true), s); \
        return launch_adj_fn(adjoint_kernel<C, W, K, ST, false>, a, W, adj_smem_bytes<C, W>(false), s);         \
    }
    MGK_ADJ_CFG_LIST(MGK_ADJ_CASE)
#undef MGK_ADJ_CASE
    return hipErrorInvalidValue;
}

}  // namespace mgk
