// tiled_adjoint_impl.h -- the discrete adjoint on lines split over several
// workgroups (included by the tiled_adjoint_k*_s*.hip translation units).
//
// Reverse sweep (tiled_adjoint_kernel).  Tile g of a line (balanced lengths,
// as for the forward split lines) is owned by one workgroup, which keeps the
// adjoint of its cells in registers and walks backwards over the steps of a
// stored trajectory (the stage inputs of every step, written by
// tiled_stage_store_kernel).  Per reverse Runge-Kutta stage, J_A(v)^T mu:
//   1. the stage input v of the tile plus 4 cells on each side is read from
//      HBM into LDS, mu of the tile into LDS;
//   2. reconstructions of the tile's cells (plus the two edge neighbours), the
//      tile's candidate for the alpha_LF maximum (value, key) and its share of
//      the adjoint of alpha_LF, written by summation by parts as
//          abar = 1/(2 dx) sum_j mu_j (d_{j-1} - d_j),  d_k = u^-_{k+1/2} - u^+_{k+1/2},
//      which needs mu of the tile only;
//   3. the tile publishes (value, key, share) and mu of its three first and
//      three last cells, meets the other tiles of the line at a global
//      counter, and reads back every tile's triple (all tiles combine them in
//      the same order) and its neighbours' edge mu;
//   4. reverse of the flux and WENO5 arithmetic for its cells and for the two
//      cells beyond each edge (their contributions to the tile's edge cells);
//      contributions between threads go through target-indexed LDS slots.
// One global synchronisation per reverse stage.
//
// Recompute (tiled_stage_store_kernel): forward steps of a split line (the
// forward split-line machinery of tiled_impl.h) storing every stage input.
#pragma once
#include "adjoint_impl.h"
#include "tiled_impl.h"

namespace mgk {

// LDS: V[T + 8] (tile cell c at c + 4) | MU[T + 6] (c at c + 3) | bm[NT] | bp[NT] |
//      SP[nsp][T] | HC[8] | red[3 NW] | misc[8]
template <int CPT, int NW>
struct TASmem {
    static constexpr int NT = 64 * NW;
    static constexpr int T = NT * CPT;
    static constexpr int NSP = (CPT == 1) ? 4 : 2;
    double* V;
    double* MU;
    double* bm;
    double* bp;
    double* SP[4];
    double* HC;
    double* red;
    double* misc;
    __device__ __forceinline__ void init(double* base)
    {
        V = base;
        MU = V + T + 8;
        bm = MU + T + 6;
        bp = bm + NT;
        double* p = bp + NT;
        for (int i = 0; i < 4; ++i) {
            SP[i] = p;
            if (i < NSP) p += T;
        }
        HC = p;
        red = HC + 8;
        misc = red + 3 * NW;
    }
};

template <int CPT, int NW>
constexpr size_t tiled_adj_smem_bytes()
{
    return sizeof(double) * ((size_t)64 * NW * CPT + 8 + (size_t)64 * NW * CPT + 6 + 2 * 64 * NW +
                             (CPT == 1 ? 4 : 2) * (size_t)64 * NW * CPT + 8 + 3 * NW + 8);
}

// (value, key) pair order of the alpha_LF maximum: larger value, then smaller key
__device__ __forceinline__ bool key_better(double ov, double ok, double bv, double bk)
{
    return ov > bv || (ov == bv && ok < bk);
}

// out = J_A(v)^T mu for the tile's cells; v is the stage input line in HBM.
template <int CPT, int NW, int K>
__device__ __forceinline__ bool op_AT_t(const double* vline, const double (&mu)[CPT], double (&out)[CPT],
                                        const TGeo<CPT, NW>& g, const TASmem<CPT, NW>& sa, const PhiConst& pc,
                                        TSync& ts, int64_t nx)
{
    // phase 1: v (tile + 4 cells each side) and mu of the tile into LDS
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            sa.V[4 + g.j0 + q] = vline[g.x0 + g.j0 + q];
            sa.MU[3 + g.j0 + q] = mu[q];
        }
    }
    if (threadIdx.x < 8) {
        const int c = (threadIdx.x < 4) ? (int)threadIdx.x - 4 : g.Tv + ((int)threadIdx.x - 4);
        int64_t cell = (g.x0 + c) % nx;
        if (cell < 0) cell += nx;
        sa.V[4 + c] = vline[cell];
    }
    __syncthreads();

    // phase 2: reconstructions, alpha_LF candidate, share of the adjoint of alpha_LF
    double w[CPT + 6];  // tile cells j0-3 .. j0+CPT+2
#pragma unroll
    for (int p = 0; p < CPT + 6; ++p) w[p] = sa.V[g.j0 + 1 + p];
    double um[CPT], up[CPT];
    double um_l = 0.0, up_r = 0.0;  // u^- of cell j0-1 (thread 0), u^+ of cell Tv (last thread)
    if (K == 0) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            um[q] = w[3 + q];
            up[q] = w[3 + q];
        }
        um_l = w[2];
        up_r = w[CPT + 3];
    } else {
        double E[CPT + 6];
#pragma unroll
        for (int p = 1; p <= CPT + 4; ++p) E[p] = weno5_e(w[p - 1], w[p], w[p + 1], pc.eps);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int p = q + 3;
            weno5_cell(w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], E[p - 1], E[p], E[p + 1], um[q], up[q]);
        }
        if (g.t == 0) {
            double unused;
            weno5_cell(w[0], w[1], w[2], w[3], w[4], E[1], E[2], E[3], um_l, unused);
        }
        if (g.t == g.tlast) {
            double unused;
            weno5_cell(w[CPT + 1], w[CPT + 2], w[CPT + 3], w[CPT + 4], w[CPT + 5], E[CPT + 2], E[CPT + 3],
                       E[CPT + 4], unused, up_r);
        }
    }
    sa.bm[g.t] = um[CPT - 1];
    sa.bp[g.t] = up[0];
    // candidates: u^-_k has key 2k, u^+_k (the left face of cell k+1) key 2k+1
    double bv = -1.0, bk = 0.0, ab = 0.0;
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int64_t j = g.x0 + g.j0 + q;
            const double km = 2.0 * (double)j;
            const double kp = 2.0 * (double)(j == 0 ? nx - 1 : j - 1) + 1.0;
            const double am = fabs(um[q]), ap = fabs(up[q]);
            if (key_better(am, km, bv, bk)) {
                bv = am;
                bk = km;
            }
            if (key_better(ap, kp, bv, bk)) {
                bv = ap;
                bk = kp;
            }
        }
    }
    __syncthreads();
    if (g.active) {
        const double uml = (g.t == 0) ? um_l : sa.bm[g.t - 1];
        const double upr = (g.t == g.tlast) ? up_r : sa.bp[min(g.t + 1, 64 * NW - 1)];
        double dprev = uml - up[0];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const double d = um[q] - ((q + 1 < CPT) ? up[q + 1] : upr);
            ab = fma(mu[q], dprev - d, ab);
            dprev = d;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const double ok = __shfl_xor(bk, o, 64);
        if (key_better(ov, ok, bv, bk)) {
            bv = ov;
            bk = ok;
        }
        ab = ab + __shfl_xor(ab, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        const int wv = threadIdx.x >> 6;
        sa.red[3 * wv] = bv;
        sa.red[3 * wv + 1] = bk;
        sa.red[3 * wv + 2] = ab;
    }
    __syncthreads();

    // publish and meet the other tiles (see op_A_t for the ordering argument)
    const int parity = ts.ep & 1;
    ts.ep += 1;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane < 9) {
            double val;
            if (lane < 3) {
                double tv = sa.red[0], tk = sa.red[1], ta = sa.red[2];
#pragma unroll
                for (int wv = 1; wv < NW; ++wv) {
                    if (key_better(sa.red[3 * wv], sa.red[3 * wv + 1], tv, tk)) {
                        tv = sa.red[3 * wv];
                        tk = sa.red[3 * wv + 1];
                    }
                    ta = ta + sa.red[3 * wv + 2];
                }
                val = (lane == 0) ? tv : (lane == 1 ? tk : ta);
            } else if (lane < 6) {
                val = sa.MU[3 + (lane - 3)];  // first three cells
            } else {
                val = sa.MU[3 + g.Tv - 3 + (lane - 6)];  // last three cells
            }
            __hip_atomic_store(ts.slot(ts.tile, parity) + lane, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_s_waitcnt(0);
        if (lane == 0) {
            __hip_atomic_fetch_add(ts.cnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long target = (unsigned long long)ts.G * (unsigned long long)ts.ep;
            long long spins = 0;
            double bad = 0.0;
            while (__hip_atomic_load(ts.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(ts.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                    ++spins > kTileSpinLimit) {
                    __hip_atomic_store(ts.err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bad = 1.0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            sa.misc[3] = bad;
        }
        // every tile's triple, combined in the same order by every workgroup
        double mv = -1.0, mk = 0.0, tot = 0.0;
        for (int i0 = 0; i0 < ts.G; i0 += 64) {
            const int i = i0 + lane;
            double v = -1.0, k = 0.0, s = 0.0;
            if (i < ts.G) {
                const double* sl = ts.slot(i, parity);
                v = load_agent(sl);
                k = load_agent(sl + 1);
                s = load_agent(sl + 2);
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double ov = __shfl_xor(v, o, 64);
                const double ok = __shfl_xor(k, o, 64);
                if (key_better(ov, ok, v, k)) {
                    v = ov;
                    k = ok;
                }
                s = s + __shfl_xor(s, o, 64);
            }
            if (key_better(v, k, mv, mk)) {
                mv = v;
                mk = k;
            }
            tot = tot + s;
        }
        if (lane < 6) {
            // lanes 0..2: the left neighbour's last three mu -> cells -3..-1;
            // lanes 3..5: the right neighbour's first three -> cells Tv..Tv+2
            const int nb = (lane < 3) ? (ts.tile + ts.G - 1) % ts.G : (ts.tile + 1) % ts.G;
            const double m = load_agent(ts.slot(nb, parity) + ((lane < 3) ? 6 + lane : lane));
            if (lane < 3) sa.MU[lane] = m;
            else sa.MU[3 + g.Tv + (lane - 3)] = m;
        }
        if (lane == 0) {
            if (pc.alpha_fixed > 0.0) {
                sa.misc[0] = pc.alpha_fixed;
                sa.misc[2] = 0.0;
            } else {
                sa.misc[0] = lf_alpha(mv, pc.fa, pc.fb);
                sa.misc[2] = (tot * pc.half_inv_dx) * 2.0 * fabs(pc.fa);  // d alpha / d u* = 2|fa| sign(u*)
            }
            sa.misc[1] = mk;
        }
    }
    __syncthreads();
    const double alpha = sa.misc[0], mk = sa.misc[1], csub = sa.misc[2];
    const bool ok = sa.misc[3] == 0.0;

    // phase 3: reverse of flux and reconstruction
    const double inv_dx = 2.0 * pc.half_inv_dx;
    double acc[CPT + 4];
#pragma unroll
    for (int i = 0; i < CPT + 4; ++i) acc[i] = 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int64_t j = g.x0 + g.j0 + q;
        const double km = 2.0 * (double)j;
        const double kp = 2.0 * (double)(j == 0 ? nx - 1 : j - 1) + 1.0;
        const double cm = (km == mk) ? csub : 0.0;
        const double cp = (kp == mk) ? csub : 0.0;
        const double muq = sa.MU[3 + g.j0 + q];
        const double grq = (sa.MU[4 + g.j0 + q] - muq) * inv_dx;
        const double glq = (muq - sa.MU[2 + g.j0 + q]) * inv_dx;
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
        __builtin_amdgcn_sched_barrier(0);
    }
    // the two cells beyond each edge: lanes 0..3 of wave 0 (cells -2, -1, Tv, Tv+1)
    double hc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (K != 0 && threadIdx.x < 4) {
        const int c = (threadIdx.x < 2) ? (int)threadIdx.x - 2 : g.Tv + ((int)threadIdx.x - 2);
        int64_t j = (g.x0 + c) % nx;
        if (j < 0) j += nx;
        const double km = 2.0 * (double)j;
        const double kp = 2.0 * (double)(j == 0 ? nx - 1 : j - 1) + 1.0;
        const double cm = (km == mk) ? csub : 0.0;
        const double cp = (kp == mk) ? csub : 0.0;
        const double muq = sa.MU[3 + c];
        const double grq = (sa.MU[4 + c] - muq) * inv_dx;
        const double glq = (muq - sa.MU[2 + c]) * inv_dx;
        auto adj = [&](double um_, double up_, double& umb, double& upb) {
            umb = fma(cm, sgn(um_), grq * fma(0.5, flux_fprime(um_, pc.fa, pc.fb), 0.5 * alpha));
            upb = fma(cp, sgn(up_), glq * fma(0.5, flux_fprime(up_, pc.fa, pc.fb), -0.5 * alpha));
        };
        weno5_cell_vjp_f(sa.V[4 + c - 2], sa.V[4 + c - 1], sa.V[4 + c], sa.V[4 + c + 1], sa.V[4 + c + 2], pc.eps,
                         adj, hc);
    }
    if (g.active) {
        if (CPT == 1) {
            if (g.j0 >= 1) sa.SP[0][g.j0 - 1] = acc[1];
            if (g.j0 >= 2) sa.SP[2][g.j0 - 2] = acc[0];
            if (g.j0 + 1 < g.Tv) sa.SP[1][g.j0 + 1] = acc[3];
            if (g.j0 + 2 < g.Tv) sa.SP[3][g.j0 + 2] = acc[4];
        } else {
            if (g.j0 >= 2) {
                sa.SP[0][g.j0 - 1] = acc[1];
                sa.SP[0][g.j0 - 2] = acc[0];
            }
            if (g.j0 + CPT + 1 < g.Tv) {
                sa.SP[1][g.j0 + CPT] = acc[CPT + 2];
                sa.SP[1][g.j0 + CPT + 1] = acc[CPT + 3];
            }
        }
    }
    if (K != 0 && threadIdx.x < 4) {
        // HC[0] = cell -2 -> 0, HC[1] = cell -1 -> 0, HC[2] = cell -1 -> 1,
        // HC[3] = cell Tv -> Tv-2, HC[4] = cell Tv -> Tv-1, HC[5] = cell Tv+1 -> Tv-1
        if (threadIdx.x == 0) sa.HC[0] = hc[4];
        if (threadIdx.x == 1) {
            sa.HC[1] = hc[3];
            sa.HC[2] = hc[4];
        }
        if (threadIdx.x == 2) {
            sa.HC[3] = hc[0];
            sa.HC[4] = hc[1];
        }
        if (threadIdx.x == 3) sa.HC[5] = hc[0];
    }
    __syncthreads();

    // phase 4: gather
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int c = g.j0 + q;
            double o = acc[q + 2];
            if (CPT == 1) {
                if (c + 1 < g.Tv) o += sa.SP[0][c];
                if (c >= 1) o += sa.SP[1][c];
                if (c + 2 < g.Tv) o += sa.SP[2][c];
                if (c >= 2) o += sa.SP[3][c];
            } else {
                if (q >= CPT - 2 && g.t != g.tlast) o += sa.SP[0][c];
                if (q <= 1 && g.t != 0) o += sa.SP[1][c];
            }
            if (K != 0) {
                if (c == 0) o += sa.HC[0] + sa.HC[1];
                if (c == 1) o += sa.HC[2];
                if (c == g.Tv - 2) o += sa.HC[3];
                if (c == g.Tv - 1) o += sa.HC[4] + sa.HC[5];
            }
            out[q] = o;
        }
    }
    return ok;
}

// lam <- (dPhi/du)^T lam over one step; the stage inputs are at base + s*nx
template <int CPT, int NW, int K, int ST>
__device__ __forceinline__ bool rev_step_t(double (&lam)[CPT], const double* base, double dt,
                                           const TGeo<CPT, NW>& g, const TASmem<CPT, NW>& sa, const PhiConst& pc,
                                           TSync& ts, int64_t nx)
{
    double t[CPT];
    if (ST == 1) {
        if (!op_AT_t<CPT, NW, K>(base, lam, t, g, sa, pc, ts, nx)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) lam[q] = fma(dt, t[q], lam[q]);
    } else if (ST == 2) {
        double l1[CPT];
        if (!op_AT_t<CPT, NW, K>(base + nx, lam, t, g, sa, pc, ts, nx)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) l1[q] = fma(0.5 * dt, t[q], 0.5 * lam[q]);
        if (!op_AT_t<CPT, NW, K>(base, l1, t, g, sa, pc, ts, nx)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) lam[q] = fma(dt, t[q], fma(0.5, lam[q], l1[q]));
    } else {
        double l1[CPT], l2[CPT];
        if (!op_AT_t<CPT, NW, K>(base + 2 * nx, lam, t, g, sa, pc, ts, nx)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            l2[q] = fma((2.0 / 3.0) * dt, t[q], (2.0 / 3.0) * lam[q]);
            lam[q] = (1.0 / 3.0) * lam[q];
        }
        if (!op_AT_t<CPT, NW, K>(base + nx, l2, t, g, sa, pc, ts, nx)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            l1[q] = fma(0.25 * dt, t[q], 0.25 * l2[q]);
            lam[q] = fma(0.75, l2[q], lam[q]);
        }
        if (!op_AT_t<CPT, NW, K>(base, l1, t, g, sa, pc, ts, nx)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) lam[q] = fma(dt, t[q], lam[q] + l1[q]);
    }
    return true;
}

template <int CPT, int NW>
__device__ __forceinline__ void tiled_sync_view(const AdjArgs& a, int G, int tile, int grp, TSync& ts)
{
    ts.err = a.tile_sync;
    ts.cnt = a.tile_sync + kTileCounterStride * (1 + grp);
    ts.ring = 2;
    ts.pub = a.tile_pub + (int64_t)grp * G * 2 * kTileSlot;
    ts.G = G;
    ts.tile = tile;
    ts.ep = 0;
}

// Reverse sweep over nsteps stored steps of line b (lines in groups of G tiles).
template <int CPT, int NW, int K, int ST>
__global__ __launch_bounds__(64 * NW) void tiled_adjoint_kernel(AdjArgs a)
{
    extern __shared__ double smem_raw[];
    TASmem<CPT, NW> sa;
    sa.init(smem_raw);
    const int G = a.tiles;
    const int tile = blockIdx.x % G;
    const int grp = blockIdx.x / G;
    TGeo<CPT, NW> g;
    g.init(a.nx, tile, G);
    TSync ts;
    tiled_sync_view<CPT, NW>(a, G, tile, grp, ts);
    const int64_t nx = a.nx;
    for (int64_t b = grp; b < a.nlines; b += a.groups) {
        double lam[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) lam[q] = g.active ? a.lam_in[b * nx + g.x0 + g.j0 + q] : 0.0;
        for (int n = a.nsteps - 1; n >= 0; --n) {
            const double* base = a.traj + b * a.traj_stride + (int64_t)n * ST * nx;
            if (!rev_step_t<CPT, NW, K, ST>(lam, base, a.dt, g, sa, a.pc, ts, nx)) return;
        }
        if (g.active) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) a.lam_out[b * nx + g.x0 + g.j0 + q] = lam[q];
        }
    }
}

// Forward steps of split lines storing every stage input: line b starts from
// u + b*u_stride*nx; step n's stage inputs go to traj_out + b*traj_stride + (n*ST + s)*nx.
template <int CPT, int NW, int K, int ST>
__global__ __launch_bounds__(64 * NW) void tiled_stage_store_kernel(AdjArgs a)
{
    extern __shared__ double smem_raw[];
    TSmem<CPT, NW> sm;
    sm.init(smem_raw);
    const int G = a.tiles;
    const int tile = blockIdx.x % G;
    const int grp = blockIdx.x / G;
    TGeo<CPT, NW> g;
    g.init(a.nx, tile, G);
    TSync ts;
    tiled_sync_view<CPT, NW>(a, G, tile, grp, ts);
    // the forward stages exchange through the sweeps' slot ring (op_A_t)
    ts.cnt = nullptr;
    ts.ring = kTileRing;
    ts.pub = a.tile_pub + (int64_t)grp * G * kTileRing * kTileSlot;
    const int64_t nx = a.nx;
    const PhiConst& pc = a.pc;
    for (int64_t b = grp; b < a.nlines; b += a.groups) {
        double x[CPT], gx;
        t_load(x, gx, a.u + b * a.u_stride * nx, g);
        for (int n = 0; n < a.nsteps; ++n) {
            double* base = a.traj_out + b * a.traj_stride + (int64_t)n * ST * nx;
            t_store(x, base, g);
            double A[CPT], gA;
            if (ST == 1) {
                if (!op_A_t<CPT, NW, K, false>(x, gx, A, gA, g, sm, pc, ts)) return;
#pragma unroll
                for (int q = 0; q < CPT; ++q) x[q] = rk_first(x[q], A[q], a.dt);
                gx = rk_first(gx, gA, a.dt);
            } else if (ST == 2) {
                double v[CPT], gv;
                if (!op_A_t<CPT, NW, K, false>(x, gx, A, gA, g, sm, pc, ts)) return;
#pragma unroll
                for (int q = 0; q < CPT; ++q) v[q] = rk_first(x[q], A[q], a.dt);
                gv = rk_first(gx, gA, a.dt);
                t_store(v, base + nx, g);
                if (!op_A_t<CPT, NW, K, false>(v, gv, A, gA, g, sm, pc, ts)) return;
#pragma unroll
                for (int q = 0; q < CPT; ++q) x[q] = rk2_second(x[q], v[q], A[q], 0.5 * a.dt);
                gx = rk2_second(gx, gv, gA, 0.5 * a.dt);
            } else {
                double v[CPT], gv;
                if (!op_A_t<CPT, NW, K, false>(x, gx, A, gA, g, sm, pc, ts)) return;
#pragma unroll
                for (int q = 0; q < CPT; ++q) v[q] = rk_first(x[q], A[q], a.dt);
                gv = rk_first(gx, gA, a.dt);
                t_store(v, base + nx, g);
                if (!op_A_t<CPT, NW, K, false>(v, gv, A, gA, g, sm, pc, ts)) return;
#pragma unroll
                for (int q = 0; q < CPT; ++q) v[q] = rk3_second(x[q], v[q], A[q], 0.25 * a.dt);
                gv = rk3_second(gx, gv, gA, 0.25 * a.dt);
                t_store(v, base + 2 * nx, g);
                if (!op_A_t<CPT, NW, K, false>(v, gv, A, gA, g, sm, pc, ts)) return;
#pragma unroll
                for (int q = 0; q < CPT; ++q) x[q] = rk3_third(x[q], v[q], A[q], (2.0 / 3.0) * a.dt);
                gx = rk3_third(gx, gv, gA, (2.0 / 3.0) * a.dt);
            }
        }
    }
}

template <class Fn>
static hipError_t launch_coop_adj(Fn fn, const AdjArgs& a, int nw, size_t shmem, bool forward, hipStream_t s)
{
    hipError_t e;
    if (shmem > 65536) {
        e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        if (e != hipSuccess) return e;
    }
    int dev = 0, ncu = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, 64 * nw, shmem)) != hipSuccess)
        return e;
    const long long cap = std::min((long long)per_cu * ncu, (long long)kTileMaxWorkgroups);
    const int G = a.tiles;
    if (G < 1 || cap < G) return hipErrorCooperativeLaunchTooLarge;
    AdjArgs b = a;
    b.groups = (int)std::min((long long)a.nlines, cap / G);
    e = launch_clear_ints((int*)b.tile_sync, 2 * kTileCounterStride * (b.groups + 1), s);
    if (e != hipSuccess) return e;
    if (forward) {
        // forward stages: every slot of the launch's groups starts empty
        e = launch_fill_u64((unsigned long long*)b.tile_pub, kSlotEmpty, (int64_t)b.groups * G * kTileRing * kTileSlot,
                            s);
        if (e != hipSuccess) return e;
    }
    void* args[] = {(void*)&b};
    return hipLaunchCooperativeKernel((const void*)fn, dim3((unsigned)(b.groups * G)), dim3(64 * nw), args,
                                      (unsigned)shmem, s);
}

// Tiles must be whole threads (for CPT > 1: nx % tiles == 0 and
// (nx / tiles) % CPT == 0) and hold at least 6 cells.
template <int K, int ST>
hipError_t launch_tiled_adjoint_ks(const AdjArgs& a, const KernelCfg& cfg, int store_mode, hipStream_t s)
{
#define MGK_TADJ_CASE(C, W)                                                                                   \
    if (cfg.cpt == C && cfg.nw == W) {                                                                        \
        const int64_t nx = a.nx, G = a.tiles;                                                                 \
        if (G < 1 || (C > 1 && (nx % G != 0 || (nx / G) % C != 0)) || nx / G < 6 ||                         \
            (nx + G - 1) / G > 64 * W * C)                                                                    \
            return hipErrorInvalidValue;                                                                      \
        if (store_mode)                                                                                       \
            return launch_coop_adj(tiled_stage_store_kernel<C, W, K, ST>, a, W, tiled_smem_bytes(C, W), true, s); \
        return launch_coop_adj(tiled_adjoint_kernel<C, W, K, ST>, a, W, tiled_adj_smem_bytes<C, W>(), false, s); \
    }
    MGK_TADJ_CFG_LIST(MGK_TADJ_CASE)
#undef MGK_TADJ_CASE
    return hipErrorInvalidValue;
}

}  // namespace mgk
