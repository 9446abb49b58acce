// sys_tiled_impl.h -- system sweeps (shallow water, Euler) on lines longer
// than one workgroup holds (included by the sys_tiled_s*_k*.hip translation
// units).
//
// A line of n cells is split into G tiles of balanced length; tile g is owned
// by one workgroup with one cell per thread, and two threads past the tile's
// last cell are kept free (the launcher sizes the workgroup so).  Each tile
// also keeps NG = K + 1 ghost cells on each side (tile_ghosts), owned by the
// first 2 NG threads.  Per Runge-Kutta stage a tile:
//   1. mirrors its cells and ghosts into LDS (one plane per component),
//      barrier;
//   2. reconstructs characteristic-wise (sec 2.1.1) in each of its cells, and
//      with the two free threads in the edge ghosts -1 (its u^- is the left
//      state of the tile's left edge face) and Tv (its u^+ the right state of
//      the right edge face); the tile's largest wave speed (eq eigs), barrier;
//   3. splits twice the LF flux of both faces of each cell (eq LFflux) into
//          2F = Fa - alpha_LF Fb,  Fa = f(u^-) + f(u^+),  Fb = u^+ - u^-
//      (Roe, eq roeflux: Fa is twice the flux, Fb = 0), and publishes the
//      tile maximum and the (Fa, Fb) of the right faces of its first NG cells
//      and of the left faces of its last NG cells;
//   4. polls every tile's maximum of the stage (alpha_LF) and its
//      neighbours' edge data, barrier;
//   5. updates its cells and ghosts.  A ghost's faces come from its owner's
//      published parts (or the tile's own edge faces), combined with
//      alpha_LF exactly as the owner combines them, so ghosts stay bitwise
//      equal to the owners' cells, and the split line bitwise equal to one
//      workgroup per line.
// The exchange is the one of tiled_impl.h: every published value is its own
// arrival flag (slots start as kSlotEmpty), a ring of kTileRing slots per
// tile, device-coherent 64-bit accesses, bounded spins, cooperative
// persistent launches with line groups taking chunks round-robin.
#pragma once
#include <climits>

#include "sys_impl.h"
#include "tiled_impl.h"

namespace mgk {

// LDS misc area of a system tile
constexpr int kSysMisc = 64;
constexpr int kSysMiscErr = kSysMisc - 1;

// geometry of tile `tile` of G over a line of n cells
template <int NG>
struct STGeo {
    int n, x0, Tv;  // cells of the line; the tile's first cell and length
    int t, npad, P; // thread, threads, LDS plane length npad + 2 NG + 1
    int gk;         // ghost of the thread: 0..NG-1 cells -NG..-1, NG..2NG-1 cells Tv..Tv+NG-1; else -1
    int gcell;      // line cell of that ghost
    int gpos;       // its LDS position
    int rc;         // tile cell the thread reconstructs: its own, Tv, -1, or INT_MIN
    // LDS position of tile cell c, -NG <= c < Tv + NG (ghosts after the npad
    // cell positions; anything else at the spare position P - 1)
    __device__ __forceinline__ int pos(int c) const
    {
        if (c < 0) return npad + NG + c;
        if (c < Tv) return c;
        if (c < Tv + NG) return npad + NG + (c - Tv);
        return P - 1;
    }
    __device__ __forceinline__ void init(int ncell, int tile, int G)
    {
        n = ncell;
        x0 = (int)((int64_t)tile * n / G);
        Tv = (int)((int64_t)(tile + 1) * n / G) - x0;
        t = threadIdx.x;
        npad = blockDim.x;
        P = npad + 2 * NG + 1;
        gk = (t < 2 * NG) ? t : -1;
        gcell = 0;
        gpos = P - 1;
        if (gk >= 0) {
            const int c = (gk < NG) ? gk - NG : Tv + (gk - NG);
            int cell = (x0 + c) % n;
            if (cell < 0) cell += n;
            gcell = cell;
            gpos = pos(c);
        }
        rc = (t < Tv) ? t : (t == Tv) ? Tv : (t == Tv + 1) ? -1 : INT_MIN;
    }
};

// LDS: line[D P] | bm[D P] | bp[D P] | amax[kSysMaxWaves] | misc[kSysMisc]
//   misc[0] alpha_LF; [1, 1 + E) the left neighbour's left-face data of its
//   last NG cells; [1 + E, 1 + 2E) the right neighbour's right-face data of
//   its first NG cells (E = 2 NG D: per cell NG.. D values of Fa, then D of
//   Fb); [1 + 2E, 1 + 2E + 2D) (Fa, Fb) of the tile's left edge face;
//   [1 + 2E + 2D, 1 + 2E + 4D) of its right edge face; [kSysMiscErr] error
template <int D>
struct STSmem {
    double *line, *bm, *bp, *amax, *misc;
    __device__ __forceinline__ void init(double* base, int P)
    {
        line = base;
        bm = line + D * P;
        bp = bm + D * P;
        amax = bp + D * P;
        misc = amax + kSysMaxWaves;
    }
};

inline size_t sys_tiled_smem_bytes(int D, int K, int threads)
{
    const int NG = (K == 3) ? 4 : 3;
    return sizeof(double) * ((size_t)3 * D * (threads + 2 * NG + 1) + kSysMaxWaves + kSysMisc);
}

// the group's slots: tile tl, ring position r at pub + (tl kTileRing + r) kSysTileSlot
//   [0] tile max wave speed; [1, 1 + E) (Fa, Fb) of the right faces of the
//   tile's first NG cells; [1 + E, 1 + 2E) of the left faces of its last NG
struct SSync {
    unsigned long long* err;
    double* pub;
    int G, tile;
    long long ep;  // stages done by this workgroup
    __device__ __forceinline__ double* slot(int tl, int r) const
    {
        return pub + ((int64_t)tl * kTileRing + r) * kSysTileSlot;
    }
};

// A(V) of the tile's cells and A(gv) of the thread's ghost (eq spaceDisc);
// false when the line's synchronisation failed
template <int SYS, int K, bool ROE>
__device__ __forceinline__ bool op_A_st(const double (&V)[Phys<SYS>::D], const double (&gv)[Phys<SYS>::D],
                                        double (&A)[Phys<SYS>::D], double (&gA)[Phys<SYS>::D],
                                        const STGeo<tile_ghosts<K>()>& g, const STSmem<Phys<SYS>::D>& sm,
                                        const PhiConst& pc, SSync& ts)
{
    constexpr int D = Phys<SYS>::D;
    constexpr int NG = tile_ghosts<K>();
    constexpr int E = 2 * NG * D;
    constexpr int OWNL = 1 + 2 * E, OWNR = OWNL + 2 * D;
    static_assert(1 + 2 * E <= kSysTileSlot, "slot too short");
    static_assert(OWNR + 2 * D <= kSysMiscErr, "misc too short");
    const double pp = pc.fb;
    const int P = g.P;
    const bool own = g.t < g.Tv;

    // 1. mirror
    if (own) {
#pragma unroll
        for (int d = 0; d < D; ++d) sm.line[d * P + g.t] = V[d];
    }
    if (g.gk >= 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) sm.line[d * P + g.gpos] = gv[d];
    }
    __syncthreads();

    // 2. reconstruct (as op_A_sys, the window read through pos)
    double um[D], up[D];
    if (g.rc != INT_MIN) {
        double Vc[D];
#pragma unroll
        for (int d = 0; d < D; ++d) Vc[d] = own ? V[d] : sm.line[d * P + g.pos(g.rc)];
#pragma unroll
        for (int d = 0; d < D; ++d) um[d] = up[d] = Vc[d];
        if constexpr (K > 0) {
            double lam[D], R[D][D], L[D][D];
            Phys<SYS>::eig_state(Vc, pp, lam, R, L);
            double w[2 * K + 1][D];
#pragma unroll
            for (int j = 0; j <= 2 * K; ++j) {
                const int p = g.pos(g.rc - K + j);
#pragma unroll
                for (int d = 0; d < D; ++d) w[j][d] = (j == K) ? Vc[d] : sm.line[d * P + p];
            }
            double wmq[D], wpq[D];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                double cw[2 * K + 1];
#pragma unroll
                for (int j = 0; j <= 2 * K; ++j) {
                    double acc = L[q][0] * w[j][0];
#pragma unroll
                    for (int d = 1; d < D; ++d) acc = fma(L[q][d], w[j][d], acc);
                    cw[j] = acc;
                }
                char_weno<K>(cw, pc.eps, wmq[q], wpq[q]);
            }
#pragma unroll
            for (int d = 0; d < D; ++d) {
                double am = R[d][0] * wmq[0], ap = R[d][0] * wpq[0];
#pragma unroll
                for (int q = 1; q < D; ++q) {
                    am = fma(R[d][q], wmq[q], am);
                    ap = fma(R[d][q], wpq[q], ap);
                }
                um[d] = am;
                up[d] = ap;
            }
        }
        const int p = g.pos(g.rc);
        if (own || g.rc == -1) {
#pragma unroll
            for (int d = 0; d < D; ++d) sm.bm[d * P + p] = um[d];
        }
        if (own || g.rc == g.Tv) {
#pragma unroll
            for (int d = 0; d < D; ++d) sm.bp[d * P + p] = up[d];
        }
    }
    if constexpr (!ROE) {
        double lmax = own ? fmax(Phys<SYS>::max_speed(um, pp), Phys<SYS>::max_speed(up, pp)) : 0.0;
        lmax = wave_max(lmax);
        if ((threadIdx.x & 63) == 0) sm.amax[threadIdx.x >> 6] = lmax;
    }
    __syncthreads();

    // 3. flux parts of the cell's faces, published by the edge cells' owners
    double Fal[D], Fbl[D], Far[D], Fbr[D];
#pragma unroll
    for (int d = 0; d < D; ++d) Fal[d] = Fbl[d] = Far[d] = Fbr[d] = 0.0;
    if (own) {
        double lm[D], rp[D];
        const int pl = g.pos(g.t - 1), pr = g.pos(g.t + 1);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lm[d] = sm.bm[d * P + pl];  // u^-_{i-1/2}
            rp[d] = sm.bp[d * P + pr];  // u^+_{i+1/2}
        }
        if constexpr (ROE) {
            sys_flux2<SYS, true>(lm, up, pp, 0.0, Fal);
            sys_flux2<SYS, true>(um, rp, pp, 0.0, Far);
        } else {
            // the operands and order of sys_flux2's LF branch
            double f1[D], f2[D];
            Phys<SYS>::flux(lm, pp, f1);
            Phys<SYS>::flux(up, pp, f2);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                Fal[d] = f1[d] + f2[d];
                Fbl[d] = up[d] - lm[d];
            }
            Phys<SYS>::flux(um, pp, f1);
            Phys<SYS>::flux(rp, pp, f2);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                Far[d] = f1[d] + f2[d];
                Fbr[d] = rp[d] - um[d];
            }
        }
    }
    const int r = (int)(ts.ep % kTileRing);
    ts.ep += 1;
    double* mine = ts.slot(ts.tile, r);
    const bool pubR = g.t < NG;  // (every tile holds at least NG cells)
    const bool pubL = own && g.t >= g.Tv - NG;
    // each writer's emptying stores of the previous stage complete first
    if (g.t == 0 || pubR || pubL) __builtin_amdgcn_s_waitcnt(0);
    if (g.t == 0) {
        double v = 0.0;
        if constexpr (!ROE) {
            v = sm.amax[0];
            for (int w2 = 1; w2 < (g.npad >> 6); ++w2) v = fmax(v, sm.amax[w2]);
        }
        store_agent(mine, v);
    }
    if (pubR) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            store_agent(mine + 1 + g.t * 2 * D + d, Far[d]);
            store_agent(mine + 1 + g.t * 2 * D + D + d, Fbr[d]);
        }
    }
    if (pubL) {
        const int j = g.t - (g.Tv - NG);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            store_agent(mine + 1 + E + j * 2 * D + d, Fal[d]);
            store_agent(mine + 1 + E + j * 2 * D + D + d, Fbl[d]);
        }
    }
    if (g.t == 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            sm.misc[OWNL + d] = Fal[d];
            sm.misc[OWNL + D + d] = Fbl[d];
        }
    }
    if (g.t == g.Tv - 1) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            sm.misc[OWNR + d] = Far[d];
            sm.misc[OWNR + D + d] = Fbr[d];
        }
    }

    // 4. wave 0 polls the G maxima and the neighbours' 2 E edge values
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int G = ts.G;
        const int nbl = (ts.tile + G - 1) % G, nbr = (ts.tile + 1) % G;
        double mx = 0.0;
        int bad = 0;
        for (int it = lane; it < G + 2 * E; it += 64) {
            const double* src;
            int dst = -1;
            if (it < G) {
                src = ts.slot(it, r);
            } else {
                const int e = it - G;
                src = (e < E) ? ts.slot(nbl, r) + 1 + E + e : ts.slot(nbr, r) + 1 + (e - E);
                dst = 1 + e;
            }
            unsigned long long bits = load_bits(src);
            long long spins = 0;
            while (bits == kSlotEmpty) {
                if (__hip_atomic_load(ts.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                    ++spins > kTileSpinLimit) {
                    __hip_atomic_store(ts.err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bad = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                bits = load_bits(src);
            }
            const double v = __longlong_as_double((long long)bits);
            if (dst < 0) mx = fmax(mx, v);
            else sm.misc[dst] = bad ? 0.0 : v;
        }
        mx = wave_max(mx);
        const bool any_bad = __ballot(bad) != 0;
        if (lane == 0) {
            sm.misc[0] = ROE ? 0.0 : (pc.alpha_fixed > 0.0) ? pc.alpha_fixed : mx;
            sm.misc[kSysMiscErr] = any_bad ? 1.0 : 0.0;
        }
    }
    __syncthreads();

    // every tile has published this stage, so every reader is done with the
    // previous one: its writers empty that slot
    {
        double* old = ts.slot(ts.tile, (r + kTileRing - 1) % kTileRing);
        if (g.t == 0) store_empty(old);
        if (pubR) {
#pragma unroll
            for (int i = 0; i < 2 * D; ++i) store_empty(old + 1 + g.t * 2 * D + i);
        }
        if (pubL) {
            const int j = g.t - (g.Tv - NG);
#pragma unroll
            for (int i = 0; i < 2 * D; ++i) store_empty(old + 1 + E + j * 2 * D + i);
        }
    }

    // 5. A of the cell (as op_A_sys: (F_{i-1/2} - F_{i+1/2}) / (2 dx)) and of the ghost
    const double alpha = sm.misc[0];
    const bool ok = sm.misc[kSysMiscErr] == 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double fl = ROE ? Fal[d] : fma(-alpha, Fbl[d], Fal[d]);
        const double fr = ROE ? Far[d] : fma(-alpha, Fbr[d], Far[d]);
        A[d] = own ? (fl - fr) * pc.half_inv_dx : 0.0;
    }
    if (g.gk >= 0) {
        // positions in misc of the (Fa, Fb) of the ghost's left and right faces
        int il, ir;
        if (g.gk < NG) {  // cell gk - NG: faces are the left neighbour's left faces of cells gk, gk + 1
            il = 1 + g.gk * 2 * D;
            ir = (g.gk < NG - 1) ? 1 + (g.gk + 1) * 2 * D : OWNL;
        } else {  // cell Tv + r2: the right faces of the right neighbour's cells r2 - 1, r2
            const int r2 = g.gk - NG;
            il = (r2 == 0) ? OWNR : 1 + E + (r2 - 1) * 2 * D;
            ir = 1 + E + r2 * 2 * D;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double fl = ROE ? sm.misc[il + d] : fma(-alpha, sm.misc[il + D + d], sm.misc[il + d]);
            const double fr = ROE ? sm.misc[ir + d] : fma(-alpha, sm.misc[ir + D + d], sm.misc[ir + d]);
            gA[d] = (fl - fr) * pc.half_inv_dx;
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) gA[d] = 0.0;
    }
    return ok;
}

// x <- Phi(x), the ghost gx alongside (eq SSPRK1/2/3, the operations of phi_sys)
template <int SYS, int K, int ST, bool ROE>
__device__ __forceinline__ bool phi_st(double (&x)[Phys<SYS>::D], double (&gx)[Phys<SYS>::D], double dt,
                                       const STGeo<tile_ghosts<K>()>& g, const STSmem<Phys<SYS>::D>& sm,
                                       const PhiConst& pc, SSync& ts)
{
    constexpr int D = Phys<SYS>::D;
    double A[D], gA[D], v[D], gv[D];
    if (!op_A_st<SYS, K, ROE>(x, gx, A, gA, g, sm, pc, ts)) return false;
    if constexpr (ST == 1) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            x[d] = rk_first(x[d], A[d], dt);
            gx[d] = rk_first(gx[d], gA[d], dt);
        }
    } else if constexpr (ST == 2) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            v[d] = rk_first(x[d], A[d], dt);
            gv[d] = rk_first(gx[d], gA[d], dt);
        }
        if (!op_A_st<SYS, K, ROE>(v, gv, A, gA, g, sm, pc, ts)) return false;
        const double hdt = 0.5 * dt;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            x[d] = rk2_second(x[d], v[d], A[d], hdt);
            gx[d] = rk2_second(gx[d], gv[d], gA[d], hdt);
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            v[d] = rk_first(x[d], A[d], dt);
            gv[d] = rk_first(gx[d], gA[d], dt);
        }
        if (!op_A_st<SYS, K, ROE>(v, gv, A, gA, g, sm, pc, ts)) return false;
        const double qdt = 0.25 * dt;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            v[d] = rk3_second(x[d], v[d], A[d], qdt);
            gv[d] = rk3_second(gx[d], gv[d], gA[d], qdt);
        }
        if (!op_A_st<SYS, K, ROE>(v, gv, A, gA, g, sm, pc, ts)) return false;
        const double tdt = (2.0 / 3.0) * dt;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            x[d] = rk3_third(x[d], v[d], A[d], tdt);
            gx[d] = rk3_third(gx[d], gv[d], gA[d], tdt);
        }
    }
    return true;
}

// transfers of the tile's cells of a line (component d of cell i at d n + i),
// the thread's ghost alongside where it reads
template <int D, int NG>
__device__ __forceinline__ void st_load(double (&x)[D], double (&gx)[D], const double* src, const STGeo<NG>& g)
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        x[d] = (g.t < g.Tv) ? src[(int64_t)d * g.n + g.x0 + g.t] : 0.0;
        gx[d] = (g.gk >= 0) ? src[(int64_t)d * g.n + g.gcell] : 0.0;
    }
}

template <int D, int NG>
__device__ __forceinline__ void st_store(const double (&x)[D], double* dst, const STGeo<NG>& g)
{
    if (g.t < g.Tv) {
#pragma unroll
        for (int d = 0; d < D; ++d) dst[(int64_t)d * g.n + g.x0 + g.t] = x[d];
    }
}

template <int D, int NG>
__device__ __forceinline__ void st_add(double (&x)[D], double (&gx)[D], const double* src, const STGeo<NG>& g)
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (g.t < g.Tv) x[d] = x[d] + src[(int64_t)d * g.n + g.x0 + g.t];
        if (g.gk >= 0) gx[d] = gx[d] + src[(int64_t)d * g.n + g.gcell];
    }
}

template <int D, int NG>
__device__ __forceinline__ void st_copy(const double* src, double* dst, const STGeo<NG>& g)
{
    if (g.t < g.Tv) {
#pragma unroll
        for (int d = 0; d < D; ++d) dst[(int64_t)d * g.n + g.x0 + g.t] = src[(int64_t)d * g.n + g.x0 + g.t];
    }
}

// sum over the tile of (x - b)^2 in a fixed order; valid in thread 0
template <int D, int NG>
__device__ __forceinline__ double st_sqdiff(const double (&x)[D], const double* b, const STGeo<NG>& g,
                                            const STSmem<D>& sm)
{
    double s = 0.0;
    if (g.t < g.Tv) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double e = x[d] - b[(int64_t)d * g.n + g.x0 + g.t];
            s = fma(e, e, s);
        }
    }
    s = wave_sum(s);
    // amax is free here: the next stage writes it only after its first barrier
    if ((threadIdx.x & 63) == 0) sm.amax[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (g.npad >> 6); ++w) tot += sm.amax[w];
    }
    return tot;
}

// One chunk on one tile: the roles of sys_body (without a scheme per level)
template <int SYS, int K, int ST, bool ROE, int END>
__device__ __forceinline__ bool st_chunk(const SweepArgs& a, int c, const STGeo<tile_ghosts<K>()>& g,
                                         const STSmem<Phys<SYS>::D>& sm, SSync& ts)
{
    constexpr int D = Phys<SYS>::D;
    const int64_t nx = a.nx;
    const double* src = (a.side_in != nullptr && c > 0) ? a.side_in + (int64_t)c * nx
                                                        : a.ustart + (int64_t)c * a.ustart_stride * nx;
    double x[D], gx[D];
    st_load(x, gx, src, g);
    if (a.ucommit != nullptr) st_store(x, a.ucommit + (int64_t)c * a.ucommit_stride * nx, g);
    if (a.inject_last && c == a.nchunks - 1) {
        const double* last = (a.side_in != nullptr) ? a.side_in + (int64_t)a.nchunks * nx
                                                    : a.ustart + (int64_t)a.nchunks * a.ustart_stride * nx;
        st_copy<D>(last, a.ucommit + (int64_t)a.nchunks * a.ucommit_stride * nx, g);
    }
    const double* cstart = (a.ystart != nullptr) ? a.ystart + (int64_t)c * a.ystart_stride * nx : src;
    if (END == END_RESTRICT && c == 0) {
        st_copy<D>(cstart, a.uc_out, g);
        st_copy<D>(a.g != nullptr ? a.g : cstart, a.gc_out, g);
    }

    const int64_t n0 = (int64_t)c * a.m;
    for (int j = 1; j <= a.nsteps; ++j) {
        if (!phi_st<SYS, K, ST, ROE>(x, gx, a.dt, g, sm, a.pc, ts)) return false;
        if (a.g != nullptr) st_add(x, gx, a.g + (n0 + j) * nx, g);
        if (a.fout != nullptr) {
            if (a.fout_every <= 1) st_store(x, a.fout + (n0 + j) * nx, g);
            else if ((n0 + j) % a.fout_every == 0) st_store(x, a.fout + ((n0 + j) / a.fout_every) * nx, g);
        }
    }

    if constexpr (END == END_NONE) return true;
    if constexpr (END == END_PHI) {
        if (!phi_st<SYS, K, ST, ROE>(x, gx, a.dt, g, sm, a.pc, ts)) return false;
        st_store(x, a.side_out + (int64_t)c * nx, g);
        return true;
    }
    const int64_t n1 = n0 + a.m;
    if (!phi_st<SYS, K, ST, ROE>(x, gx, a.dt, g, sm, a.pc, ts)) return false;
    if (a.g != nullptr) st_add(x, gx, a.g + n1 * nx, g);
    const double* cnext = a.cref + (int64_t)(c + 1) * a.cref_stride * nx;
    if (a.resid_partial != nullptr) {
        const double s = st_sqdiff(x, cnext, g, sm);
        if (threadIdx.x == 0) a.resid_partial[(int64_t)c * ts.G + ts.tile] = s;
    }
    if (a.r_out != nullptr && g.t < g.Tv) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int64_t i = (int64_t)d * g.n + g.x0 + g.t;
            a.r_out[(int64_t)c * nx + i] = x[d] - cnext[i];
        }
    }
    if constexpr (END == END_CSTEP) {
        if (a.side_out != nullptr) st_store(x, a.side_out + (int64_t)(c + 1) * nx, g);
        return true;
    }
    if (a.coarse_injection) st_copy<D>(cnext, a.uc_out + (int64_t)(c + 1) * nx, g);
    else st_store(x, a.uc_out + (int64_t)(c + 1) * nx, g);
    double y[D], gy[D];
    st_load(y, gy, cstart, g);
    PhiConst pcn = a.pc;
    if (a.alpha_next > 0.0) pcn.alpha_fixed = a.alpha_next;
    if (!phi_st<SYS, K, ST, ROE>(y, gy, a.dt_next, g, sm, pcn, ts)) return false;
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = x[d] - y[d];
    st_store(y, a.gc_out + (int64_t)(c + 1) * nx, g);
    return true;
}

// workgroup b: tile b % G of line group b / G, which takes chunks grp, grp + groups, ...
template <int SYS, int K, int ST, bool ROE, int END>
__device__ __forceinline__ void st_body(const SweepArgs& a)
{
    constexpr int D = Phys<SYS>::D;
    if (a.flag != nullptr && *a.flag != 0) return;
    extern __shared__ double smem_raw[];
    const int G = a.tiles;
    const int tile = blockIdx.x % G;
    const int grp = blockIdx.x / G;
    STGeo<tile_ghosts<K>()> g;
    g.init(a.nx / D, tile, G);
    STSmem<D> sm;
    sm.init(smem_raw, g.P);
    SSync ts;
    ts.err = a.tile_sync;
    ts.pub = a.tile_pub + (int64_t)grp * G * kTileRing * kSysTileSlot;
    ts.G = G;
    ts.tile = tile;
    ts.ep = 0;
    for (int c = grp; c < a.nchunks; c += a.groups)
        if (!st_chunk<SYS, K, ST, ROE, END>(a, c, g, sm, ts)) return;
}

template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_tiled_f_kernel(SweepArgs a)
{
    st_body<SYS, K, ST, ROE, END_NONE>(a);
}
template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_tiled_fc_kernel(SweepArgs a)
{
    st_body<SYS, K, ST, ROE, END_CSTEP>(a);
}
template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_tiled_fr_kernel(SweepArgs a)
{
    st_body<SYS, K, ST, ROE, END_RESTRICT>(a);
}
template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_tiled_phi_kernel(SweepArgs a)
{
    st_body<SYS, K, ST, ROE, END_PHI>(a);
}

template <int SYS, int K, int ST, bool ROE>
static hipError_t launch_sys_tiled_f(const SweepArgs& a, int threads, hipStream_t s)
{
    const size_t shmem = sys_tiled_smem_bytes(Phys<SYS>::D, K, threads);
    auto go = [&](auto fn) -> hipError_t {
        hipError_t e;
        if (shmem > 65536) {
            e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
            if (e != hipSuccess) return e;
        }
        int dev = 0, ncu = 0, per_cu = 0;
        if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
        if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, threads, shmem)) != hipSuccess)
            return e;
        // resident workgroups, within what the synchronisation scratch holds
        const long long slots = (long long)(tile_scratch_bytes() - tile_sync_bytes()) /
                                ((long long)sizeof(double) * kTileRing * kSysTileSlot);
        const long long cap = std::min((long long)per_cu * ncu, slots);
        const int G = a.tiles;
        if (G < 1 || cap < G) return hipErrorCooperativeLaunchTooLarge;
        SweepArgs b = a;
        b.groups = (int)std::min((long long)a.nchunks, cap / G);
        e = launch_clear_ints((int*)b.tile_sync, 2, s);
        if (e != hipSuccess) return e;
        e = launch_fill_u64((unsigned long long*)b.tile_pub, kSlotEmpty,
                            (int64_t)b.groups * G * kTileRing * kSysTileSlot, s);
        if (e != hipSuccess) return e;
        void* args[] = {(void*)&b};
        return hipLaunchCooperativeKernel((const void*)fn, dim3((unsigned)(b.groups * G)), dim3(threads), args,
                                          (unsigned)shmem, s);
    };
    switch (a.end_mode) {
    case END_NONE: return go(sys_tiled_f_kernel<SYS, K, ST, ROE>);
    case END_CSTEP: return go(sys_tiled_fc_kernel<SYS, K, ST, ROE>);
    case END_RESTRICT: return go(sys_tiled_fr_kernel<SYS, K, ST, ROE>);
    case END_PHI: return go(sys_tiled_phi_kernel<SYS, K, ST, ROE>);
    default: return hipErrorInvalidValue;
    }
}

// threads: a multiple of 64, at most 512, at least the longest tile + 2; every
// tile at least tile_ghosts<K>() cells (the launcher's caller checks both)
template <int SYS, int K>
hipError_t launch_sys_tiled_sk(const SweepArgs& a, int threads, int stepper, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
    const int n = a.nx / Phys<SYS>::D;
    const int G = a.tiles;
    if (threads < 64 || threads > 512 || threads % 64 != 0 || G < 1 || (n + G - 1) / G + 2 > threads ||
        n / G < tile_ghosts<K>() || a.coarse_split || a.gc_sub != nullptr)
        return hipErrorInvalidValue;
    const bool roe = a.pc.roe != 0;
    if (stepper == 1)
        return roe ? launch_sys_tiled_f<SYS, K, 1, true>(a, threads, s) : launch_sys_tiled_f<SYS, K, 1, false>(a, threads, s);
    if (stepper == 2)
        return roe ? launch_sys_tiled_f<SYS, K, 2, true>(a, threads, s) : launch_sys_tiled_f<SYS, K, 2, false>(a, threads, s);
    return roe ? launch_sys_tiled_f<SYS, K, 3, true>(a, threads, s) : launch_sys_tiled_f<SYS, K, 3, false>(a, threads, s);
}

}  // namespace mgk
