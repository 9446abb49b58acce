// tiled_impl.h -- sweep kernels for lines longer than one workgroup holds
// (included by the tiled_k*_s*.hip translation units).
//
// A line of nx cells is split into G tiles of T = 64*NW*CPT cells (the last
// tile may be shorter, always a multiple of CPT).  Tile g is owned by one
// workgroup, which keeps its cells in registers and, per Runge-Kutta stage:
//   1. mirrors its cells and six ghost cells (three on each side, owned by the
//      neighbouring tiles) into LDS, barrier;
//   2. reconstructs u^-/u^+ of its cells (sec 2.1.1) plus one extra
//      reconstruction in each edge ghost cell, so that it can form every
//      interface flux of its cells itself;
//   3. splits twice the LF flux of each interface (eq LFflux) into the parts
//      before and after the global coefficient is known,
//          2F = Fa - alpha_LF Fb,  Fa = f(u^-) + f(u^+),  Fb = u^+ - u^-
//      (with the Roe flux, eq roeflux, Fa is twice the flux and Fb = 0),
//      and publishes its local max |u^{+-}| and (Fa, Fb) of the three
//      interfaces inside each edge to a global slot;
//   4. meets the other tiles of the line at a global counter (one arrival per
//      tile, bounded spin), reads alpha_LF = max over all tiles (eq eigs) and
//      its neighbours' edge data;
//   5. updates its cells and, with the neighbours' data, its six ghost cells,
//      evaluating exactly the operations the owners evaluate on the same
//      operands, so ghosts stay bitwise equal to the owners' cells.
// One global synchronisation per stage; everything else stays on chip.
//
// All workgroups of a line must be resident at once: the launch is
// cooperative and persistent, groups of G workgroups take lines (chunks)
// round-robin, and every spin has a bound after which the kernel records an
// error and every workgroup leaves.
#pragma once
#include <algorithm>

#include "sweep_impl.h"

namespace mgk {

constexpr long long kTileSpinLimit = 1LL << 22;

// LDS: tl[T + 7] | bm[64 NW] | bp[64 NW] | amax[NW] | misc[40]
//   tl: the tile's cells transposed (cell c at (c mod CPT) * threads + c / CPT,
//   so that every window position is read lane-contiguously, free of bank
//   conflicts), ghost cells -3..-1 at T..T+2 and Tv..Tv+2 at T+3..T+5, one
//   scratch slot at T+6 for window positions past the ghosts
//   misc[0] alpha_LF, [1..2] (Fa, Fb) of the tile's left edge interface,
//   [3..4] of its right edge interface, [5..10] the left neighbour's
//   right-edge data, [11..16] the right neighbour's left-edge data,
//   [17..28] this tile's edge data staged for publication, [39] error flag
template <int CPT, int NW>
struct TSmem {
    double* tl;
    double* bm;
    double* bp;
    double* amax;
    double* misc;
    __device__ __forceinline__ void init(double* base)
    {
        tl = base;
        bm = tl + 64 * NW * CPT + 7;
        bp = bm + 64 * NW;
        amax = bp + 64 * NW;
        misc = amax + NW;
    }
};

// Tiles have balanced lengths: tile g covers cells floor(g nx / G) ..
// floor((g+1) nx / G) - 1 (at most 64 NW CPT cells, at least 3).  Thread t
// owns tile cells t CPT .. t CPT + CPT - 1; the last active thread may own
// fewer (ragged).
template <int CPT, int NW>
struct TGeo {
    int64_t x0;     // first cell of the tile in the line
    int t;          // thread index in the workgroup
    int j0;         // first own cell, local to the tile
    int nvalid;     // own cells (CPT, fewer for the ragged thread, 0 past the end)
    int Tv;         // cells in this tile
    int tlast;      // thread owning the tile's last cell
    bool active;    // owns cells
    int gk;         // ghost handled by this thread: 0..2 left, 3..5 right, -1 none
    int gpos;       // LDS position of that ghost
    int64_t gcell;  // its cell in the line (periodic)
    int halo[6];    // LDS slots of window positions 0..2 and CPT+3..CPT+5

    // LDS slot of tile cell c, -3 <= c (see TSmem)
    __device__ __forceinline__ int tslot(int c) const
    {
        const int T = 64 * NW * CPT;
        if (c < 0) return T + 3 + c;
        if (c < Tv) return (c % CPT) * (64 * NW) + c / CPT;
        if (c < Tv + 3) return T + 3 + (c - Tv);
        return T + 6;
    }
    __device__ __forceinline__ int own(int q) const { return q * (64 * NW) + t; }

    __device__ __forceinline__ void init(int64_t nx, int tile, int G)
    {
        x0 = (int64_t)tile * nx / G;
        Tv = (int)((int64_t)(tile + 1) * nx / G - x0);
        t = threadIdx.x;
        j0 = t * CPT;
        active = j0 < Tv;
        nvalid = active ? min(CPT, Tv - j0) : 0;
        tlast = (Tv - 1) / CPT;
        gk = (t < 6) ? t : -1;
        gpos = 0;
        gcell = 0;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            halo[p] = active ? tslot(j0 - 3 + p) : 64 * NW * CPT + 6;
            halo[3 + p] = active ? tslot(j0 + CPT + p) : 64 * NW * CPT + 6;
        }
        if (gk >= 0) {
            int64_t cell;
            gpos = 64 * NW * CPT + gk;
            if (gk < 3) {
                cell = x0 - 3 + gk;
            } else {
                cell = x0 + Tv + (gk - 3);
            }
            cell %= nx;
            if (cell < 0) cell += nx;
            gcell = cell;
        }
    }
};

// Per-workgroup view of the synchronisation scratch of its line group.
struct TSync {
    unsigned long long* cnt;  // arrival counter of the group (monotonic within a launch)
    unsigned long long* err;  // set when a spin times out; every workgroup then leaves
    double* pub;              // slots of the group: (tile * 2 + parity) * kTileSlot
    int G;
    int tile;
    long long ep;  // synchronisations done by this workgroup
    __device__ __forceinline__ double* slot(int tl, int parity) const
    {
        return pub + ((int64_t)tl * 2 + parity) * kTileSlot;
    }
};

__device__ __forceinline__ double load_agent(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A(V) on the tile (eq spaceDisc, eq LFflux) and on the ghost cell gv of
// threads 0..5.  RAG: some tile of the line ends inside a thread.  Returns
// false when the line's synchronisation failed.
//
// Published slot (one per tile and stage parity):
//   [0] max |u^{+-}| over the tile, [1..3] Fa at the right faces of tile cells
//   0, 1, 2, [4..6] Fb there, [7..9] Fa at the left faces of cells Tv-3,
//   Tv-2, Tv-1, [10..12] Fb there.
template <int CPT, int NW, int K, bool RAG, bool ROE = false>
__device__ __forceinline__ bool op_A_t(const double (&V)[CPT], double gv, double (&A)[CPT], double& gA,
                                       const TGeo<CPT, NW>& g, const TSmem<CPT, NW>& sm, const PhiConst& pc,
                                       TSync& ts)
{
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (!RAG || q < g.nvalid) sm.tl[g.own(q)] = V[q];
    }
    if (g.gk >= 0) sm.tl[g.gpos] = gv;
    __syncthreads();

    // window w[p] = tile cell j0 - 3 + p, p = 0..CPT+5; past the ragged end it
    // continues into the right ghost cells (then the scratch slot)
    double w[CPT + 6];
#pragma unroll
    for (int q = 0; q < CPT; ++q) w[3 + q] = (RAG && q >= g.nvalid) ? sm.tl[g.tslot(g.j0 + q)] : V[q];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        w[p] = sm.tl[g.halo[p]];
        w[CPT + 3 + p] = sm.tl[g.halo[3 + p]];
    }
    double um[CPT], up[CPT];
    double um_l = 0.0, up_r = 0.0;  // u^- in ghost cell -1, u^+ in ghost cell Tv
    const int pr = 3 + (RAG ? g.nvalid : CPT);  // window position of ghost cell Tv (last thread)
    static_assert(K <= 2, "split lines keep three ghost cells per side: WENO degree <= 2");
    if constexpr (K == 0) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            um[q] = w[3 + q];
            up[q] = w[3 + q];
        }
        um_l = w[2];
        if (g.t == g.tlast) {
#pragma unroll
            for (int p = 3; p <= CPT + 3; ++p)
                if (p == pr) up_r = w[p];
        }
    } else if constexpr (K == 1) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) weno3_cell(w[q + 2], w[q + 3], w[q + 4], pc.eps, um[q], up[q]);
        if (g.t == 0) {
            double unused;
            weno3_cell(w[1], w[2], w[3], pc.eps, um_l, unused);
        }
        if (g.t == g.tlast) {
            if (!RAG || pr == CPT + 3) {
                double unused;
                weno3_cell(w[CPT + 2], w[CPT + 3], w[CPT + 4], pc.eps, unused, up_r);
            } else {
#pragma unroll
                for (int q = 0; q < CPT; ++q)
                    if (q + 3 == pr) up_r = up[q];
            }
        }
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
            if (!RAG || pr == CPT + 3) {
                double unused;
                weno5_cell(w[CPT + 1], w[CPT + 2], w[CPT + 3], w[CPT + 4], w[CPT + 5], E[CPT + 2], E[CPT + 3],
                           E[CPT + 4], unused, up_r);
            } else {
                // the ragged thread's ghost cell sits inside its window: its u^+
                // is the mirror reconstruction already computed at that position
#pragma unroll
                for (int q = 0; q < CPT; ++q)
                    if (q + 3 == pr) up_r = up[q];
            }
        }
    }
    double lmax = 0.0;
    double lastm = um[CPT - 1];
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (!RAG || q < g.nvalid) lmax = fmax(lmax, fmax(fabs(um[q]), fabs(up[q])));
        if (RAG) {
#pragma unroll
            for (int q = 0; q < CPT - 1; ++q)
                if (q == g.nvalid - 1) lastm = um[q];
        }
    }
    sm.bm[g.t] = lastm;
    sm.bp[g.t] = up[0];
    lmax = wave_max(lmax);
    if ((threadIdx.x & 63) == 0) sm.amax[threadIdx.x >> 6] = lmax;
    __syncthreads();

    const double uml = (g.t == 0) ? um_l : sm.bm[g.t - 1];
    const double upr = (g.t == g.tlast) ? up_r : sm.bp[min(g.t + 1, 64 * NW - 1)];
    double Fa[CPT + 1], Fb[CPT + 1];
#pragma unroll
    for (int q = 0; q <= CPT; ++q) {
        const double uL = (q == 0) ? uml : um[q - 1];
        double uR = (q == CPT) ? upr : up[q];
        if (RAG && q == g.nvalid) uR = upr;
        if constexpr (ROE) {
            // the Roe flux needs no global coefficient: all of it in Fa
            Fa[q] = roe_flux2(uL, uR, pc.fa, pc.fb);
            Fb[q] = 0.0;
        } else {
            Fa[q] = flux_f(uL, pc.fa, pc.fb) + flux_f(uR, pc.fa, pc.fb);
            Fb[q] = uR - uL;
        }
    }

    // stage the edge data in LDS: right faces of cells 0..2, left faces of
    // cells Tv-3..Tv-1, and the two edge interfaces themselves
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int cell = g.j0 + q;
            if (RAG && q >= g.nvalid) continue;
            if (cell < 3) {
                sm.misc[17 + cell] = Fa[q + 1];
                sm.misc[20 + cell] = Fb[q + 1];
            }
            const int r = cell - (g.Tv - 3);
            if (r >= 0) {
                sm.misc[23 + r] = Fa[q];
                sm.misc[26 + r] = Fb[q];
            }
        }
        if (g.t == 0) {
            sm.misc[1] = Fa[0];
            sm.misc[2] = Fb[0];
        }
        if (g.t == g.tlast) {
#pragma unroll
            for (int q = 1; q <= CPT; ++q)
                if (q == (RAG ? g.nvalid : CPT)) {
                    sm.misc[3] = Fa[q];
                    sm.misc[4] = Fb[q];
                }
        }
    }
    __syncthreads();

    // thread 0 publishes and arrives; wave 0 waits for the group
    const int parity = ts.ep & 1;
    ts.ep += 1;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        // lanes 0..12 publish the slot with device-coherent stores; waiting for
        // their completion before the arrival orders them before it for any
        // reader that sees the arrival (readers use device-coherent loads), so
        // no cache write-back or invalidation of the whole L2 is needed
        if (lane < 13) {
            double v;
            if (lane == 0) {
                v = sm.amax[0];
#pragma unroll
                for (int w2 = 1; w2 < NW; ++w2) v = fmax(v, sm.amax[w2]);
            } else {
                v = sm.misc[16 + lane];
            }
            __hip_atomic_store(ts.slot(ts.tile, parity) + lane, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
            sm.misc[39] = bad;
        }
        double mx = 0.0;
        for (int i = lane; i < ts.G; i += 64) mx = fmax(mx, load_agent(ts.slot(i, parity)));
        mx = wave_max(mx);
        if (lane < 12) {
            // lanes 0..5: the left neighbour's right-edge (Fa, Fb); 6..11: the
            // right neighbour's left-edge (Fa, Fb)
            const int nb = (lane < 6) ? (ts.tile + ts.G - 1) % ts.G : (ts.tile + 1) % ts.G;
            const int idx = (lane < 6) ? 7 + lane : 1 + (lane - 6);
            sm.misc[5 + lane] = load_agent(ts.slot(nb, parity) + idx);
        }
        if (lane == 0)
            sm.misc[0] = ROE ? 0.0 : (pc.alpha_fixed > 0.0) ? pc.alpha_fixed : lf_alpha(mx, pc.fa, pc.fb);
    }
    __syncthreads();

    const double alpha = sm.misc[0];
    const bool ok = sm.misc[39] == 0.0;
    double F2[CPT + 1];
#pragma unroll
    for (int q = 0; q <= CPT; ++q) F2[q] = fma(-alpha, Fb[q], Fa[q]);
#pragma unroll
    for (int q = 0; q < CPT; ++q) A[q] = (F2[q] - F2[q + 1]) * pc.half_inv_dx;

    gA = 0.0;
    if (g.gk >= 0) {
        // (Fa, Fb) at the left and right faces of the ghost cell
        double faL, fbL, faR, fbR;
        const int k = g.gk;
        if (k < 2) {  // cells -3, -2: the left neighbour's faces
            faL = sm.misc[5 + k];
            fbL = sm.misc[8 + k];
            faR = sm.misc[6 + k];
            fbR = sm.misc[9 + k];
        } else if (k == 2) {  // cell -1: its right face is the tile's left edge
            faL = sm.misc[7];
            fbL = sm.misc[10];
            faR = sm.misc[1];
            fbR = sm.misc[2];
        } else if (k == 3) {  // cell Tv: its left face is the tile's right edge
            faL = sm.misc[3];
            fbL = sm.misc[4];
            faR = sm.misc[11];
            fbR = sm.misc[14];
        } else {  // cells Tv+1, Tv+2: the right neighbour's faces
            faL = sm.misc[11 + (k - 4)];
            fbL = sm.misc[14 + (k - 4)];
            faR = sm.misc[12 + (k - 4)];
            fbR = sm.misc[15 + (k - 4)];
        }
        gA = (fma(-alpha, fbL, faL) - fma(-alpha, fbR, faR)) * pc.half_inv_dx;
    }
    return ok;
}

// x <- Phi(x), ghost gx alongside (eq SSPRK1/2/3)
template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__device__ __forceinline__ bool phi_t(double (&x)[CPT], double& gx, double dt, const TGeo<CPT, NW>& g,
                                      const TSmem<CPT, NW>& sm, const PhiConst& pc, TSync& ts)
{
    double A[CPT], gA;
    if (ST == 1) {
        if (!op_A_t<CPT, NW, K, RAG, ROE>(x, gx, A, gA, g, sm, pc, ts)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = rk_first(x[q], A[q], dt);
        gx = rk_first(gx, gA, dt);
    } else if (ST == 2) {
        double v[CPT], gv;
        if (!op_A_t<CPT, NW, K, RAG, ROE>(x, gx, A, gA, g, sm, pc, ts)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) v[q] = rk_first(x[q], A[q], dt);
        gv = rk_first(gx, gA, dt);
        if (!op_A_t<CPT, NW, K, RAG, ROE>(v, gv, A, gA, g, sm, pc, ts)) return false;
        const double hdt = 0.5 * dt;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = rk2_second(x[q], v[q], A[q], hdt);
        gx = rk2_second(gx, gv, gA, hdt);
    } else {
        double v[CPT], gv;
        if (!op_A_t<CPT, NW, K, RAG, ROE>(x, gx, A, gA, g, sm, pc, ts)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) v[q] = rk_first(x[q], A[q], dt);
        gv = rk_first(gx, gA, dt);
        if (!op_A_t<CPT, NW, K, RAG, ROE>(v, gv, A, gA, g, sm, pc, ts)) return false;
        const double qdt = 0.25 * dt;
#pragma unroll
        for (int q = 0; q < CPT; ++q) v[q] = rk3_second(x[q], v[q], A[q], qdt);
        gv = rk3_second(gx, gv, gA, qdt);
        if (!op_A_t<CPT, NW, K, RAG, ROE>(v, gv, A, gA, g, sm, pc, ts)) return false;
        const double tdt = (2.0 / 3.0) * dt;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = rk3_third(x[q], v[q], A[q], tdt);
        gx = rk3_third(gx, gv, gA, tdt);
    }
    return true;
}

// line access restricted to the tile's own cells (and the thread's ghost cell)
template <int CPT, int NW>
__device__ __forceinline__ void t_load(double (&x)[CPT], double& gx, const double* src, const TGeo<CPT, NW>& g)
{
#pragma unroll
    for (int q = 0; q < CPT; ++q) x[q] = (q < g.nvalid) ? src[g.x0 + g.j0 + q] : 0.0;
    gx = (g.gk >= 0) ? src[g.gcell] : 0.0;
}

template <int CPT, int NW>
__device__ __forceinline__ void t_store(const double (&x)[CPT], double* dst, const TGeo<CPT, NW>& g)
{
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        if (q < g.nvalid) dst[g.x0 + g.j0 + q] = x[q];
}

// x += the tile's cells of line src (and the ghost): every load is issued
// before any is used, in bounds and without a branch (a lane that owns no
// cell reads the tile's first cells, the ragged lane its last cell in place
// of the missing ones, a lane without a ghost cell 0), and the add covers
// every slot: the stage code writes to LDS and reduces only owned cells and
// the ghosts of lanes gk >= 0, and stores skip the rest.  (Loads under
// per-cell predicates would be waited for one at a time.)
template <int CPT, int NW, bool RAG>
__device__ __forceinline__ void t_add(double (&x)[CPT], double& gx, const double* src, const TGeo<CPT, NW>& g)
{
    const double* base = src + g.x0;
    const int j0 = g.active ? g.j0 : 0;
    double t[CPT];
    if constexpr (RAG) {
        const int last = g.active ? g.nvalid - 1 : 0;
#pragma unroll
        for (int q = 0; q < CPT; ++q) t[q] = base[j0 + (q < last ? q : last)];
    } else {
#pragma unroll
        for (int q = 0; q < CPT; ++q) t[q] = base[j0 + q];
    }
    const double gt = src[g.gcell];
#pragma unroll
    for (int q = 0; q < CPT; ++q) x[q] = x[q] + t[q];
    gx = gx + gt;
}

template <int CPT, int NW>
__device__ __forceinline__ void t_copy(const double* src, double* dst, const TGeo<CPT, NW>& g)
{
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        if (q < g.nvalid) dst[g.x0 + g.j0 + q] = src[g.x0 + g.j0 + q];
}

// sum over the tile of (a - b)^2 in a fixed order; valid in thread 0
template <int CPT, int NW>
__device__ __forceinline__ double t_sqdiff(const double (&a)[CPT], const double* b, const TGeo<CPT, NW>& g,
                                           const TSmem<CPT, NW>& sm)
{
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        if (q < g.nvalid) {
            const double d = a[q] - b[g.x0 + g.j0 + q];
            s = fma(d, d, s);
        }
    s = wave_sum(s);
    // amax is free here: the next stage rewrites it only after its first barrier
    if ((threadIdx.x & 63) == 0) sm.amax[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NW; ++w) tot += sm.amax[w];
    }
    return tot;
}

// One chunk on one tile: the same roles and storage as sweep_body.
template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE>
__device__ __forceinline__ bool tiled_chunk(const SweepArgs& a, int c, const TGeo<CPT, NW>& g,
                                            const TSmem<CPT, NW>& sm, TSync& ts)
{
    const int64_t nx = a.nx;
    const double* src = (a.side_in != nullptr && c > 0) ? a.side_in + (int64_t)c * nx
                                                        : a.ustart + (int64_t)c * a.ustart_stride * nx;
    double x[CPT], gx;
    t_load(x, gx, src, g);
    wait_loads();  // (as in sweep_body_t)
    if (a.ucommit != nullptr) t_store(x, a.ucommit + (int64_t)c * a.ucommit_stride * nx, g);
    if (a.inject_last && c == a.nchunks - 1) {
        const double* last = (a.side_in != nullptr) ? a.side_in + (int64_t)a.nchunks * nx
                                                    : a.ustart + (int64_t)a.nchunks * a.ustart_stride * nx;
        t_copy(last, a.ucommit + (int64_t)a.nchunks * a.ucommit_stride * nx, g);
    }
    const double* cstart = (a.ystart != nullptr) ? a.ystart + (int64_t)c * a.ystart_stride * nx : src;
    if (END == END_RESTRICT && c == 0) {
        t_copy(cstart, a.uc_out, g);
        t_copy(a.g != nullptr ? a.g : cstart, a.gc_out, g);
    }

    const int64_t n0 = (int64_t)c * a.m;
    for (int j = 1; j <= a.nsteps; ++j) {
        if (!phi_t<CPT, NW, K, ST, RAG, ROE>(x, gx, a.dt, g, sm, a.pc, ts)) return false;
        if (a.g != nullptr) t_add<CPT, NW, RAG>(x, gx, a.g + (n0 + j) * nx, g);
        if (a.fout != nullptr) {
            if (a.fout_every <= 1) t_store(x, a.fout + (n0 + j) * nx, g);
            else if ((n0 + j) % a.fout_every == 0) t_store(x, a.fout + ((n0 + j) / a.fout_every) * nx, g);
        }
    }

    if constexpr (END == END_NONE) return true;
    if constexpr (END == END_PHI) {
        if (!phi_t<CPT, NW, K, ST, RAG, ROE>(x, gx, a.dt, g, sm, a.pc, ts)) return false;
        t_store(x, a.side_out + (int64_t)c * nx, g);
        return true;
    }
    const int64_t n1 = n0 + a.m;
    if (!phi_t<CPT, NW, K, ST, RAG, ROE>(x, gx, a.dt, g, sm, a.pc, ts)) return false;
    if (a.g != nullptr) t_add<CPT, NW, RAG>(x, gx, a.g + n1 * nx, g);
    const double* cnext = a.cref + (int64_t)(c + 1) * a.cref_stride * nx;
    if (a.resid_partial != nullptr) {
        const double s = t_sqdiff(x, cnext, g, sm);
        if (threadIdx.x == 0) a.resid_partial[(int64_t)c * ts.G + ts.tile] = s;
    }
    if (a.r_out != nullptr) {
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (q < g.nvalid) a.r_out[(int64_t)c * nx + g.x0 + g.j0 + q] = x[q] - cnext[g.x0 + g.j0 + q];
    }
    if constexpr (END == END_CSTEP) {
        if (a.side_out != nullptr) t_store(x, a.side_out + (int64_t)(c + 1) * nx, g);
        return true;
    }
    if (a.coarse_injection) t_copy(cnext, a.uc_out + (int64_t)(c + 1) * nx, g);
    else t_store(x, a.uc_out + (int64_t)(c + 1) * nx, g);
    double y[CPT], gy;
    t_load(y, gy, cstart, g);
    if (!phi_t<CPT, NW, K, ST, RAG, ROE>(y, gy, a.dt_next, g, sm, a.pc, ts)) return false;
#pragma unroll
    for (int q = 0; q < CPT; ++q) y[q] = x[q] - y[q];
    t_store(y, a.gc_out + (int64_t)(c + 1) * nx, g);
    return true;
}

// Workgroup b: tile b % G of line group b / G; the group takes chunks
// grp, grp + groups, ...  Every workgroup of a group runs the same sequence of
// steps, hence the same sequence of synchronisations.
template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE>
__device__ __forceinline__ void tiled_body_t(const SweepArgs& a)
{
    if (a.flag != nullptr && *a.flag != 0) return;
    extern __shared__ double smem_raw[];
    TSmem<CPT, NW> sm;
    sm.init(smem_raw);
    const int G = a.tiles;
    const int tile = blockIdx.x % G;
    const int grp = blockIdx.x / G;
    TGeo<CPT, NW> g;
    g.init(a.nx, tile, G);
    TSync ts;
    ts.err = a.tile_sync;
    ts.cnt = a.tile_sync + kTileCounterStride * (1 + grp);
    ts.pub = a.tile_pub + (int64_t)grp * G * 2 * kTileSlot;
    ts.G = G;
    ts.tile = tile;
    ts.ep = 0;
    for (int c = grp; c < a.nchunks; c += a.groups)
        if (!tiled_chunk<CPT, NW, K, ST, RAG, END, ROE>(a, c, g, sm, ts)) return;
}

// The four roles as separately named kernels; ROE (the numerical flux) is a
// kernel parameter, so that each flux gets its own register allocation.
template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void tiled_relax_f_kernel(SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_NONE, ROE>(a);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void tiled_relax_fc_kernel(SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_CSTEP, ROE>(a);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void tiled_relax_fr_kernel(SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_RESTRICT, ROE>(a);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) void tiled_phi_kernel(SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_PHI, ROE>(a);
}

// ---------------------------------------------------------------------------
// cooperative, persistent launch
// ---------------------------------------------------------------------------
template <class Fn>
static hipError_t launch_coop(Fn fn, const SweepArgs& a, int nw, size_t shmem, hipStream_t s)
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
    SweepArgs b = a;
    b.groups = (int)std::min((long long)a.nchunks, cap / G);
    e = launch_clear_ints((int*)b.tile_sync, 2 * kTileCounterStride * (b.groups + 1), s);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&b};
    return hipLaunchCooperativeKernel((const void*)fn, dim3((unsigned)(b.groups * G)), dim3(64 * nw), args,
                                      (unsigned)shmem, s);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
static hipError_t launch_tiled_role_f(const SweepArgs& a, hipStream_t s)
{
    const size_t shmem = tiled_smem_bytes(CPT, NW);
    switch (a.end_mode) {
    case END_NONE: return launch_coop(tiled_relax_f_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    case END_CSTEP: return launch_coop(tiled_relax_fc_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    case END_RESTRICT: return launch_coop(tiled_relax_fr_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    case END_PHI: return launch_coop(tiled_phi_kernel<CPT, NW, K, ST, RAG, ROE>, a, NW, shmem, s);
    default: return hipErrorInvalidValue;
    }
}

template <int CPT, int NW, int K, int ST, bool RAG>
static hipError_t launch_tiled_role(const SweepArgs& a, hipStream_t s)
{
    if (a.pc.roe) return launch_tiled_role_f<CPT, NW, K, ST, RAG, true>(a, s);
    return launch_tiled_role_f<CPT, NW, K, ST, RAG, false>(a, s);
}

// The tile lengths (balanced, see TGeo) must lie in [3, 64 NW CPT]; the
// launch is ragged unless every tile is a whole number of threads.
template <int CPT, int NW, int K, int ST>
static hipError_t launch_tiled_cfg(const SweepArgs& a, hipStream_t s)
{
    const int64_t nx = a.nx, G = a.tiles;
    if (G < 1 || nx / G < 3 || (nx + G - 1) / G > 64 * NW * CPT) return hipErrorInvalidValue;
    if (nx % G == 0 && (nx / G) % CPT == 0) return launch_tiled_role<CPT, NW, K, ST, false>(a, s);
    return launch_tiled_role<CPT, NW, K, ST, true>(a, s);
}

template <int K, int ST>
hipError_t launch_tiled_ks(const SweepArgs& a, const KernelCfg& cfg, hipStream_t s)
{
#define MGK_CASE(C, W) \
    if (cfg.cpt == C && cfg.nw == W) return launch_tiled_cfg<C, W, K, ST>(a, s);
    MGK_TILED_CFG_LIST(MGK_CASE)
#undef MGK_CASE
    return hipErrorInvalidValue;
}

}  // namespace mgk
