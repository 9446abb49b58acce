// tiled_impl.h -- sweep kernels for lines longer than one workgroup holds
// (included by the tiled_k*_s*.hip translation units).
//
// A line of nx cells is split into G tiles of T = 64*NW*CPT cells (the last
// tile may be shorter, always a multiple of CPT).  Tile g is owned by one
// workgroup, which keeps its cells in registers and, per Runge-Kutta stage:
//   1. mirrors its cells and 2 NG ghost cells (NG on each side, owned by the
//      neighbouring tiles; NG = 3, or 4 for WENO7) into LDS, barrier;
//   2. reconstructs u^-/u^+ of its cells (sec 2.1.1) plus one extra
//      reconstruction in each edge ghost cell, so that it can form every
//      interface flux of its cells itself;
//   3. splits twice the LF flux of each interface (eq LFflux) into the parts
//      before and after the global coefficient is known,
//          2F = Fa - alpha_LF Fb,  Fa = f(u^-) + f(u^+),  Fb = u^+ - u^-
//      (with the Roe flux, eq roeflux, Fa is twice the flux and Fb = 0),
//      and publishes its local max |u^{+-}| and (Fa, Fb) of the NG
//      interfaces inside each edge to a global slot, straight from the
//      threads that hold them;
//   4. polls the slots of the other tiles of the line (each value is its own
//      arrival flag; bounded spin) for alpha_LF = max over all tiles (eq eigs)
//      and its neighbours' edge data;
//   5. updates its cells and, with the neighbours' data, its ghost cells,
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
#include <climits>

#include "sweep_impl.h"

namespace mgk {

constexpr long long kTileSpinLimit = 1LL << 22;

// Ghost cells per tile side: the reconstruction of degree K in a cell reads
// K + 1 cells on each side of it, and a tile reconstructs one cell beyond
// each of its edges, so degree 3 (WENO7) needs 4, lower degrees 3.
template <int K>
constexpr int tile_ghosts()
{
    return K == 3 ? 4 : 3;
}

// LDS: tl[T + 2 NG + 1] | bm[64 NW] | bp[64 NW] | amax[NW] | misc[40] | misc2[40]
//   tl: the tile's cells transposed (cell c at (c mod CPT) * threads + c / CPT,
//   so that every window position is read lane-contiguously, free of bank
//   conflicts), ghost cells -NG..-1 at T..T+NG-1 and Tv..Tv+NG-1 at
//   T+NG..T+2NG-1, one scratch slot at T+2NG for window positions past the
//   ghosts (NG ghost cells per side, tile_ghosts)
//   misc[0] alpha_LF, [1..2] (Fa, Fb) of the tile's left edge interface,
//   [3..4] of its right edge interface, [5..5+2NG-1] the left neighbour's
//   right-edge data (NG Fa, then NG Fb), [5+2NG..5+4NG-1] the right
//   neighbour's left-edge data, [39] error flag; misc2 the same for the second
//   chunk of a paired sweep
template <int CPT, int NW>
struct TSmem {
    double* tl;
    double* bm;
    double* bp;
    double* amax;
    double* misc;
    double* misc2;
    template <int NG = 3>
    __device__ __forceinline__ void init(double* base)
    {
        tl = base;
        bm = tl + 64 * NW * CPT + 2 * NG + 1;
        bp = bm + 64 * NW;
        amax = bp + 64 * NW;
        misc = amax + NW;
        misc2 = misc + 40;
    }
};

// Tiles have balanced lengths in whole threads: with U = floor(nx / CPT),
// tile g covers cells CPT floor(g U / G) .. CPT floor((g+1) U / G) - 1, the
// last tile also the nx mod CPT cells left over (at most 64 NW CPT cells, at
// least 4).  Thread t owns tile cells t CPT .. t CPT + CPT - 1; only the last
// tile's last active thread may own fewer (ragged), and only when CPT does
// not divide nx.
template <int CPT, int NW>
struct TGeo {
    int64_t x0;     // first cell of the tile in the line
    int t;          // thread index in the workgroup
    int j0;         // first own cell, local to the tile
    int nvalid;     // own cells (CPT, fewer for the ragged thread, 0 past the end)
    int Tv;         // cells in this tile
    int tlast;      // thread owning the tile's last cell
    bool active;    // owns cells
    int ng;         // ghost cells per side
    int gk;         // ghost handled by this thread: 0..ng-1 left, ng..2ng-1 right, -1 none
    int gpos;       // LDS position of that ghost
    int64_t gcell;  // its cell in the line (periodic)
    int halo[8];    // LDS slots of window positions 0..ng-1 and CPT+ng..CPT+2ng-1

    // LDS slot of tile cell c, -ng <= c (see TSmem)
    __device__ __forceinline__ int tslot(int c) const
    {
        const int T = 64 * NW * CPT;
        if (c < 0) return T + ng + c;
        if (c < Tv) return (c % CPT) * (64 * NW) + c / CPT;
        if (c < Tv + ng) return T + ng + (c - Tv);
        return T + 2 * ng;
    }
    __device__ __forceinline__ int own(int q) const { return q * (64 * NW) + t; }

    template <int NG = 3>
    __device__ __forceinline__ void init(int64_t nx, int tile, int G)
    {
        ng = NG;
        const int64_t units = nx / CPT;  // whole threads' worth of cells
        x0 = (int64_t)CPT * ((int64_t)tile * units / G);
        Tv = (tile == G - 1) ? (int)(nx - x0) : (int)((int64_t)CPT * ((int64_t)(tile + 1) * units / G) - x0);
        t = threadIdx.x;
        j0 = t * CPT;
        active = j0 < Tv;
        nvalid = active ? min(CPT, Tv - j0) : 0;
        tlast = (Tv - 1) / CPT;
        gk = (t < 2 * NG) ? t : -1;
        gpos = 0;
        gcell = 0;
#pragma unroll
        for (int p = 0; p < NG; ++p) {
            halo[p] = active ? tslot(j0 - NG + p) : 64 * NW * CPT + 2 * NG;
            halo[NG + p] = active ? tslot(j0 + CPT + p) : 64 * NW * CPT + 2 * NG;
        }
        if (gk >= 0) {
            int64_t cell;
            gpos = 64 * NW * CPT + gk;
            if (gk < NG) {
                cell = x0 - NG + gk;
            } else {
                cell = x0 + Tv + (gk - NG);
            }
            cell %= nx;
            if (cell < 0) cell += nx;
            gcell = cell;
        }
    }
};

// Per-workgroup view of the synchronisation scratch of its line group.
struct TSync {
    unsigned long long* cnt;  // arrival counter of the group (split-line adjoint only)
    unsigned long long* err;  // set when a spin times out; every workgroup then leaves
    double* pub;              // slots of the group: (tile * kTileRing + stage % kTileRing) * kTileSlot
    int G;
    int tile;
    long long ep;  // stages done by this workgroup
    int ring;      // slots per tile: kTileRing (sweeps) or 2 (adjoint, by parity)
    __device__ __forceinline__ double* slot(int tl, int r) const
    {
        return pub + ((int64_t)tl * ring + r) * kTileSlot;
    }
};

// device-coherent accesses of the slots (no cache write-back or
// invalidation of the whole L2 is involved)
__device__ __forceinline__ double load_agent(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long load_bits(const double* p)
{
    return __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_agent(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_empty(double* p)
{
    __hip_atomic_store((unsigned long long*)p, kSlotEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Empties every slot value this thread may have written at the previous
// stage (of any kind: thread 0 the maximum, the owners of the NG first and
// NG last cells their edge values), so that each slot position is always
// written and emptied by one and the same thread.
template <int CPT, int NW, int NG, bool RAG>
__device__ __forceinline__ void empty_own(double* old, const TGeo<CPT, NW>& g)
{
    if (threadIdx.x == 0) store_empty(old);
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int cell = g.j0 + q;
            if (RAG && q >= g.nvalid) continue;
            if (cell < NG) {
                store_empty(old + 1 + cell);
                store_empty(old + 1 + NG + cell);
            }
            const int rr = cell - (g.Tv - NG);
            if (rr >= 0) {
                store_empty(old + 1 + 2 * NG + rr);
                store_empty(old + 1 + 3 * NG + rr);
            }
        }
    }
}

// A(V) on the tile (eq spaceDisc, eq LFflux) and on the ghost cell gv of
// threads 0..2NG-1.  RAG: some tile of the line ends inside a thread.
// Returns false when the line's synchronisation failed.
//
// Published slot (one per tile and stage, in a ring of kTileRing):
//   [0] max |u^{+-}| over the tile, [1..NG] Fa at the right faces of tile
//   cells 0..NG-1, [NG+1..2NG] Fb there, [2NG+1..3NG] Fa at the left faces of
//   cells Tv-NG..Tv-1, [3NG+1..4NG] Fb there.
// Every value is its own arrival flag: a slot holds kSlotEmpty until written,
// and a reader polls each value it needs until it is no longer empty (64-bit
// stores and loads are single-copy atomic).  Each value is written by the
// thread that computed it (the max by thread 0 after the block reduction,
// the edge fluxes by their owners), so no barrier gathers them first.
// Reuse: the slot of stage s is emptied again by its writers right after
// their tile has read every tile's stage s + 1 values, which proves that
// every reader is done with stage s; its next use is stage s + 3.  A writer
// waits for its emptying stores to complete before it publishes stage s + 2,
// and a reader reads stage s + 3 only after it saw that writer's stage s + 2
// value, so it can never take a value of stage s for one of stage s + 3.
// The operator comes in two halves.  opA_begin mirrors V into LDS,
// reconstructs, forms (Fa, Fb) of the thread's faces and publishes; opA_end
// waits for every tile's values of the stage and forms A and gA.  misc is the
// LDS area of the chunk (TSmem::misc, or misc2 for the second chunk of a
// paired sweep).  Between the halves a workgroup may run the first half of
// another chunk, whose reconstruction then hides the wait.
template <int CPT, int NW, int K, bool RAG, bool ROE = false>
__device__ __forceinline__ void opA_begin(const double (&V)[CPT], double gv, double (&Fa)[CPT + 1],
                                          double (&Fb)[CPT + 1], const TGeo<CPT, NW>& g,
                                          const TSmem<CPT, NW>& sm, double* misc, const PhiConst& pc,
                                          const TSync& ts)
{
    // the LDS mirror: the windows of other threads read only the first and
    // last NG cells of a whole thread (every cell when CPT <= 2 NG); ragged
    // tiles, where a window may reach past a short thread, mirror every cell
    constexpr int NGW = tile_ghosts<K>();
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (RAG ? q < g.nvalid : (q < NGW || q >= CPT - NGW)) sm.tl[g.own(q)] = V[q];
    }
    if (g.gk >= 0) sm.tl[g.gpos] = gv;
    __syncthreads();

    // window w[p] = tile cell j0 - NG + p, p = 0..CPT+2NG-1; past the ragged
    // end it continues into the right ghost cells (then the scratch slot)
    constexpr int NG = tile_ghosts<K>();
    double w[CPT + 2 * NG];
#pragma unroll
    for (int q = 0; q < CPT; ++q) w[NG + q] = (RAG && q >= g.nvalid) ? sm.tl[g.tslot(g.j0 + q)] : V[q];
#pragma unroll
    for (int p = 0; p < NG; ++p) {
        w[p] = sm.tl[g.halo[p]];
        w[CPT + NG + p] = sm.tl[g.halo[NG + p]];
    }
    double um[CPT], up[CPT];
    double um_l = 0.0, up_r = 0.0;  // u^- in ghost cell -1, u^+ in ghost cell Tv
    const int pr = NG + (RAG ? g.nvalid : CPT);  // window position of ghost cell Tv (last thread)
    if constexpr (K == 0) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            um[q] = w[NG + q];
            up[q] = w[NG + q];
        }
        um_l = w[NG - 1];
        if (g.t == g.tlast) {
#pragma unroll
            for (int p = NG; p <= CPT + NG; ++p)
                if (p == pr) up_r = w[p];
        }
    } else if constexpr (K == 1) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) weno3_cell(w[q + NG - 1], w[q + NG], w[q + NG + 1], pc.eps, um[q], up[q]);
        if (g.t == 0) {
            double unused;
            weno3_cell(w[NG - 2], w[NG - 1], w[NG], pc.eps, um_l, unused);
        }
        if (g.t == g.tlast) {
            if (!RAG || pr == CPT + NG) {
                double unused;
                weno3_cell(w[CPT + NG - 1], w[CPT + NG], w[CPT + NG + 1], pc.eps, unused, up_r);
            } else {
#pragma unroll
                for (int q = 0; q < CPT; ++q)
                    if (q + NG == pr) up_r = up[q];
            }
        }
    } else if constexpr (K == 2) {
        double E[CPT + 2 * NG];
#pragma unroll
        for (int p = NG - 2; p <= CPT + NG + 1; ++p) E[p] = weno5_e(w[p - 1], w[p], w[p + 1], pc.eps);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int p = q + NG;
            weno5_cell(w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], E[p - 1], E[p], E[p + 1], um[q], up[q]);
        }
        if (g.t == 0) {
            double unused;
            const int p = NG - 1;
            weno5_cell(w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], E[p - 1], E[p], E[p + 1], um_l, unused);
        }
        if (g.t == g.tlast) {
            if (!RAG || pr == CPT + NG) {
                double unused;
                const int p = CPT + NG;
                weno5_cell(w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], E[p - 1], E[p], E[p + 1], unused, up_r);
            } else {
                // the ragged thread's ghost cell sits inside its window: its u^+
                // is the mirror reconstruction already computed at that position
#pragma unroll
                for (int q = 0; q < CPT; ++q)
                    if (q + NG == pr) up_r = up[q];
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int p = q + NG;
            weno7_cell(w[p - 3], w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], w[p + 3], pc.eps, um[q], up[q]);
        }
        if (g.t == 0) {
            double unused;
            const int p = NG - 1;
            weno7_cell(w[p - 3], w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], w[p + 3], pc.eps, um_l, unused);
        }
        if (g.t == g.tlast) {
            if (!RAG || pr == CPT + NG) {
                double unused;
                const int p = CPT + NG;
                weno7_cell(w[p - 3], w[p - 2], w[p - 1], w[p], w[p + 1], w[p + 2], w[p + 3], pc.eps, unused, up_r);
            } else {
#pragma unroll
                for (int q = 0; q < CPT; ++q)
                    if (q + NG == pr) up_r = up[q];
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

    // publish: the tile max (thread 0), the edge fluxes (their owners), each
    // after the thread's earlier emptying stores have completed; stage the
    // two edge interfaces of the tile itself in LDS for the ghost cells
    const int r = (int)(ts.ep % kTileRing);
    double* mine = ts.slot(ts.tile, r);
    const bool edge_owner = g.active && (g.j0 < NG || g.j0 + g.nvalid > g.Tv - NG);
    if (threadIdx.x == 0 || edge_owner) __builtin_amdgcn_s_waitcnt(0);
    if (threadIdx.x == 0) {
        // the wave maxima stay in LDS until the next stage's reduction
        double v = sm.amax[0];
#pragma unroll
        for (int w2 = 1; w2 < NW; ++w2) v = fmax(v, sm.amax[w2]);
        store_agent(mine, v);
    }
    if (edge_owner) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int cell = g.j0 + q;
            if (RAG && q >= g.nvalid) continue;
            if (cell < NG) {
                store_agent(mine + 1 + cell, Fa[q + 1]);
                store_agent(mine + 1 + NG + cell, Fb[q + 1]);
            }
            const int rr = cell - (g.Tv - NG);
            if (rr >= 0) {
                store_agent(mine + 1 + 2 * NG + rr, Fa[q]);
                store_agent(mine + 1 + 3 * NG + rr, Fb[q]);
            }
        }
    }
    if (g.active) {
        if (g.t == 0) {
            misc[1] = Fa[0];
            misc[2] = Fb[0];
        }
        if (g.t == g.tlast) {
#pragma unroll
            for (int q = 1; q <= CPT; ++q)
                if (q == (RAG ? g.nvalid : CPT)) {
                    misc[3] = Fa[q];
                    misc[4] = Fb[q];
                }
        }
    }
}

template <int CPT, int NW, int K, bool RAG, bool ROE = false>
__device__ __forceinline__ bool opA_end(const double (&Fa)[CPT + 1], const double (&Fb)[CPT + 1],
                                        double (&A)[CPT], double& gA, const TGeo<CPT, NW>& g,
                                        const TSmem<CPT, NW>& sm, double* misc, const PhiConst& pc, TSync& ts)
{
    constexpr int NG = tile_ghosts<K>();
    // wave 0 polls the G tile maxima and the neighbours' 4 NG edge values
    const int r = (int)(ts.ep % kTileRing);
    ts.ep += 1;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int G = ts.G;
        double mx = 0.0;
        int bad = 0;
        for (int it = lane; it < G + 4 * NG; it += 64) {
            const double* src;
            int dst = -1;
            if (it < G) {
                src = ts.slot(it, r);
            } else {
                // items G..G+2NG-1: the left neighbour's right-edge (Fa, Fb);
                // G+2NG..G+4NG-1: the right neighbour's left-edge (Fa, Fb)
                const int e = it - G;
                const int nb = (e < 2 * NG) ? (ts.tile + G - 1) % G : (ts.tile + 1) % G;
                src = ts.slot(nb, r) + ((e < 2 * NG) ? 1 + 2 * NG + e : 1 + (e - 2 * NG));
                dst = 5 + e;
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
            else misc[dst] = bad ? 0.0 : v;
        }
        mx = wave_max(mx);
        const bool any_bad = __ballot(bad) != 0;
        if (lane == 0) {
            misc[0] = ROE ? 0.0 : (pc.alpha_fixed > 0.0) ? pc.alpha_fixed : lf_alpha(mx, pc.fa, pc.fb);
            misc[39] = any_bad ? 1.0 : 0.0;
        }
    }
    __syncthreads();

    // every tile has now published this stage, so every reader is done with
    // the previous one: its writers empty that slot (used again 3 stages on)
    empty_own<CPT, NW, NG, RAG>(ts.slot(ts.tile, (r + kTileRing - 1) % kTileRing), g);

    const double alpha = misc[0];
    const bool ok = misc[39] == 0.0;
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
        if (k < NG - 1) {  // cells -NG .. -2: the left neighbour's faces
            faL = misc[5 + k];
            fbL = misc[5 + NG + k];
            faR = misc[6 + k];
            fbR = misc[6 + NG + k];
        } else if (k == NG - 1) {  // cell -1: its right face is the tile's left edge
            faL = misc[5 + k];
            fbL = misc[5 + NG + k];
            faR = misc[1];
            fbR = misc[2];
        } else if (k == NG) {  // cell Tv: its left face is the tile's right edge
            faL = misc[3];
            fbL = misc[4];
            faR = misc[5 + 2 * NG];
            fbR = misc[5 + 3 * NG];
        } else {  // cells Tv+1 .. Tv+NG-1: the right neighbour's faces
            const int r2 = k - NG;
            faL = misc[5 + 2 * NG + r2 - 1];
            fbL = misc[5 + 3 * NG + r2 - 1];
            faR = misc[5 + 2 * NG + r2];
            fbR = misc[5 + 3 * NG + r2];
        }
        gA = (fma(-alpha, fbL, faL) - fma(-alpha, fbR, faR)) * pc.half_inv_dx;
    }
    return ok;
}

template <int CPT, int NW, int K, bool RAG, bool ROE = false>
__device__ __forceinline__ bool op_A_t(const double (&V)[CPT], double gv, double (&A)[CPT], double& gA,
                                       const TGeo<CPT, NW>& g, const TSmem<CPT, NW>& sm, const PhiConst& pc,
                                       TSync& ts)
{
    double Fa[CPT + 1], Fb[CPT + 1];
    opA_begin<CPT, NW, K, RAG, ROE>(V, gv, Fa, Fb, g, sm, sm.misc, pc, ts);
    return opA_end<CPT, NW, K, RAG, ROE>(Fa, Fb, A, gA, g, sm, sm.misc, pc, ts);
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

// ---------------------------------------------------------------------------
// fine-integrator matching (sec 3.3.1) on split lines: the average E and the
// central difference D of psi (sweep_impl.h) need each cell's two
// neighbours; at the tile's edges those are the neighbour tiles' edge cells,
// exchanged once per operator application through the same slots.
// ---------------------------------------------------------------------------
// One exchange of cell values: the tile publishes its first and last W cells
// (W = 1: the neighbours of the edge cells for E and D; W = NG: the ghost
// cells of the neighbours) at the positions their owners use for edge data
// at a Runge-Kutta stage, plus a zero maximum, and wave 0 reads every tile's
// maximum (so the ring's rule for emptying holds unchanged) and the
// neighbours' values: misc[5 + e], e < W the left neighbour's cell Tv - W + e,
// e >= W the right neighbour's cell e - W.  Every thread that emptied slot
// values waits for those stores before the barrier, so the tile's maximum,
// published after it, orders them before any reader's next use of the slot.
template <int CPT, int NW, int NG, bool RAG, int W>
__device__ __forceinline__ bool tile_swap(const double (&v)[CPT], const TGeo<CPT, NW>& g, double* misc, TSync& ts)
{
    const bool edge_owner = g.active && (g.j0 < NG || g.j0 + g.nvalid > g.Tv - NG);
    if (threadIdx.x == 0 || edge_owner) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int r = (int)(ts.ep % kTileRing);
    ts.ep += 1;
    double* mine = ts.slot(ts.tile, r);
    if (threadIdx.x == 0) store_agent(mine, 0.0);
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int cell = g.j0 + q;
            if (RAG && q >= g.nvalid) continue;
            if (cell < W) store_agent(mine + 1 + cell, v[q]);
            const int rr = cell - (g.Tv - W);
            if (rr >= 0) store_agent(mine + 1 + 2 * NG + (NG - W) + rr, v[q]);
        }
    }
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int G = ts.G;
        int bad = 0;
        for (int it = lane; it < G + 2 * W; it += 64) {
            const double* src;
            int dst = -1;
            if (it < G) {
                src = ts.slot(it, r);
            } else {
                const int e = it - G;
                src = (e < W) ? ts.slot((ts.tile + G - 1) % G, r) + 1 + 2 * NG + (NG - W) + e
                              : ts.slot((ts.tile + 1) % G, r) + 1 + (e - W);
                dst = 5 + e;
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
            if (dst >= 0) misc[dst] = bad ? 0.0 : __longlong_as_double((long long)bits);
        }
        const bool any_bad = __ballot(bad) != 0;
        if (lane == 0) misc[39] = any_bad ? 1.0 : 0.0;
    }
    __syncthreads();
    empty_own<CPT, NW, NG, RAG>(ts.slot(ts.tile, (r + kTileRing - 1) % kTileRing), g);
    return misc[39] == 0.0;
}

// out = E(v) (avg) or D(v) (diff) on the tile, the operations of ed_op; out may alias v
template <int CPT, int NW, int NG, bool RAG, bool DIFF>
__device__ __forceinline__ bool ed_t(const double (&v)[CPT], double (&out)[CPT], const TGeo<CPT, NW>& g,
                                     const TSmem<CPT, NW>& sm, const PhiConst& pc, TSync& ts)
{
    __syncthreads();  // earlier readers of the line are done
    if (g.active) {
#pragma unroll
        for (int q = 0; q < CPT; ++q)
            if (!RAG || q < g.nvalid) sm.tl[g.own(q)] = v[q];
    }
    if (!tile_swap<CPT, NW, NG, RAG, 1>(v, g, sm.misc, ts)) return false;
    const int last = RAG ? g.nvalid - 1 : CPT - 1;
    const double nl = (g.t == 0) ? sm.misc[5] : sm.tl[g.tslot(g.j0 - 1)];
    const double nr = (g.t == g.tlast) ? sm.misc[6] : sm.tl[g.tslot(g.j0 + last + 1)];
    double r[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const double left = (q == 0) ? nl : v[q - 1];
        const double right = (q == last) ? nr : ((q + 1 < CPT) ? v[q + 1] : nr);
        r[q] = DIFF ? (right - left) * pc.half_inv_dx : 0.5 * (right + left);
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) out[q] = r[q];
    return true;
}

// x <- Psi(x) on the tile (the steps of psi, sweep_impl.h), then the ghost
// cells take their owners' new values
template <int CPT, int NW, int NG, bool RAG>
__device__ __forceinline__ bool psi_t(double (&x)[CPT], double& gx, int order, int M, double dt,
                                      const TGeo<CPT, NW>& g, const TSmem<CPT, NW>& sm, const PhiConst& pc, TSync& ts)
{
    double f[CPT], T[CPT], v[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        v[q] = x[q];
        f[q] = flux_f(x[q], pc.fa, pc.fb);
    }
    if (!ed_t<CPT, NW, NG, RAG, true>(f, T, g, sm, pc, ts)) return false;
    if (order == 0) {
        for (int r = 0; r < M; ++r)
            if (!ed_t<CPT, NW, NG, RAG, false>(v, v, g, sm, pc, ts)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = v[q] - (double)M * dt * T[q];
    } else {
        for (int k = 1; k < M; ++k) {
            if (!ed_t<CPT, NW, NG, RAG, false>(v, v, g, sm, pc, ts)) return false;
            if (!ed_t<CPT, NW, NG, RAG, false>(T, T, g, sm, pc, ts)) return false;
#pragma unroll
            for (int q = 0; q < CPT; ++q) f[q] = flux_f(v[q], pc.fa, pc.fb);
            double Df[CPT];
            if (!ed_t<CPT, NW, NG, RAG, true>(f, Df, g, sm, pc, ts)) return false;
#pragma unroll
            for (int q = 0; q < CPT; ++q) T[q] = T[q] + Df[q];
        }
        if (!ed_t<CPT, NW, NG, RAG, false>(v, v, g, sm, pc, ts)) return false;
#pragma unroll
        for (int q = 0; q < CPT; ++q) x[q] = v[q] - dt * T[q];
    }
    if (!tile_swap<CPT, NW, NG, RAG, NG>(x, g, sm.misc, ts)) return false;
    if (g.gk >= 0) gx = sm.misc[5 + g.gk];
    return true;
}

// one step of the level: Phi, or the matching coarse integrator of M fine
// steps (forward Euler with the LF flux only, as level_step)
template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__device__ __forceinline__ bool level_step_t(double (&x)[CPT], double& gx, double dt, int M, const SweepArgs& a,
                                             const TGeo<CPT, NW>& g, const TSmem<CPT, NW>& sm, const PhiConst& pc,
                                             TSync& ts)
{
    if constexpr (K == 0 && ST == 1 && !ROE) {
        if (a.psi_order != 0 && M > 0)
            return psi_t<CPT, NW, tile_ghosts<K>(), RAG>(x, gx, a.psi_order - 1, M, a.dt_fine, g, sm, pc, ts);
    }
    return phi_t<CPT, NW, K, ST, RAG, ROE>(x, gx, dt, g, sm, pc, ts);
}

// A whole thread's cells at a 16-byte aligned address move as pairs.
template <int CPT>
__device__ __forceinline__ bool t_pairs(const double* p, int nvalid)
{
    return CPT % 2 == 0 && nvalid == CPT && (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

// line access restricted to the tile's own cells (and the thread's ghost cell)
template <int CPT, int NW>
__device__ __forceinline__ void t_load(double (&x)[CPT], double& gx, const double* src, const TGeo<CPT, NW>& g)
{
#pragma unroll
    for (int q = 0; q < CPT; ++q) x[q] = (q < g.nvalid) ? src[g.x0 + g.j0 + q] : 0.0;
    gx = (g.gk >= 0) ? src[g.gcell] : 0.0;
}

// Stores of whole threads go out as 16-byte pairs where aligned: thread t's
// cells lie 8 CPT bytes from its neighbour's, so each store instruction of a
// wave touches 64 cache lines, and pairs halve the requests per line
// written.  (Loads stay single: as pairs, their registers made the sweep
// kernels spill more.)
template <int CPT, int NW>
__device__ __forceinline__ void t_store(const double (&x)[CPT], double* dst, const TGeo<CPT, NW>& g)
{
    double* p = dst + g.x0 + g.j0;
    if (t_pairs<CPT>(p, g.nvalid)) {
#pragma unroll
        for (int q = 0; q + 1 < CPT; q += 2) {
            double2 v;
            v.x = x[q];
            v.y = x[q + 1];
            *reinterpret_cast<double2*>(p + q) = v;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        if (q < g.nvalid) p[q] = x[q];
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
    const double* a = src + g.x0 + g.j0;
    double* b = dst + g.x0 + g.j0;
    if (t_pairs<CPT>(a, g.nvalid) && t_pairs<CPT>(b, g.nvalid)) {
#pragma unroll
        for (int q = 0; q + 1 < CPT; q += 2)
            *reinterpret_cast<double2*>(b + q) = *reinterpret_cast<const double2*>(a + q);
        return;
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        if (q < g.nvalid) b[q] = a[q];
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
        if (!level_step_t<CPT, NW, K, ST, RAG, ROE>(x, gx, a.dt, a.psi_M, a, g, sm, a.pc, ts)) return false;
        if (a.g != nullptr) t_add<CPT, NW, RAG>(x, gx, a.g + (n0 + j) * nx, g);
        if (a.fout != nullptr) {
            if (a.fout_every <= 1) t_store(x, a.fout + (n0 + j) * nx, g);
            else if ((n0 + j) % a.fout_every == 0) t_store(x, a.fout + ((n0 + j) / a.fout_every) * nx, g);
        }
    }

    if constexpr (END == END_NONE) return true;
    if constexpr (END == END_PHI) {
        if (!level_step_t<CPT, NW, K, ST, RAG, ROE>(x, gx, a.dt, a.psi_M, a, g, sm, a.pc, ts)) return false;
        t_store(x, a.side_out + (int64_t)c * nx, g);
        return true;
    }
    const int64_t n1 = n0 + a.m;
    if (!level_step_t<CPT, NW, K, ST, RAG, ROE>(x, gx, a.dt, a.psi_M, a, g, sm, a.pc, ts)) return false;
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
    // the coarse step: its own LF coefficient where the scheme ties it to the step (lf_dx_dt)
    PhiConst pcn = a.pc;
    if (a.alpha_next > 0.0) pcn.alpha_fixed = a.alpha_next;
    if (!level_step_t<CPT, NW, K, ST, RAG, ROE>(y, gy, a.dt_next, a.psi_M_next, a, g, sm, pcn, ts)) return false;
#pragma unroll
    for (int q = 0; q < CPT; ++q) y[q] = x[q] - y[q];
    t_store(y, a.gc_out + (int64_t)(c + 1) * nx, g);
    return true;
}

// ---------------------------------------------------------------------------
// paired sweeps: two chunks per workgroup
// ---------------------------------------------------------------------------
// A chunk is a fixed program of Phi applications ("jobs"): nsteps F-steps,
// then the role's end (one more Phi for the C-step, the FAS restriction or
// END_PHI, and for the restriction a last Phi of the chunk-start line with the
// coarse step).  Each job is ST stages.  A paired sweep runs two chunks A and B
// of the same group in lock step, offset by half a stage:
//     begin(A, s)  begin(B, s)  end(A, s)  begin(A, s+1)  end(B, s)  begin(B, s+1)  end(A, s+1) ...
// so that every wait for the other tiles (end) follows the reconstruction of
// the other chunk, which covers the latency of the device-memory exchange.
// Each chunk has its own slots (and ring) and its own LDS area; the per-cell
// operations are those of tiled_chunk, so the results are bitwise the same.
template <int CPT>
struct TLane {
    double x[CPT], gx;                 // Phi input, then its result
    double v[CPT], gv;                 // intermediate Runge-Kutta stage
    double Fa[CPT + 1], Fb[CPT + 1];   // published fluxes, waiting for alpha_LF
    double xs[CPT];                    // restriction: the C-point result while the start line is stepped
    int c;                             // chunk
};

template <int END>
__device__ __forceinline__ int chunk_jobs(const SweepArgs& a)
{
    return a.nsteps + (END == END_NONE ? 0 : (END == END_RESTRICT ? 2 : 1));
}

// chunk c before its first stage (the preamble of tiled_chunk)
template <int CPT, int NW, int END>
__device__ __forceinline__ void lane_start(const SweepArgs& a, TLane<CPT>& L, const TGeo<CPT, NW>& g)
{
    const int64_t nx = a.nx;
    const int c = L.c;
    const double* src = (a.side_in != nullptr && c > 0) ? a.side_in + (int64_t)c * nx
                                                        : a.ustart + (int64_t)c * a.ustart_stride * nx;
    t_load(L.x, L.gx, src, g);
    wait_loads();
    if (a.ucommit != nullptr) t_store(L.x, a.ucommit + (int64_t)c * a.ucommit_stride * nx, g);
    if (a.inject_last && c == a.nchunks - 1) {
        const double* last = (a.side_in != nullptr) ? a.side_in + (int64_t)a.nchunks * nx
                                                    : a.ustart + (int64_t)a.nchunks * a.ustart_stride * nx;
        t_copy(last, a.ucommit + (int64_t)a.nchunks * a.ucommit_stride * nx, g);
    }
    if (END == END_RESTRICT && c == 0) {
        const double* cstart = (a.ystart != nullptr) ? a.ystart : src;
        t_copy(cstart, a.uc_out, g);
        t_copy(a.g != nullptr ? a.g : cstart, a.gc_out, g);
    }
}

// after the last stage of job j (tiled_chunk's work between Phi applications)
template <int CPT, int NW, bool RAG, int END>
__device__ __forceinline__ void lane_job_done(const SweepArgs& a, int j, TLane<CPT>& L, const TGeo<CPT, NW>& g,
                                              const TSmem<CPT, NW>& sm, const TSync& ts)
{
    const int64_t nx = a.nx;
    const int c = L.c;
    const int64_t n0 = (int64_t)c * a.m;
    if (j < a.nsteps) {
        if (a.g != nullptr) t_add<CPT, NW, RAG>(L.x, L.gx, a.g + (n0 + j + 1) * nx, g);
        if (a.fout != nullptr) {
            if (a.fout_every <= 1) t_store(L.x, a.fout + (n0 + j + 1) * nx, g);
            else if ((n0 + j + 1) % a.fout_every == 0) t_store(L.x, a.fout + ((n0 + j + 1) / a.fout_every) * nx, g);
        }
        return;
    }
    if constexpr (END == END_PHI) {
        t_store(L.x, a.side_out + (int64_t)c * nx, g);
        return;
    }
    if (j == a.nsteps) {
        const int64_t n1 = n0 + a.m;
        if (a.g != nullptr) t_add<CPT, NW, RAG>(L.x, L.gx, a.g + n1 * nx, g);
        const double* cnext = a.cref + (int64_t)(c + 1) * a.cref_stride * nx;
        if (a.resid_partial != nullptr) {
            const double sq = t_sqdiff(L.x, cnext, g, sm);
            if (threadIdx.x == 0) a.resid_partial[(int64_t)c * ts.G + ts.tile] = sq;
        }
        if (a.r_out != nullptr) {
#pragma unroll
            for (int q = 0; q < CPT; ++q)
                if (q < g.nvalid) a.r_out[(int64_t)c * nx + g.x0 + g.j0 + q] = L.x[q] - cnext[g.x0 + g.j0 + q];
        }
        if constexpr (END == END_CSTEP) {
            if (a.side_out != nullptr) t_store(L.x, a.side_out + (int64_t)(c + 1) * nx, g);
            return;
        }
        if (a.coarse_injection) t_copy(cnext, a.uc_out + (int64_t)(c + 1) * nx, g);
        else t_store(L.x, a.uc_out + (int64_t)(c + 1) * nx, g);
        // the last job steps the chunk-start line with the coarse step
        const double* src = (a.side_in != nullptr && c > 0) ? a.side_in + (int64_t)c * nx
                                                            : a.ustart + (int64_t)c * a.ustart_stride * nx;
        const double* cstart = (a.ystart != nullptr) ? a.ystart + (int64_t)c * a.ystart_stride * nx : src;
#pragma unroll
        for (int q = 0; q < CPT; ++q) L.xs[q] = L.x[q];
        t_load(L.x, L.gx, cstart, g);
        return;
    }
    // restriction: g_c = t - Phi_{l+1}(start line)
    double y[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) y[q] = L.xs[q] - L.x[q];
    t_store(y, a.gc_out + (int64_t)(c + 1) * nx, g);
}

// end of stage k of lane L, its Runge-Kutta combination, the job's end when
// the stage was its last, and the first half of stage k + 1
template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE>
__device__ __forceinline__ bool lane_step(const SweepArgs& a, int k, int nst, TLane<CPT>& L, const TGeo<CPT, NW>& g,
                                          const TSmem<CPT, NW>& sm, double* misc, TSync& ts)
{
    double A[CPT], gA;
    const int j = k / ST, st = k - j * ST;
    const bool coarse = END == END_RESTRICT && j == chunk_jobs<END>(a) - 1;
    PhiConst pcj = a.pc;
    if (coarse && a.alpha_next > 0.0) pcj.alpha_fixed = a.alpha_next;
    if (!opA_end<CPT, NW, K, RAG, ROE>(L.Fa, L.Fb, A, gA, g, sm, misc, pcj, ts)) return false;
    const double dt = coarse ? a.dt_next : a.dt;
    if (ST == 1) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) L.x[q] = rk_first(L.x[q], A[q], dt);
        L.gx = rk_first(L.gx, gA, dt);
    } else if (ST == 2) {
        if (st == 0) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) L.v[q] = rk_first(L.x[q], A[q], dt);
            L.gv = rk_first(L.gx, gA, dt);
        } else {
            const double hdt = 0.5 * dt;
#pragma unroll
            for (int q = 0; q < CPT; ++q) L.x[q] = rk2_second(L.x[q], L.v[q], A[q], hdt);
            L.gx = rk2_second(L.gx, L.gv, gA, hdt);
        }
    } else {
        if (st == 0) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) L.v[q] = rk_first(L.x[q], A[q], dt);
            L.gv = rk_first(L.gx, gA, dt);
        } else if (st == 1) {
            const double qdt = 0.25 * dt;
#pragma unroll
            for (int q = 0; q < CPT; ++q) L.v[q] = rk3_second(L.x[q], L.v[q], A[q], qdt);
            L.gv = rk3_second(L.gx, L.gv, gA, qdt);
        } else {
            const double tdt = (2.0 / 3.0) * dt;
#pragma unroll
            for (int q = 0; q < CPT; ++q) L.x[q] = rk3_third(L.x[q], L.v[q], A[q], tdt);
            L.gx = rk3_third(L.gx, L.gv, gA, tdt);
        }
    }
    if (st == ST - 1) lane_job_done<CPT, NW, RAG, END>(a, j, L, g, sm, ts);
    if (k + 1 < nst) {
        const bool first = (st == ST - 1);
        double V[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) V[q] = first ? L.x[q] : L.v[q];
        opA_begin<CPT, NW, K, RAG, ROE>(V, first ? L.gx : L.gv, L.Fa, L.Fb, g, sm, misc, a.pc, ts);
    }
    return true;
}

// chunks cA and cB (cB < 0: none) on one tile
template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE>
__device__ __forceinline__ bool tiled_pair(const SweepArgs& a, int cA, int cB, const TGeo<CPT, NW>& g,
                                           const TSmem<CPT, NW>& sm, TSync& tsA, TSync& tsB)
{
    const bool two = cB >= 0;
    TLane<CPT> LA, LB;
    LA.c = cA;
    LB.c = two ? cB : cA;
    lane_start<CPT, NW, END>(a, LA, g);
    if (two) lane_start<CPT, NW, END>(a, LB, g);
    const int nst = chunk_jobs<END>(a) * ST;
    if (nst == 0) return true;
    opA_begin<CPT, NW, K, RAG, ROE>(LA.x, LA.gx, LA.Fa, LA.Fb, g, sm, sm.misc, a.pc, tsA);
    if (two) opA_begin<CPT, NW, K, RAG, ROE>(LB.x, LB.gx, LB.Fa, LB.Fb, g, sm, sm.misc2, a.pc, tsB);
    for (int k = 0; k < nst; ++k) {
        if (!lane_step<CPT, NW, K, ST, RAG, END, ROE>(a, k, nst, LA, g, sm, sm.misc, tsA)) return false;
        if (two && !lane_step<CPT, NW, K, ST, RAG, END, ROE>(a, k, nst, LB, g, sm, sm.misc2, tsB)) return false;
    }
    return true;
}

// Workgroup b: tile b % G of line group b / G; the group takes chunks
// grp, grp + groups, ...  Every workgroup of a group runs the same sequence of
// steps, hence the same sequence of synchronisations.
template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE, bool PAIR>
__device__ __forceinline__ void tiled_body_t(const SweepArgs& a)
{
    if (a.flag != nullptr && *a.flag != 0) return;
    extern __shared__ double smem_raw[];
    TSmem<CPT, NW> sm;
    sm.template init<tile_ghosts<K>()>(smem_raw);
    const int G = a.tiles;
    const int tile = blockIdx.x % G;
    const int grp = blockIdx.x / G;
    TGeo<CPT, NW> g;
    g.template init<tile_ghosts<K>()>(a.nx, tile, G);
    TSync ts;
    ts.cnt = nullptr;
    ts.ring = kTileRing;
    ts.err = a.tile_sync;
    ts.pub = a.tile_pub + (int64_t)grp * (PAIR ? 2 : 1) * G * kTileRing * kTileSlot;
    ts.G = G;
    ts.tile = tile;
    ts.ep = 0;
    if constexpr (PAIR) {
        if constexpr (K == 0 && ST == 1 && !ROE) {
            if (a.psi_order != 0) {  // matching integrator: one chunk at a time
                for (int c = grp; c < a.nchunks; c += a.groups)
                    if (!tiled_chunk<CPT, NW, K, ST, RAG, END, ROE>(a, c, g, sm, ts)) return;
                return;
            }
        }
        // chunks grp, grp + groups, ... taken two at a time, each with its own slots
        TSync ts2 = ts;
        ts2.pub = ts.pub + (int64_t)G * kTileRing * kTileSlot;
        for (int c = grp; c < a.nchunks; c += 2 * a.groups) {
            const int c2 = c + a.groups;
            if (!tiled_pair<CPT, NW, K, ST, RAG, END, ROE>(a, c, c2 < a.nchunks ? c2 : -1, g, sm, ts, ts2)) return;
        }
    } else {
        for (int c = grp; c < a.nchunks; c += a.groups)
            if (!tiled_chunk<CPT, NW, K, ST, RAG, END, ROE>(a, c, g, sm, ts)) return;
    }
}

// The four roles as separately named kernels; ROE (the numerical flux) is a
// kernel parameter, so that each flux gets its own register allocation.
// PAIR: two chunks per workgroup (tiled_pair); with fewer than 16 waves such
// a workgroup keeps up to 256 VGPRs for the two chunks' state.
// Whole-thread tiles are compiled for 4 waves per SIMD (at most 128 VGPRs):
// with 16 waves that is one workgroup per compute unit either way, but the
// schedule built for that occupancy ran the 65536-cell F-sweep 12 % faster
// (15.0 against 16.9 ms); ragged tiles keep the compiler's budget, which
// holds them free of register spills.
#define MGK_TILED_WAVES_PER_EU (RAG ? 1 : ((PAIR && NW < 16) || CPT >= 16) ? 2 : 4)
template <int CPT, int NW, int K, int ST, bool RAG, bool ROE, bool PAIR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MGK_TILED_WAVES_PER_EU))) void tiled_relax_f_kernel(
    SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_NONE, ROE, PAIR>(a);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE, bool PAIR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MGK_TILED_WAVES_PER_EU))) void tiled_relax_fc_kernel(
    SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_CSTEP, ROE, PAIR>(a);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE, bool PAIR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MGK_TILED_WAVES_PER_EU))) void tiled_relax_fr_kernel(
    SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_RESTRICT, ROE, PAIR>(a);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE, bool PAIR>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(MGK_TILED_WAVES_PER_EU))) void tiled_phi_kernel(
    SweepArgs a)
{
    tiled_body_t<CPT, NW, K, ST, RAG, END_PHI, ROE, PAIR>(a);
}

// ---------------------------------------------------------------------------
// batches: every split-line problem of a phase in one persistent launch
// ---------------------------------------------------------------------------
// Work items are the (problem, chunk) pairs of the launch's table, problem i
// owning items offset[i] .. offset[i+1] - 1.  Line group grp (workgroups
// grp G .. grp G + G - 1) takes items grp, grp + groups, ..., or, with one
// item per problem, the items a greedy schedule gives it (up to
// kBatchSchedGroups groups and kBatchSchedItems items).  Each item runs
// exactly tiled_chunk on its problem's arguments, with the problem's own
// tile geometry; the group's slot ring simply continues from item to item.
// A problem whose stop flag is set (it converged) contributes no work.
constexpr int kBatchSchedGroups = 256;
constexpr int kBatchSchedItems = 1024;

template <int CPT, int NW, int K, int ST, bool RAG, int END, bool ROE>
__device__ __forceinline__ void tiled_batch_body(const BatchLaunch& t)
{
    extern __shared__ double smem_raw[];
    TSmem<CPT, NW> sm;
    sm.template init<tile_ghosts<K>()>(smem_raw);
    const int G = t.tiles;
    const int tile = blockIdx.x % G;
    const int grp = blockIdx.x / G;
    TSync ts;
    ts.cnt = nullptr;
    ts.ring = kTileRing;
    ts.err = t.tile_sync;
    ts.pub = t.tile_pub + (int64_t)grp * G * kTileRing * kTileSlot;
    ts.G = G;
    ts.tile = tile;
    ts.ep = 0;
    // One work item per problem (serial solves, listed longest first) and more
    // items than line groups: the items go to the groups by the greedy rule
    // (each to the group with the fewest steps so far, ties to the lowest
    // group), which every workgroup evaluates identically; otherwise group g
    // takes items g, g + groups, ...
    __shared__ int owner[kBatchSchedItems];
    const bool sched = t.nblocks == t.nprob && t.groups < t.nblocks && t.groups <= kBatchSchedGroups &&
                       t.nblocks <= kBatchSchedItems;
    if (sched) {
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            long long load[kBatchSchedGroups / 64];
#pragma unroll
            for (int r = 0; r < kBatchSchedGroups / 64; ++r) load[r] = (lane + 64 * r < t.groups) ? 0 : LLONG_MAX;
            for (int j = 0; j < t.nblocks; ++j) {
                long long best = LLONG_MAX;
                int bg = 0;
#pragma unroll
                for (int r = 0; r < kBatchSchedGroups / 64; ++r)
                    if (load[r] < best) {
                        best = load[r];
                        bg = lane + 64 * r;
                    }
                // lowest (load, group) over the wave
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) {
                    const long long ob = __shfl_xor(best, off);
                    const int og = __shfl_xor(bg, off);
                    if (ob < best || (ob == best && og < bg)) {
                        best = ob;
                        bg = og;
                    }
                }
                if (lane == (bg & 63)) load[bg >> 6] += t.args[t.problem[j]].nsteps;
                if (lane == 0) owner[j] = bg;
            }
        }
        __syncthreads();
    }
    for (int j = sched ? 0 : grp; j < t.nblocks; j += sched ? 1 : t.groups) {
        if (sched && owner[j] != grp) continue;
        int lo = 0, hi = t.nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (t.offset[mid] <= j) lo = mid;
            else hi = mid - 1;
        }
        const SweepArgs a = t.args[t.problem[lo]];
        if (a.flag != nullptr && *a.flag != 0) continue;
        TGeo<CPT, NW> g;
        g.template init<tile_ghosts<K>()>(a.nx, tile, G);
        if (!tiled_chunk<CPT, NW, K, ST, RAG, END, ROE>(a, j - t.offset[lo], g, sm, ts)) return;
    }
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(RAG ? 1 : 4))) void tiled_batch_f_kernel(
    BatchLaunch t)
{
    tiled_batch_body<CPT, NW, K, ST, RAG, END_NONE, ROE>(t);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(RAG ? 1 : 4))) void tiled_batch_fc_kernel(
    BatchLaunch t)
{
    tiled_batch_body<CPT, NW, K, ST, RAG, END_CSTEP, ROE>(t);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(RAG ? 1 : 4))) void tiled_batch_fr_kernel(
    BatchLaunch t)
{
    tiled_batch_body<CPT, NW, K, ST, RAG, END_RESTRICT, ROE>(t);
}

// ---------------------------------------------------------------------------
// cooperative, persistent launch
// ---------------------------------------------------------------------------
template <class Fn>
static hipError_t launch_coop(Fn fn, const SweepArgs& a, int nw, size_t shmem, bool pair, hipStream_t s)
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
    // clear the error word and empty every slot of the launch's groups
    e = launch_clear_ints((int*)b.tile_sync, 2, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u64((unsigned long long*)b.tile_pub, kSlotEmpty,
                        (int64_t)b.groups * (pair ? 2 : 1) * G * kTileRing * kTileSlot, s);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&b};
    return hipLaunchCooperativeKernel((const void*)fn, dim3((unsigned)(b.groups * G)), dim3(64 * nw), args,
                                      (unsigned)shmem, s);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE, bool PAIR>
static hipError_t launch_tiled_role_f(const SweepArgs& a, hipStream_t s)
{
    const size_t shmem = tiled_smem_bytes(CPT, NW);
    switch (a.end_mode) {
    case END_NONE: return launch_coop(tiled_relax_f_kernel<CPT, NW, K, ST, RAG, ROE, PAIR>, a, NW, shmem, PAIR, s);
    case END_CSTEP: return launch_coop(tiled_relax_fc_kernel<CPT, NW, K, ST, RAG, ROE, PAIR>, a, NW, shmem, PAIR, s);
    case END_RESTRICT:
        return launch_coop(tiled_relax_fr_kernel<CPT, NW, K, ST, RAG, ROE, PAIR>, a, NW, shmem, PAIR, s);
    case END_PHI: return launch_coop(tiled_phi_kernel<CPT, NW, K, ST, RAG, ROE, PAIR>, a, NW, shmem, PAIR, s);
    default: return hipErrorInvalidValue;
    }
}

template <int CPT, int NW, int K, int ST, bool RAG, bool PAIR>
static hipError_t launch_tiled_role(const SweepArgs& a, hipStream_t s)
{
    if (a.pc.roe) return launch_tiled_role_f<CPT, NW, K, ST, RAG, true, PAIR>(a, s);
    return launch_tiled_role_f<CPT, NW, K, ST, RAG, false, PAIR>(a, s);
}

// The tile lengths (balanced in whole threads, see TGeo) must lie in
// [3, 64 NW CPT]; the launch is ragged unless CPT divides nx.
template <int CPT, int NW, int K, int ST, bool PAIR>
static hipError_t launch_tiled_cfg(const SweepArgs& a, hipStream_t s)
{
    const int64_t nx = a.nx, G = a.tiles;
    if (!tiles_fit(nx, G, CPT, NW)) return hipErrorInvalidValue;
    if (nx % CPT == 0) return launch_tiled_role<CPT, NW, K, ST, false, PAIR>(a, s);
    return launch_tiled_role<CPT, NW, K, ST, true, PAIR>(a, s);
}

template <int K, int ST>
hipError_t launch_tiled_ks(const SweepArgs& a, const KernelCfg& cfg, hipStream_t s)
{
#define MGK_CASE(C, W) \
    if (cfg.cpt == C && cfg.nw == W && cfg.intervals == 1) return launch_tiled_cfg<C, W, K, ST, false>(a, s);
    MGK_TILED_CFG_LIST(MGK_CASE)
#undef MGK_CASE
#define MGK_CASE(C, W) \
    if (cfg.cpt == C && cfg.nw == W && cfg.intervals == 2) return launch_tiled_cfg<C, W, K, ST, true>(a, s);
    MGK_TILED_PAIR_CFG_LIST(MGK_CASE)
#undef MGK_CASE
    return hipErrorInvalidValue;
}

// every split-line problem of a batch phase (same shape and tile count) in
// one cooperative, persistent launch
template <class Fn>
static hipError_t launch_coop_batch(Fn fn, const BatchLaunch& t, int nw, size_t shmem, hipStream_t s)
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
    const int G = t.tiles;
    if (G < 1 || cap < G) return hipErrorCooperativeLaunchTooLarge;
    BatchLaunch b = t;
    b.groups = (int)std::min((long long)t.nblocks, cap / G);
    e = launch_clear_ints((int*)b.tile_sync, 2, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u64((unsigned long long*)b.tile_pub, kSlotEmpty, (int64_t)b.groups * G * kTileRing * kTileSlot, s);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&b};
    return hipLaunchCooperativeKernel((const void*)fn, dim3((unsigned)(b.groups * G)), dim3(64 * nw), args,
                                      (unsigned)shmem, s);
}

template <int CPT, int NW, int K, int ST, bool RAG, bool ROE>
static hipError_t launch_tiled_batch_role(const BatchLaunch& t, hipStream_t s)
{
    const size_t shmem = tiled_smem_bytes(CPT, NW);
    switch (t.end_mode) {
    case END_NONE: return launch_coop_batch(tiled_batch_f_kernel<CPT, NW, K, ST, RAG, ROE>, t, NW, shmem, s);
    case END_CSTEP: return launch_coop_batch(tiled_batch_fc_kernel<CPT, NW, K, ST, RAG, ROE>, t, NW, shmem, s);
    case END_RESTRICT: return launch_coop_batch(tiled_batch_fr_kernel<CPT, NW, K, ST, RAG, ROE>, t, NW, shmem, s);
    default: return hipErrorInvalidValue;
    }
}

template <int CPT, int NW, int K, int ST>
static hipError_t launch_tiled_batch_cfg(const BatchLaunch& t, hipStream_t s)
{
    if (t.ragged) {
        if (t.roe) return launch_tiled_batch_role<CPT, NW, K, ST, true, true>(t, s);
        return launch_tiled_batch_role<CPT, NW, K, ST, true, false>(t, s);
    }
    if (t.roe) return launch_tiled_batch_role<CPT, NW, K, ST, false, true>(t, s);
    return launch_tiled_batch_role<CPT, NW, K, ST, false, false>(t, s);
}

template <int K, int ST>
hipError_t launch_tiled_batch_ks(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s)
{
    if (t.nblocks <= 0) return hipSuccess;
#define MGK_CASE(C, W) \
    if (cfg.cpt == C && cfg.nw == W && cfg.intervals == 1) return launch_tiled_batch_cfg<C, W, K, ST>(t, s);
    MGK_TILED_BATCH_CFG_LIST(MGK_CASE)
#undef MGK_CASE
    return hipErrorInvalidValue;
}

}  // namespace mgk
