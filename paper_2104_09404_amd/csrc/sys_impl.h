// sys_impl.h -- sweep kernels for systems of conservation laws: shallow water
// (D = 2, eq shallowWater) and the Euler equations of an ideal gas (D = 3,
// eq Euler), included by the sys_s*_k*.hip translation units.
//
// One workgroup per line, one cell per thread (lines of up to 512 cells),
// the cell's D components in registers.  A line of a system is stored as its
// D components one after the other, nx cells each, so SweepArgs.nx is D nx
// and every node offset of the scalar path carries over.  Per Runge-Kutta
// stage (sec 2.2) a thread:
//   1. writes its cell to LDS (one plane per component), barrier;
//   2. reconstructs characteristic-wise (sec 2.1.1): the cells i-K..i+K are
//      projected on the left eigenvectors of the cell's own state, each
//      characteristic variable goes through the scalar WENO of degree K
//      (cell_math.h), and u^-_{i+1/2}, u^+_{i-1/2} are mapped back with the
//      right eigenvectors; publishes both, and for the Lax-Friedrichs flux
//      the cell's largest wave speed (wave max, one LDS slot per wave),
//      barrier;
//   3. forms twice the flux of both of its faces -- LF with the global
//      alpha_LF (eq LFflux, eigs) or Roe with Roe averages and the
//      Harten-Hyman fix (eq roeflux) -- and the stage update.  Both threads
//      of an interface evaluate its flux from the same operands, so every
//      component is conserved to round-off.
// The flux parameter (g for shallow water, gamma for Euler) arrives in pc.fb.
#pragma once
#include "sweep_impl.h"

namespace mgk {

constexpr int kSysMaxWaves = 16;

template <int SYS>
struct Phys;

// shallow water: u = (h, hu), f = (hu, hu^2/h + g h^2/2)
template <>
struct Phys<2> {
    static constexpr int D = 2;
    __device__ static void flux(const double (&u)[2], double g, double (&f)[2])
    {
        const double v = u[1] / u[0];
        f[0] = u[1];
        f[1] = fma(u[1], v, 0.5 * g * u[0] * u[0]);
    }
    // lambda = v -/+ c, c = sqrt(g h); R = [[1, 1], [v - c, v + c]];
    // L = R^-1 = (1/(2c)) [[v + c, -1], [-(v - c), 1]]
    __device__ static void eig(double v, double h, double g, double (&lam)[2], double (&R)[2][2],
                               double (&L)[2][2])
    {
        const double c = sqrt(g * h), ic = 0.5 / c;
        lam[0] = v - c;
        lam[1] = v + c;
        R[0][0] = 1.0;
        R[0][1] = 1.0;
        R[1][0] = lam[0];
        R[1][1] = lam[1];
        L[0][0] = lam[1] * ic;
        L[0][1] = -ic;
        L[1][0] = -lam[0] * ic;
        L[1][1] = ic;
    }
    __device__ static void eig_state(const double (&u)[2], double g, double (&lam)[2], double (&R)[2][2],
                                     double (&L)[2][2])
    {
        eig(u[1] / u[0], u[0], g, lam, R, L);
    }
    __device__ static void speeds(const double (&u)[2], double g, double (&lam)[2])
    {
        const double v = u[1] / u[0], c = sqrt(g * u[0]);
        lam[0] = v - c;
        lam[1] = v + c;
    }
    __device__ static double max_speed(const double (&u)[2], double g)
    {
        return fabs(u[1] / u[0]) + sqrt(g * u[0]);
    }
    // Roe averages: h = (h- + h+)/2, v = sqrt(h)-weighted mean velocity
    __device__ static void roe_eig(const double (&uL)[2], const double (&uR)[2], double g, double (&lam)[2],
                                   double (&R)[2][2], double (&L)[2][2])
    {
        const double sL = sqrt(uL[0]), sR = sqrt(uR[0]);
        const double v = (uR[1] / uR[0] * sR + uL[1] / uL[0] * sL) / (sR + sL);
        eig(v, 0.5 * (uR[0] + uL[0]), g, lam, R, L);
    }
};

// Euler: u = (rho, rho v, E), p = (gamma - 1)(E - rho v^2/2), H = (E + p)/rho
template <>
struct Phys<3> {
    static constexpr int D = 3;
    __device__ static double pressure(const double (&u)[3], double gam)
    {
        return (gam - 1.0) * (u[2] - 0.5 * u[1] * (u[1] / u[0]));
    }
    __device__ static void flux(const double (&u)[3], double gam, double (&f)[3])
    {
        const double v = u[1] / u[0], p = pressure(u, gam);
        f[0] = u[1];
        f[1] = fma(u[1], v, p);
        f[2] = (u[2] + p) * v;
    }
    // lambda = v - c, v, v + c with c^2 = (gamma - 1)(H - v^2/2); R has the
    // columns (1, v - c, H - v c), (1, v, v^2/2), (1, v + c, H + v c); with
    // b1 = (gamma - 1)/c^2 and b2 = b1 v^2/2 its inverse has the rows
    //   (b2 + v/c, -(b1 v + 1/c), b1)/2,  (1 - b2, b1 v, -b1),  (b2 - v/c, -(b1 v - 1/c), b1)/2
    __device__ static void eig(double v, double H, double gam, double (&lam)[3], double (&R)[3][3],
                               double (&L)[3][3])
    {
        const double gm = gam - 1.0;
        const double c2 = gm * fma(-0.5 * v, v, H), c = sqrt(c2), ic = 1.0 / c;
        const double b1 = gm / c2, b2 = 0.5 * b1 * v * v, vc = v * c;
        lam[0] = v - c;
        lam[1] = v;
        lam[2] = v + c;
        R[0][0] = 1.0;
        R[1][0] = lam[0];
        R[2][0] = H - vc;
        R[0][1] = 1.0;
        R[1][1] = v;
        R[2][1] = 0.5 * v * v;
        R[0][2] = 1.0;
        R[1][2] = lam[2];
        R[2][2] = H + vc;
        const double vic = v * ic;
        L[0][0] = 0.5 * (b2 + vic);
        L[0][1] = -0.5 * fma(b1, v, ic);
        L[0][2] = 0.5 * b1;
        L[1][0] = 1.0 - b2;
        L[1][1] = b1 * v;
        L[1][2] = -b1;
        L[2][0] = 0.5 * (b2 - vic);
        L[2][1] = -0.5 * fma(b1, v, -ic);
        L[2][2] = 0.5 * b1;
    }
    __device__ static void eig_state(const double (&u)[3], double gam, double (&lam)[3], double (&R)[3][3],
                                     double (&L)[3][3])
    {
        const double p = pressure(u, gam);
        eig(u[1] / u[0], (u[2] + p) / u[0], gam, lam, R, L);
    }
    __device__ static void speeds(const double (&u)[3], double gam, double (&lam)[3])
    {
        const double v = u[1] / u[0], c = sqrt(gam * pressure(u, gam) / u[0]);
        lam[0] = v - c;
        lam[1] = v;
        lam[2] = v + c;
    }
    __device__ static double max_speed(const double (&u)[3], double gam)
    {
        return fabs(u[1] / u[0]) + sqrt(gam * pressure(u, gam) / u[0]);
    }
    // Roe averages: sqrt(rho)-weighted velocity and enthalpy
    __device__ static void roe_eig(const double (&uL)[3], const double (&uR)[3], double gam, double (&lam)[3],
                                   double (&R)[3][3], double (&L)[3][3])
    {
        const double sL = sqrt(uL[0]), sR = sqrt(uR[0]);
        const double HL = (uL[2] + pressure(uL, gam)) / uL[0], HR = (uR[2] + pressure(uR, gam)) / uR[0];
        const double v = (uR[1] / uR[0] * sR + uL[1] / uL[0] * sL) / (sR + sL);
        const double H = (HR * sR + HL * sL) / (sR + sL);
        eig(v, H, gam, lam, R, L);
    }
};

// twice the interface flux from the two face states
template <int SYS, bool ROE>
__device__ __forceinline__ void sys_flux2(const double (&uL)[Phys<SYS>::D], const double (&uR)[Phys<SYS>::D],
                                          double par, double alpha, double (&F2)[Phys<SYS>::D])
{
    constexpr int D = Phys<SYS>::D;
    double fL[D], fR[D];
    Phys<SYS>::flux(uL, par, fL);
    Phys<SYS>::flux(uR, par, fR);
    if constexpr (!ROE) {
#pragma unroll
        for (int d = 0; d < D; ++d) F2[d] = fma(-alpha, uR[d] - uL[d], fL[d] + fR[d]);
    } else {
        double lam[D], R[D][D], L[D][D], lL[D], lR[D];
        Phys<SYS>::roe_eig(uL, uR, par, lam, R, L);
        Phys<SYS>::speeds(uL, par, lL);
        Phys<SYS>::speeds(uR, par, lR);
#pragma unroll
        for (int d = 0; d < D; ++d) F2[d] = fL[d] + fR[d];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double jump = 0.0;  // alpha_k = l_k . (u+ - u-)
#pragma unroll
            for (int d = 0; d < D; ++d) jump = fma(L[k][d], uR[d] - uL[d], jump);
            const double delta = fmax(0.0, fmax(lam[k] - lL[k], lR[k] - lam[k]));
            const double al = fabs(lam[k]);
            const double q = (al < delta) ? 0.5 * (lam[k] * lam[k] / delta + delta) : al;
            const double w = q * jump;
#pragma unroll
            for (int d = 0; d < D; ++d) F2[d] = fma(-w, R[d][k], F2[d]);
        }
    }
}

// geometry: thread t owns cell t of an n-cell line (t < n)
struct SysGeo {
    int n, t, npad, left, right;
    bool active;
    __device__ __forceinline__ void init(int ncell)
    {
        n = ncell;
        t = threadIdx.x;
        npad = blockDim.x;
        active = t < n;
        left = (t == 0) ? n - 1 : t - 1;
        right = (t == n - 1) ? 0 : t + 1;
    }
};

// LDS: line[D npad] | bm[D npad] | bp[D npad] | amax[2 kSysMaxWaves] | wred[kSysMaxWaves]
template <int D>
struct SysSmem {
    double *line, *bm, *bp, *amax, *wred;
    __device__ __forceinline__ void init(double* base, int npad)
    {
        line = base;
        bm = line + D * npad;
        bp = bm + D * npad;
        amax = bp + D * npad;
        wred = amax + 2 * kSysMaxWaves;
    }
};

inline size_t sys_smem_bytes(int D, int npad) { return sizeof(double) * (size_t)(3 * D * npad + 3 * kSysMaxWaves); }

// scalar WENO of degree K of one characteristic variable over cells i-K..i+K:
// wm = its value at i+1/2, wp at i-1/2
template <int K>
__device__ __forceinline__ void char_weno(const double (&cw)[2 * K + 1], double eps, double& wm, double& wp)
{
    if constexpr (K == 1) {
        weno3_cell(cw[0], cw[1], cw[2], eps, wm, wp);
    } else if constexpr (K == 2) {
        const double Em = weno5_e(cw[0], cw[1], cw[2], eps);
        const double E0 = weno5_e(cw[1], cw[2], cw[3], eps);
        const double Ep = weno5_e(cw[2], cw[3], cw[4], eps);
        weno5_cell(cw[0], cw[1], cw[2], cw[3], cw[4], Em, E0, Ep, wm, wp);
    } else {
        weno7_cell(cw[0], cw[1], cw[2], cw[3], cw[4], cw[5], cw[6], eps, wm, wp);
    }
}

// A(V) of the thread's cell (eq spaceDisc)
template <int SYS, int K, bool ROE>
__device__ __forceinline__ void op_A_sys(const double (&V)[Phys<SYS>::D], double (&A)[Phys<SYS>::D], const SysGeo& g,
                                         const SysSmem<Phys<SYS>::D>& sm, const PhiConst& pc, int& par)
{
    constexpr int D = Phys<SYS>::D;
    const double pp = pc.fb;  // g or gamma
    if (g.active) {
#pragma unroll
        for (int d = 0; d < D; ++d) sm.line[d * g.npad + g.t] = V[d];
    }
    __syncthreads();
    double um[D], up[D];
#pragma unroll
    for (int d = 0; d < D; ++d) um[d] = up[d] = V[d];
    if (g.active) {
        if constexpr (K > 0) {
            double lam[D], R[D][D], L[D][D];
            Phys<SYS>::eig_state(V, pp, lam, R, L);
            double w[2 * K + 1][D];
#pragma unroll
            for (int j = 0; j <= 2 * K; ++j) {
                const int c = wrapi(g.t - K + j, g.n);
#pragma unroll
                for (int d = 0; d < D; ++d) w[j][d] = (j == K) ? V[d] : sm.line[d * g.npad + c];
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
#pragma unroll
        for (int d = 0; d < D; ++d) {
            sm.bm[d * g.npad + g.t] = um[d];
            sm.bp[d * g.npad + g.t] = up[d];
        }
    }
    double alpha = 0.0;
    if constexpr (!ROE) {
        double lmax = g.active ? fmax(Phys<SYS>::max_speed(um, pp), Phys<SYS>::max_speed(up, pp)) : 0.0;
        lmax = wave_max(lmax);
        const int nw = g.npad >> 6;
        if ((threadIdx.x & 63) == 0) sm.amax[par * kSysMaxWaves + (threadIdx.x >> 6)] = lmax;
        __syncthreads();
        alpha = pc.alpha_fixed;
        if (!(alpha > 0.0)) {
            for (int w2 = 0; w2 < nw; ++w2) lmax = fmax(lmax, sm.amax[par * kSysMaxWaves + w2]);
            alpha = lmax;
        }
        par ^= 1;
    } else {
        __syncthreads();
    }
    if (g.active) {
        double lm[D], rp[D], Fl[D], Fr[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lm[d] = sm.bm[d * g.npad + g.left];   // u^-_{i-1/2}
            rp[d] = sm.bp[d * g.npad + g.right];  // u^+_{i+1/2}
        }
        sys_flux2<SYS, ROE>(lm, up, pp, alpha, Fl);
        sys_flux2<SYS, ROE>(um, rp, pp, alpha, Fr);
#pragma unroll
        for (int d = 0; d < D; ++d) A[d] = (Fl[d] - Fr[d]) * pc.half_inv_dx;
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) A[d] = 0.0;
    }
}

// x <- Phi(x) with step dt (eq SSPRK1/2/3)
template <int SYS, int K, int ST, bool ROE>
__device__ __forceinline__ void phi_sys(double (&x)[Phys<SYS>::D], double dt, const SysGeo& g,
                                        const SysSmem<Phys<SYS>::D>& sm, const PhiConst& pc, int& par)
{
    constexpr int D = Phys<SYS>::D;
    double A[D], v[D];
    op_A_sys<SYS, K, ROE>(x, A, g, sm, pc, par);
    if constexpr (ST == 1) {
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = rk_first(x[d], A[d], dt);
    } else if constexpr (ST == 2) {
#pragma unroll
        for (int d = 0; d < D; ++d) v[d] = rk_first(x[d], A[d], dt);
        op_A_sys<SYS, K, ROE>(v, A, g, sm, pc, par);
        const double hdt = 0.5 * dt;
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = rk2_second(x[d], v[d], A[d], hdt);
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) v[d] = rk_first(x[d], A[d], dt);
        op_A_sys<SYS, K, ROE>(v, A, g, sm, pc, par);
        const double qdt = 0.25 * dt;
#pragma unroll
        for (int d = 0; d < D; ++d) v[d] = rk3_second(x[d], v[d], A[d], qdt);
        op_A_sys<SYS, K, ROE>(v, A, g, sm, pc, par);
        const double tdt = (2.0 / 3.0) * dt;
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = rk3_third(x[d], v[d], A[d], tdt);
    }
}

// line transfers of the thread's cell (components d n + t of a line)
template <int D>
__device__ __forceinline__ void sys_load(double (&x)[D], const double* src, const SysGeo& g)
{
    if (g.active) {
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = src[d * g.n + g.t];
    }
}
template <int D>
__device__ __forceinline__ void sys_store(const double (&x)[D], double* dst, const SysGeo& g)
{
    if (g.active) {
#pragma unroll
        for (int d = 0; d < D; ++d) dst[d * g.n + g.t] = x[d];
    }
}
template <int D>
__device__ __forceinline__ void sys_add(double (&x)[D], const double* src, const SysGeo& g)
{
    if (g.active) {
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] += src[d * g.n + g.t];
    }
}
template <int D>
__device__ __forceinline__ void sys_copy(const double* src, double* dst, const SysGeo& g)
{
    if (g.active) {
#pragma unroll
        for (int d = 0; d < D; ++d) dst[d * g.n + g.t] = src[d * g.n + g.t];
    }
}
// sum of squares of (x - b) over the line, in a fixed order; valid in thread 0
template <int D>
__device__ __forceinline__ double sys_sqdiff(const double (&x)[D], const double* b, const SysGeo& g,
                                             const SysSmem<D>& sm)
{
    double s = 0.0;
    if (g.active) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double e = x[d] - b[d * g.n + g.t];
            s = fma(e, e, s);
        }
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sm.wred[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (g.npad >> 6); ++w) tot += sm.wred[w];
    }
    return tot;
}

// One chunk of one line per workgroup: the roles of sweep_body_t (SweepArgs)
// for a system; a.nx is the line length D n in memory
template <int SYS, int K, int ST, bool ROE, int END>
__device__ __forceinline__ void sys_body(const SweepArgs& a, const int c)
{
    constexpr int D = Phys<SYS>::D;
    if (a.flag != nullptr && *a.flag != 0) return;
    extern __shared__ double smem_raw[];
    SysGeo g;
    g.init(a.nx / D);
    SysSmem<D> sm;
    sm.init(smem_raw, g.npad);
    int par = 0;
    const int64_t nx = a.nx;

    const double* src = (a.side_in != nullptr && c > 0) ? a.side_in + (int64_t)c * nx
                                                        : a.ustart + (int64_t)c * a.ustart_stride * nx;
    double x[D];
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = 0.0;
    sys_load(x, src, g);
    wait_loads();  // (as in sweep_body_t)
    if (a.ucommit != nullptr) sys_store(x, a.ucommit + (int64_t)c * a.ucommit_stride * nx, g);
    if (a.inject_last && c == a.nchunks - 1) {
        const double* last = (a.side_in != nullptr) ? a.side_in + (int64_t)a.nchunks * nx
                                                    : a.ustart + (int64_t)a.nchunks * a.ustart_stride * nx;
        sys_copy<D>(last, a.ucommit + (int64_t)a.nchunks * a.ucommit_stride * nx, g);
    }
    const double* cstart = (a.ystart != nullptr) ? a.ystart + (int64_t)c * a.ystart_stride * nx : src;
    if (END == END_RESTRICT && c == 0) {
        sys_copy<D>(cstart, a.uc_out, g);
        sys_copy<D>(a.g != nullptr ? a.g : cstart, a.gc_out, g);
    }

    const int64_t n0 = (int64_t)c * a.m;
    for (int j = 1; j <= a.nsteps; ++j) {
        phi_sys<SYS, K, ST, ROE>(x, a.dt, g, sm, a.pc, par);
        if (a.g != nullptr) sys_add(x, a.g + (n0 + j) * nx, g);
        if (a.fout != nullptr) {
            if (a.fout_every <= 1) sys_store(x, a.fout + (n0 + j) * nx, g);
            else if ((n0 + j) % a.fout_every == 0) sys_store(x, a.fout + ((n0 + j) / a.fout_every) * nx, g);
        }
    }

    if constexpr (END == END_NONE) return;
    if constexpr (END == END_PHI) {
        phi_sys<SYS, K, ST, ROE>(x, a.dt, g, sm, a.pc, par);
        if (a.gc_sub != nullptr) {
            double* out = a.gc_sub + (int64_t)(c + 1) * nx;
            if (g.active) {
#pragma unroll
                for (int d = 0; d < D; ++d) out[d * g.n + g.t] = out[d * g.n + g.t] - x[d];
            }
            return;
        }
        sys_store(x, a.side_out + (int64_t)c * nx, g);
        return;
    }
    const int64_t n1 = n0 + a.m;
    phi_sys<SYS, K, ST, ROE>(x, a.dt, g, sm, a.pc, par);
    if (a.g != nullptr) sys_add(x, a.g + n1 * nx, g);
    const double* cnext = a.cref + (int64_t)(c + 1) * a.cref_stride * nx;
    if (a.resid_partial != nullptr) {
        const double s = sys_sqdiff(x, cnext, g, sm);
        if (threadIdx.x == 0) a.resid_partial[c] = s;
    }
    if (a.r_out != nullptr && g.active) {
#pragma unroll
        for (int d = 0; d < D; ++d) a.r_out[(int64_t)c * nx + d * g.n + g.t] = x[d] - cnext[d * g.n + g.t];
    }
    if constexpr (END == END_CSTEP) {
        if (a.side_out != nullptr) sys_store(x, a.side_out + (int64_t)(c + 1) * nx, g);
        return;
    }
    if (a.coarse_injection) sys_copy<D>(cnext, a.uc_out + (int64_t)(c + 1) * nx, g);
    else sys_store(x, a.uc_out + (int64_t)(c + 1) * nx, g);
    if (a.coarse_split) {
        sys_store(x, a.gc_out + (int64_t)(c + 1) * nx, g);
        return;
    }
    double y[D];
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = 0.0;
    sys_load(y, cstart, g);
    PhiConst pcn = a.pc;
    if (a.alpha_next > 0.0) pcn.alpha_fixed = a.alpha_next;
    phi_sys<SYS, K, ST, ROE>(y, a.dt_next, g, sm, pcn, par);
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = x[d] - y[d];
    sys_store(y, a.gc_out + (int64_t)(c + 1) * nx, g);
}

template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_relax_f_kernel(SweepArgs a)
{
    sys_body<SYS, K, ST, ROE, END_NONE>(a, blockIdx.x);
}
template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_relax_fc_kernel(SweepArgs a)
{
    sys_body<SYS, K, ST, ROE, END_CSTEP>(a, blockIdx.x);
}
template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_relax_fr_kernel(SweepArgs a)
{
    sys_body<SYS, K, ST, ROE, END_RESTRICT>(a, blockIdx.x);
}
template <int SYS, int K, int ST, bool ROE>
__global__ __launch_bounds__(512) void sys_phi_kernel(SweepArgs a)
{
    sys_body<SYS, K, ST, ROE, END_PHI>(a, blockIdx.x);
}

template <int SYS, int K, int ST, bool ROE>
static hipError_t launch_sys_f(const SweepArgs& a, int threads, hipStream_t s)
{
    const size_t shmem = sys_smem_bytes(Phys<SYS>::D, threads);
    auto go = [&](auto fn) -> hipError_t {
        if (shmem > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(fn, dim3(a.nchunks), dim3(threads), shmem, s, a);
        return hipGetLastError();
    };
    switch (a.end_mode) {
    case END_NONE: return go(sys_relax_f_kernel<SYS, K, ST, ROE>);
    case END_CSTEP: return go(sys_relax_fc_kernel<SYS, K, ST, ROE>);
    case END_RESTRICT: return go(sys_relax_fr_kernel<SYS, K, ST, ROE>);
    case END_PHI: return go(sys_phi_kernel<SYS, K, ST, ROE>);
    default: return hipErrorInvalidValue;
    }
}

// threads: a multiple of 64 covering the line's cells, at most 512 (so that the
// kernels keep up to 256 VGPRs: the Euler WENO7 stage needs about 140)
template <int SYS, int K>
hipError_t launch_sys_sk(const SweepArgs& a, int threads, int stepper, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
    if (threads < 64 || threads > 512 || threads % 64 != 0 || a.nx / Phys<SYS>::D > threads)
        return hipErrorInvalidValue;
    const bool roe = a.pc.roe != 0;
    if (stepper == 1) return roe ? launch_sys_f<SYS, K, 1, true>(a, threads, s) : launch_sys_f<SYS, K, 1, false>(a, threads, s);
    if (stepper == 2) return roe ? launch_sys_f<SYS, K, 2, true>(a, threads, s) : launch_sys_f<SYS, K, 2, false>(a, threads, s);
    return roe ? launch_sys_f<SYS, K, 3, true>(a, threads, s) : launch_sys_f<SYS, K, 3, false>(a, threads, s);
}

}  // namespace mgk
