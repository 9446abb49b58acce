// cell_math.h -- per-cell arithmetic of the sweep kernels (WENO reconstructions
// of orders 3, 5 and 7, Lax-Friedrichs and Roe fluxes), written once and
// compiled for the GPU by the kernels and for the host by the CPU test of the
// kernel arithmetic.
#pragma once
#include <math.h>

#ifdef __HIPCC__
#define MGK_HD __host__ __device__ __forceinline__
#else
#define MGK_HD inline
#endif

namespace mgk {

// 13/12 (a - 2b + c)^2 + eps: the second-difference part of the smoothness
// indicator of the stencil centred on b (shared by neighbouring cells), with
// the eps of eq omega folded in
MGK_HD double weno5_e(double a, double b, double c, double eps)
{
    const double d2 = fma(-2.0, b, a + c);
    return fma((13.0 / 12.0) * d2, d2, eps);
}

// 1/x for x > 0 in the normal range: hardware reciprocal estimate refined by
// two Newton steps (the host build of this header starts from 1/x itself)
MGK_HD double recip(double x)
{
#ifdef __HIP_DEVICE_COMPILE__
    double r = __builtin_amdgcn_rcp(x);
#else
    double r = 1.0 / x;
#endif
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// WENO5-JS reconstructions of cell p from its window w0..w4 = u_{p-2}..u_{p+2}
// (sec 2.1.1, eq C, B, omega, D; stencil r = cells {p-r, ..., p-r+2}):
//   um = u^-_{p+1/2} (right face), up = u^+_{p-1/2} (left face, mirror image).
// Em, E0, Ep are weno5_e centred on p-1, p, p+1 (eps included).
//
// Smoothness indicators in the Jiang-Shu form of the printed B_r (the integral
// is over the reconstruction cell p, so the first-derivative term depends on
// where p sits in the stencil):
//   bL (cells p-2..p)   = 13/12 D2_{p-1}^2 + ((w0 - 4 w1 + 3 w2)/2)^2
//   bC (cells p-1..p+1) = 13/12 D2_p^2     + ((w3 - w1)/2)^2
//   bR (cells p..p+2)   = 13/12 D2_{p+1}^2 + ((3 w2 - 4 w3 + w4)/2)^2
// The mirror image reconstructs from the same three cell sets, so both faces
// share bL, bC, bR.  With s_r = (eps + b_r)^2, alpha_r = d_r / s_r; multiplying
// the numerator and denominator of sum(alpha_r q_r) / sum(alpha_r) by
// sL sC sR removes the divisions by s_r, and both faces share one reciprocal
// of the product of their denominators.  Linear weights: u^- takes 3/10 on
// cells p..p+2, 6/10 centred, 1/10 on p-2..p; u^+ the mirror (1/10, 6/10,
// 3/10).  The candidate values of eq C carry their linear weight d_r and the
// 1/6 of the printed c table.
MGK_HD void weno5_cell(double w0, double w1, double w2, double w3, double w4, double Em, double E0, double Ep,
                       double& um, double& up)
{
    const double b = fma(1.5, w2, fma(-2.0, w1, 0.5 * w0));
    const double d = 0.5 * (w3 - w1);
    const double e = fma(1.5, w2, fma(-2.0, w3, 0.5 * w4));
    double sL = fma(b, b, Em);
    double sC = fma(d, d, E0);
    double sR = fma(e, e, Ep);
    sL *= sL;
    sC *= sC;
    sR *= sR;
    const double PLC = sL * sC, PLR = sL * sR, PCR = sC * sR;
    const double h1 = 0.1 * w2, h5 = 0.5 * w2, h11 = (11.0 / 60.0) * w2;
    // u^-_{p+1/2}: 3/10 (2w2 + 5w3 - w4)/6, 6/10 (-w1 + 5w2 + 2w3)/6, 1/10 (2w0 - 7w1 + 11w2)/6
    const double cR = fma(-0.05, w4, fma(0.25, w3, h1));
    const double cC = fma(0.2, w3, fma(-0.1, w1, h5));
    const double cL = fma(2.0 / 60.0, w0, fma(-7.0 / 60.0, w1, h11));
    // u^+_{p-1/2}: 1/10 (11w2 - 7w3 + 2w4)/6, 6/10 (2w1 + 5w2 - w3)/6, 3/10 (-w0 + 5w1 + 2w2)/6
    const double dR = fma(2.0 / 60.0, w4, fma(-7.0 / 60.0, w3, h11));
    const double dC = fma(0.2, w1, fma(-0.1, w3, h5));
    const double dL = fma(-0.05, w0, fma(0.25, w1, h1));
    const double nm = fma(PCR, cL, fma(PLR, cC, PLC * cR));
    const double dm = fma(0.1, PCR, fma(0.6, PLR, 0.3 * PLC));
    const double np = fma(PCR, dL, fma(PLR, dC, PLC * dR));
    const double dp = fma(0.3, PCR, fma(0.6, PLR, 0.1 * PLC));
    const double inv = recip(dm * dp);
    um = nm * (dp * inv);
    up = np * (dm * inv);
}

// WENO3 (k = 1) reconstructions of cell p from w0, w1, w2 = u_{p-1}, u_p, u_{p+1}
// (sec 2.1.1 with two 2-cell stencils):
//   u^-_{p+1/2}: (w1 + w2)/2 with weight 2/3 and indicator (w2 - w1)^2,
//                (3 w1 - w0)/2 with weight 1/3 and indicator (w1 - w0)^2;
//   u^+_{p-1/2}: the mirror image, (w0 + w1)/2 (2/3, (w1 - w0)^2) and
//                (3 w1 - w2)/2 (1/3, (w2 - w1)^2).
// With s = (eps + beta)^2 the weights reduce to u^- = (2 sL cR + sR cL)/(2 sL + sR)
// (sR of the right stencil, sL of the left one) and u^+ likewise; both faces
// share one reciprocal.
MGK_HD void weno3_cell(double w0, double w1, double w2, double eps, double& um, double& up)
{
    const double dl = w1 - w0, dr = w2 - w1;
    double sL = fma(dl, dl, eps), sR = fma(dr, dr, eps);
    sL *= sL;
    sR *= sR;
    const double cR = 0.5 * (w1 + w2), cL = fma(1.5, w1, -0.5 * w0);
    const double pL = 0.5 * (w0 + w1), pR = fma(1.5, w1, -0.5 * w2);
    const double nm = fma(2.0 * sL, cR, sR * cL), dm = fma(2.0, sL, sR);
    const double np = fma(2.0 * sR, pL, sL * pR), dp = fma(2.0, sR, sL);
    const double inv = recip(dm * dp);
    um = nm * (dp * inv);
    up = np * (dm * inv);
}

// WENO7 (k = 3) reconstructions of cell p from w0..w6 = u_{p-3}..u_{p+3}
// (sec 2.1.1 with four 4-cell stencils; stencil r = cells p-r..p-r+3).
// Candidates of u^-_{p+1/2} (times 12) and linear weights (times 35):
//   r = 0 (w3..w6):  3 w3 + 13 w4 -  5 w5 +  1 w6      4
//   r = 1 (w2..w5): -1 w2 +  7 w3 +  7 w4 -  1 w5     18
//   r = 2 (w1..w4):  1 w1 -  5 w2 + 13 w3 +  3 w4     12
//   r = 3 (w0..w3): -3 w0 + 13 w1 - 23 w2 + 25 w3      1
// Indicators (times 240) of the stencils on cells a, b, c, d (left to right):
//   r = 3: a(547a - 3882b + 4642c - 1854d) + b(7043b - 17246c + 7042d) + c(11003c - 9402d) + 2107d^2
//   r = 2: a(267a - 1642b + 1602c - 494d) + b(2843b - 5966c + 1922d) + c(3443c - 2522d) + 547d^2
//   r = 1: a(547a - 2522b + 1922c - 494d) + b(3443b - 5966c + 1602d) + c(2843c - 1642d) + 267d^2
//   r = 0: a(2107a - 9402b + 7042c - 1854d) + b(11003b - 17246c + 4642d) + c(7043c - 3882d) + 547d^2
// u^+_{p-1/2} is the mirror image: its stencil r covers the cells of u^-'s
// stencil 3-r (same indicator) with the candidate coefficients reversed.
// With s_r = (eps + beta_r)^2 the weights d_r/s_r are scaled by s0 s1 s2 s3, so
// each face needs products of three s and both share one reciprocal.
MGK_HD void weno7_cell(double w0, double w1, double w2, double w3, double w4, double w5, double w6, double eps,
                       double& um, double& up)
{
    // indicators, Horner-nested with explicit fused multiply-adds (the kernels
    // are compiled without contraction)
    const double b3 = fma(w0, fma(547.0, w0, fma(-3882.0, w1, fma(4642.0, w2, -1854.0 * w3))),
                          fma(w1, fma(7043.0, w1, fma(-17246.0, w2, 7042.0 * w3)),
                              fma(w2, fma(11003.0, w2, -9402.0 * w3), (2107.0 * w3) * w3)));
    const double b2 = fma(w1, fma(267.0, w1, fma(-1642.0, w2, fma(1602.0, w3, -494.0 * w4))),
                          fma(w2, fma(2843.0, w2, fma(-5966.0, w3, 1922.0 * w4)),
                              fma(w3, fma(3443.0, w3, -2522.0 * w4), (547.0 * w4) * w4)));
    const double b1 = fma(w2, fma(547.0, w2, fma(-2522.0, w3, fma(1922.0, w4, -494.0 * w5))),
                          fma(w3, fma(3443.0, w3, fma(-5966.0, w4, 1602.0 * w5)),
                              fma(w4, fma(2843.0, w4, -1642.0 * w5), (267.0 * w5) * w5)));
    const double b0 = fma(w3, fma(2107.0, w3, fma(-9402.0, w4, fma(7042.0, w5, -1854.0 * w6))),
                          fma(w4, fma(11003.0, w4, fma(-17246.0, w5, 4642.0 * w6)),
                              fma(w5, fma(7043.0, w5, -3882.0 * w6), (547.0 * w6) * w6)));
    const double i240 = 1.0 / 240.0;
    double s0 = fma(b0, i240, eps), s1 = fma(b1, i240, eps), s2 = fma(b2, i240, eps), s3 = fma(b3, i240, eps);
    s0 *= s0;
    s1 *= s1;
    s2 *= s2;
    s3 *= s3;
    const double s01 = s0 * s1, s23 = s2 * s3;
    const double P0 = s1 * s23, P1 = s0 * s23, P2 = s01 * s3, P3 = s01 * s2;  // products of the other three
    // u^-: candidate r (coefficients over 12) with weight d_r on P_r
    const double c0 = fma(3.0 / 12.0, w3, fma(13.0 / 12.0, w4, fma(-5.0 / 12.0, w5, w6 * (1.0 / 12.0))));
    const double c1 = fma(-1.0 / 12.0, w2, fma(7.0 / 12.0, w3, fma(7.0 / 12.0, w4, w5 * (-1.0 / 12.0))));
    const double c2 = fma(1.0 / 12.0, w1, fma(-5.0 / 12.0, w2, fma(13.0 / 12.0, w3, w4 * (3.0 / 12.0))));
    const double c3 = fma(-3.0 / 12.0, w0, fma(13.0 / 12.0, w1, fma(-23.0 / 12.0, w2, w3 * (25.0 / 12.0))));
    // u^+: mirror stencil r covers u^-'s stencil 3-r, weight d_r on P_{3-r}
    const double e0 = fma(3.0 / 12.0, w3, fma(13.0 / 12.0, w2, fma(-5.0 / 12.0, w1, w0 * (1.0 / 12.0))));
    const double e1 = fma(-1.0 / 12.0, w4, fma(7.0 / 12.0, w3, fma(7.0 / 12.0, w2, w1 * (-1.0 / 12.0))));
    const double e2 = fma(1.0 / 12.0, w5, fma(-5.0 / 12.0, w4, fma(13.0 / 12.0, w3, w2 * (3.0 / 12.0))));
    const double e3 = fma(-3.0 / 12.0, w6, fma(13.0 / 12.0, w5, fma(-23.0 / 12.0, w4, w3 * (25.0 / 12.0))));
    const double q0 = 4.0 * P0, q1 = 18.0 * P1, q2 = 12.0 * P2, q3 = P3;
    const double r0 = 4.0 * P3, r1 = 18.0 * P2, r2 = 12.0 * P1, r3 = P0;
    const double nm = fma(q0, c0, fma(q1, c1, fma(q2, c2, q3 * c3)));
    const double dm = (q0 + q1) + (q2 + q3);
    const double np = fma(r0, e0, fma(r1, e1, fma(r2, e2, r3 * e3)));
    const double dp = (r0 + r1) + (r2 + r3);
    const double inv = recip(dm * dp);
    um = nm * (dp * inv);
    up = np * (dm * inv);
}

// Reverse mode of weno5_cell.  The forward intermediates (including the three
// second-difference terms, from the window itself) are recomputed; adj(um, up,
// um_bar, up_bar) receives the two reconstructions and returns their adjoints,
// and the adjoint of the window w0..w4 is accumulated into wb[0..4].
template <class Adj>
MGK_HD void weno5_cell_vjp_f(double w0, double w1, double w2, double w3, double w4, double eps, Adj&& adj, double* wb)
{
    // forward
    const double d2m = fma(-2.0, w1, w0 + w2);
    const double d2c = fma(-2.0, w2, w1 + w3);
    const double d2p = fma(-2.0, w3, w2 + w4);
    const double Em = fma((13.0 / 12.0) * d2m, d2m, eps);
    const double E0 = fma((13.0 / 12.0) * d2c, d2c, eps);
    const double Ep = fma((13.0 / 12.0) * d2p, d2p, eps);
    const double b = fma(1.5, w2, fma(-2.0, w1, 0.5 * w0));
    const double d = 0.5 * (w3 - w1);
    const double e = fma(1.5, w2, fma(-2.0, w3, 0.5 * w4));
    const double tL = fma(b, b, Em), tC = fma(d, d, E0), tR = fma(e, e, Ep);
    const double sL = tL * tL, sC = tC * tC, sR = tR * tR;
    const double PLC = sL * sC, PLR = sL * sR, PCR = sC * sR;
    const double h1 = 0.1 * w2, h5 = 0.5 * w2, h11 = (11.0 / 60.0) * w2;
    const double cR = fma(-0.05, w4, fma(0.25, w3, h1));
    const double cC = fma(0.2, w3, fma(-0.1, w1, h5));
    const double cL = fma(2.0 / 60.0, w0, fma(-7.0 / 60.0, w1, h11));
    const double dR = fma(2.0 / 60.0, w4, fma(-7.0 / 60.0, w3, h11));
    const double dC = fma(0.2, w1, fma(-0.1, w3, h5));
    const double dL = fma(-0.05, w0, fma(0.25, w1, h1));
    const double nm = fma(PCR, cL, fma(PLR, cC, PLC * cR));
    const double dm = fma(0.1, PCR, fma(0.6, PLR, 0.3 * PLC));
    const double np = fma(PCR, dL, fma(PLR, dC, PLC * dR));
    const double dp = fma(0.3, PCR, fma(0.6, PLR, 0.1 * PLC));
    const double inv = recip(dm * dp);
    const double idm = dp * inv, idp = dm * inv;  // 1/dm, 1/dp
    const double um = nm * idm, up = np * idp;
    double um_bar, up_bar;
    adj(um, up, um_bar, up_bar);
    // reverse: um = nm/dm, up = np/dp
    const double nmb = um_bar * idm, dmb = -um_bar * um * idm;
    const double npb = up_bar * idp, dpb = -up_bar * up * idp;
    const double PLCb = fma(nmb, cR, fma(0.3, dmb, fma(npb, dR, 0.1 * dpb)));
    const double PLRb = fma(nmb, cC, fma(0.6, dmb, fma(npb, dC, 0.6 * dpb)));
    const double PCRb = fma(nmb, cL, fma(0.1, dmb, fma(npb, dL, 0.3 * dpb)));
    const double cRb = nmb * PLC, cCb = nmb * PLR, cLb = nmb * PCR;
    const double dRb = npb * PLC, dCb = npb * PLR, dLb = npb * PCR;
    const double sLb = fma(PLCb, sC, PLRb * sR);
    const double sCb = fma(PLCb, sL, PCRb * sR);
    const double sRb = fma(PLRb, sL, PCRb * sC);
    const double tLb = 2.0 * tL * sLb, tCb = 2.0 * tC * sCb, tRb = 2.0 * tR * sRb;
    const double bb = 2.0 * b * tLb, db = 2.0 * d * tCb, eb = 2.0 * e * tRb;
    // second differences: E = 13/12 d2^2 + eps, d2 = a - 2b + c
    const double d2mb = (2.0 * 13.0 / 12.0) * d2m * tLb;
    const double d2cb = (2.0 * 13.0 / 12.0) * d2c * tCb;
    const double d2pb = (2.0 * 13.0 / 12.0) * d2p * tRb;
    wb[0] += 0.5 * bb + (2.0 / 60.0) * cLb - 0.05 * dLb + d2mb;
    wb[1] += -2.0 * bb - 0.5 * db - 0.1 * cCb - (7.0 / 60.0) * cLb + 0.2 * dCb + 0.25 * dLb - 2.0 * d2mb + d2cb;
    wb[2] += 1.5 * bb + 1.5 * eb + 0.1 * cRb + 0.5 * cCb + (11.0 / 60.0) * (cLb + dRb) + 0.5 * dCb + 0.1 * dLb + d2mb -
             2.0 * d2cb + d2pb;
    wb[3] += 0.5 * db - 2.0 * eb + 0.25 * cRb + 0.2 * cCb - (7.0 / 60.0) * dRb - 0.1 * dCb + d2cb - 2.0 * d2pb;
    wb[4] += 0.5 * eb - 0.05 * cRb + (2.0 / 60.0) * dRb + d2pb;
}

// Reverse mode of weno5_cell for given adjoints of the two reconstructions.
MGK_HD void weno5_cell_vjp(double w0, double w1, double w2, double w3, double w4, double eps, double um_bar,
                           double up_bar, double* wb)
{
    weno5_cell_vjp_f(
        w0, w1, w2, w3, w4, eps,
        [&](double, double, double& umb, double& upb) {
            umb = um_bar;
            upb = up_bar;
        },
        wb);
}

// f'(u) = 2 fa u + fb
MGK_HD double flux_fprime(double u, double fa, double fb) { return fma(2.0 * fa, u, fb); }

// f(u) = u (fa u + fb): Burgers (fa = 1/2, fb = 0) or advection (fa = 0, fb = a)
MGK_HD double flux_f(double u, double fa, double fb) { return u * fma(fa, u, fb); }

// Twice the Lax-Friedrichs flux of eq LFflux: f(uL) + f(uR) - alpha (uR - uL)
MGK_HD double lf_flux2(double uL, double uR, double fa, double fb, double alpha)
{
    return fma(-alpha, uR - uL, flux_f(uL, fa, fb) + flux_f(uR, fa, fb));
}

// Twice the Roe flux with the Harten-Hyman entropy fix (sec 2.1.3, eq roeflux,
// with the 1/2 on the dissipation and q_H = (lh^2/delta + delta)/2 inside the
// fix) for f(u) = u (fa u + fb):
//   lambda(u) = 2 fa u + fb, Roe speed lh = (f(uR) - f(uL))/(uR - uL) = fa (uL + uR) + fb
//   (for Burgers the eigenvalue at the average (uL + uR)/2; for advection a),
//   delta = max(0, lh - lambda(uL), lambda(uR) - lh),
//   2F = f(uL) + f(uR) - q_H(lh) (uR - uL).
MGK_HD double roe_flux2(double uL, double uR, double fa, double fb)
{
    const double lh = fma(fa, uL + uR, fb);
    const double lL = fma(2.0 * fa, uL, fb), lR = fma(2.0 * fa, uR, fb);
    const double delta = fmax(0.0, fmax(lh - lL, lR - lh));
    const double alh = fabs(lh);
    const double q = (alh < delta) ? 0.5 * (lh * lh / delta + delta) : alh;
    return fma(-q, uR - uL, flux_f(uL, fa, fb) + flux_f(uR, fa, fb));
}

// alpha_LF = max |lambda(u^{+-})| from m = max |u^{+-}|: with lambda = 2 fa u + fb
// and one of fa, fb zero (Burgers or advection) it is 2|fa| m + |fb|
MGK_HD double lf_alpha(double m, double fa, double fb) { return fma(2.0 * fabs(fa), m, fabs(fb)); }

// Stage combinations of eq SSPRK1/2/3 (Shu-Osher form), x = u^n, v = the
// previous stage, A = A(v):
//   first stage (all):  x + dt A
//   SSPRK2 second:      x/2 + v/2 + (dt/2) A           (hdt = dt/2)
//   SSPRK3 second:      3x/4 + v/4 + (dt/4) A          (qdt = dt/4)
//   SSPRK3 third:       x/3 + 2v/3 + (2dt/3) A         (tdt = 2dt/3)
MGK_HD double rk_first(double x, double A, double dt) { return fma(dt, A, x); }
MGK_HD double rk2_second(double x, double v, double A, double hdt) { return fma(hdt, A, fma(0.5, v, 0.5 * x)); }
MGK_HD double rk3_second(double x, double v, double A, double qdt) { return fma(qdt, A, fma(0.25, v, 0.75 * x)); }
MGK_HD double rk3_third(double x, double v, double A, double tdt)
{
    return fma(tdt, A, fma(2.0 / 3.0, v, (1.0 / 3.0) * x));
}

}  // namespace mgk
