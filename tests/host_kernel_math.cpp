// Host build of the per-cell arithmetic of the GPU sweep kernels
// (paper_2104_09404_amd/csrc/cell_math.h), assembled into one line operator
// and one step in the same order as the kernels, for a CPU test against the
// reference oracle.
#include <math.h>
#include <stdlib.h>

#include "../paper_2104_09404_amd/csrc/cell_math.h"

using namespace mgk;

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

extern "C" void hk_recon(const double* w, double eps, double* um, double* up)
{
    const double Em = weno5_e(w[0], w[1], w[2], eps);
    const double E0 = weno5_e(w[1], w[2], w[3], eps);
    const double Ep = weno5_e(w[2], w[3], w[4], eps);
    weno5_cell(w[0], w[1], w[2], w[3], w[4], Em, E0, Ep, *um, *up);
}

// A(u) for one periodic line; returns alpha
extern "C" double hk_operator(int nx, const double* u, int k, double fa, double fb, double inv_dx, double eps,
                              double alpha_fixed, double* A)
{
    double* um = (double*)malloc(sizeof(double) * nx);
    double* up = (double*)malloc(sizeof(double) * nx);
    double* F = (double*)malloc(sizeof(double) * nx);
    double lmax = 0.0;
    for (int i = 0; i < nx; ++i) {
        if (k == 0) {
            um[i] = up[i] = u[i];
        } else {
            double w[5];
            for (int j = 0; j < 5; ++j) w[j] = u[wrap(i - 2 + j, nx)];
            const double Em = weno5_e(u[wrap(i - 2, nx)], u[wrap(i - 1, nx)], u[i], eps);
            const double E0 = weno5_e(u[wrap(i - 1, nx)], u[i], u[wrap(i + 1, nx)], eps);
            const double Ep = weno5_e(u[i], u[wrap(i + 1, nx)], u[wrap(i + 2, nx)], eps);
            weno5_cell(w[0], w[1], w[2], w[3], w[4], Em, E0, Ep, um[i], up[i]);
        }
        lmax = fmax(lmax, fmax(fabs(um[i]), fabs(up[i])));
    }
    const double alpha = alpha_fixed > 0.0 ? alpha_fixed : lf_alpha(lmax, fa, fb);
    // F[i] = twice the flux at the left face of cell i: u^- from cell i-1, u^+ from cell i
    for (int i = 0; i < nx; ++i) F[i] = lf_flux2(um[wrap(i - 1, nx)], up[i], fa, fb, alpha);
    for (int i = 0; i < nx; ++i) A[i] = (F[i] - F[wrap(i + 1, nx)]) * (0.5 * inv_dx);
    free(um);
    free(up);
    free(F);
    return alpha;
}

extern "C" void hk_phi(int nx, const double* u, int k, int stepper, double fa, double fb, double inv_dx, double eps,
                       double alpha_fixed, double dt, double* out)
{
    double* A = (double*)malloc(sizeof(double) * nx);
    double* v = (double*)malloc(sizeof(double) * nx);
    hk_operator(nx, u, k, fa, fb, inv_dx, eps, alpha_fixed, A);
    for (int i = 0; i < nx; ++i) v[i] = rk_first(u[i], A[i], dt);
    if (stepper == 1) {
        for (int i = 0; i < nx; ++i) out[i] = v[i];
    } else if (stepper == 2) {
        hk_operator(nx, v, k, fa, fb, inv_dx, eps, alpha_fixed, A);
        for (int i = 0; i < nx; ++i) out[i] = rk2_second(u[i], v[i], A[i], 0.5 * dt);
    } else {
        hk_operator(nx, v, k, fa, fb, inv_dx, eps, alpha_fixed, A);
        for (int i = 0; i < nx; ++i) v[i] = rk3_second(u[i], v[i], A[i], 0.25 * dt);
        hk_operator(nx, v, k, fa, fb, inv_dx, eps, alpha_fixed, A);
        for (int i = 0; i < nx; ++i) out[i] = rk3_third(u[i], v[i], A[i], (2.0 / 3.0) * dt);
    }
    free(A);
    free(v);
}

extern "C" void hk_recon_vjp(const double* w, double eps, double umb, double upb, double* wb)
{
    for (int j = 0; j < 5; ++j) wb[j] = 0.0;
    weno5_cell_vjp(w[0], w[1], w[2], w[3], w[4], eps, umb, upb, wb);
}

// WENO3 / WENO7 reconstructions of the middle cell of a window of 2k+1 cells
extern "C" void hk_recon_k(int k, const double* w, double eps, double* um, double* up)
{
    if (k == 1) weno3_cell(w[0], w[1], w[2], eps, *um, *up);
    else weno7_cell(w[0], w[1], w[2], w[3], w[4], w[5], w[6], eps, *um, *up);
}

// the Roe flux with the Harten-Hyman fix (the kernels' twice-the-flux form, halved)
extern "C" double hk_roe(double uL, double uR, double fa, double fb) { return 0.5 * roe_flux2(uL, uR, fa, fb); }
