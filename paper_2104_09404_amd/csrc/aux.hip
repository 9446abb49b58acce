// aux.hip -- small auxiliary kernels (initial fill, residual norms, flags)
// and the dispatch of sweep launches to the per-scheme translation units.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sweep.h"

namespace mgk {

template <int K, int ST>
hipError_t launch_sweep_ks(const SweepArgs& a, const KernelCfg& cfg, hipStream_t s);

template <int K, int ST>
hipError_t launch_adjoint_ks(const AdjArgs& a, const KernelCfg& cfg, int store_mode, hipStream_t s);

hipError_t launch_adjoint(const AdjArgs& a, const KernelCfg& cfg, int k, int stepper, int store_mode, hipStream_t s)
{
    if (a.nlines <= 0) return hipSuccess;
    if (k == 0) {
        if (stepper == 1) return launch_adjoint_ks<0, 1>(a, cfg, store_mode, s);
        if (stepper == 2) return launch_adjoint_ks<0, 2>(a, cfg, store_mode, s);
        return launch_adjoint_ks<0, 3>(a, cfg, store_mode, s);
    }
    if (stepper == 1) return launch_adjoint_ks<2, 1>(a, cfg, store_mode, s);
    if (stepper == 2) return launch_adjoint_ks<2, 2>(a, cfg, store_mode, s);
    return launch_adjoint_ks<2, 3>(a, cfg, store_mode, s);
}

// (k, stepper) -> the instantiation compiled in sweep_k<k>_s<stepper>.hip
#define MGK_DISPATCH_KS(FN, K, ...)                                   \
    do {                                                              \
        if (stepper == 1) return FN<K, 1>(__VA_ARGS__);               \
        if (stepper == 2) return FN<K, 2>(__VA_ARGS__);               \
        return FN<K, 3>(__VA_ARGS__);                                 \
    } while (0)

hipError_t launch_sweep(const SweepArgs& a, const KernelCfg& cfg, int k, int stepper, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
    switch (k) {
    case 0: MGK_DISPATCH_KS(launch_sweep_ks, 0, a, cfg, s);
    case 1: MGK_DISPATCH_KS(launch_sweep_ks, 1, a, cfg, s);
    case 2: MGK_DISPATCH_KS(launch_sweep_ks, 2, a, cfg, s);
    case 3: MGK_DISPATCH_KS(launch_sweep_ks, 3, a, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

template <int K, int ST>
hipError_t launch_tiled_ks(const SweepArgs& a, const KernelCfg& cfg, hipStream_t s);

template <int K, int ST>
hipError_t launch_tiled_adjoint_ks(const AdjArgs& a, const KernelCfg& cfg, int store_mode, hipStream_t s);

hipError_t launch_tiled_adjoint(const AdjArgs& a, const KernelCfg& cfg, int k, int stepper, int store_mode,
                                hipStream_t s)
{
    if (a.nlines <= 0) return hipSuccess;
    if (k == 0) {
        if (stepper == 1) return launch_tiled_adjoint_ks<0, 1>(a, cfg, store_mode, s);
        if (stepper == 2) return launch_tiled_adjoint_ks<0, 2>(a, cfg, store_mode, s);
        return launch_tiled_adjoint_ks<0, 3>(a, cfg, store_mode, s);
    }
    if (stepper == 1) return launch_tiled_adjoint_ks<2, 1>(a, cfg, store_mode, s);
    if (stepper == 2) return launch_tiled_adjoint_ks<2, 2>(a, cfg, store_mode, s);
    return launch_tiled_adjoint_ks<2, 3>(a, cfg, store_mode, s);
}

template <int SYS, int K>
hipError_t launch_sys_sk(const SweepArgs& a, int threads, int stepper, hipStream_t s);

hipError_t launch_sys(const SweepArgs& a, int threads, int flux, int k, int stepper, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
#define MGK_SYS_K(SYS)                                                  \
    switch (k) {                                                        \
    case 0: return launch_sys_sk<SYS, 0>(a, threads, stepper, s);       \
    case 1: return launch_sys_sk<SYS, 1>(a, threads, stepper, s);       \
    case 2: return launch_sys_sk<SYS, 2>(a, threads, stepper, s);       \
    case 3: return launch_sys_sk<SYS, 3>(a, threads, stepper, s);       \
    default: return hipErrorInvalidValue;                               \
    }
    if (flux == 2) { MGK_SYS_K(2) }
    if (flux == 3) { MGK_SYS_K(3) }
#undef MGK_SYS_K
    return hipErrorInvalidValue;
}

template <int SYS, int K>
hipError_t launch_sys_tiled_sk(const SweepArgs& a, int threads, int stepper, hipStream_t s);

hipError_t launch_sys_tiled(const SweepArgs& a, int threads, int flux, int k, int stepper, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
#define MGK_SYS_K(SYS)                                                        \
    switch (k) {                                                              \
    case 0: return launch_sys_tiled_sk<SYS, 0>(a, threads, stepper, s);       \
    case 1: return launch_sys_tiled_sk<SYS, 1>(a, threads, stepper, s);       \
    case 2: return launch_sys_tiled_sk<SYS, 2>(a, threads, stepper, s);       \
    case 3: return launch_sys_tiled_sk<SYS, 3>(a, threads, stepper, s);       \
    default: return hipErrorInvalidValue;                                     \
    }
    if (flux == 2) { MGK_SYS_K(2) }
    if (flux == 3) { MGK_SYS_K(3) }
#undef MGK_SYS_K
    return hipErrorInvalidValue;
}

// split lines: WENO degree 0 .. 3 (3 or 4 ghost cells per side)
hipError_t launch_tiled(const SweepArgs& a, const KernelCfg& cfg, int k, int stepper, hipStream_t s)
{
    if (a.nchunks <= 0) return hipSuccess;
    switch (k) {
    case 0: MGK_DISPATCH_KS(launch_tiled_ks, 0, a, cfg, s);
    case 1: MGK_DISPATCH_KS(launch_tiled_ks, 1, a, cfg, s);
    case 2: MGK_DISPATCH_KS(launch_tiled_ks, 2, a, cfg, s);
    case 3: MGK_DISPATCH_KS(launch_tiled_ks, 3, a, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

// dst[b] = src for b < nlines (fill every node with the initial condition)
__global__ void broadcast_kernel(const double* src, double* dst, int64_t nx, int64_t nlines)
{
    const int64_t total = nx * nlines;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i % nx];
}

// out = sqrt(sum r_i^2) in a fixed order (one workgroup)
__global__ void sumsq_norm_kernel(const double* r, int64_t n, double* out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s = fma(r[i], r[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(red[0]);
}

__global__ void clear_ints_kernel(int* p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// norm of the residual from per-chunk partial sums, in a fixed order; records
// it at hist[*counter], advances the counter and raises the convergence flag
__global__ void reduce_norm_kernel(const double* partial, int n, double* hist, int* counter, int* flag, double tol)
{
    if (*flag != 0) return;
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nrm = sqrt(red[0]);
        const int k = *counter;
        hist[k] = nrm;
        *counter = k + 1;
        if (tol >= 0.0 && nrm < tol) *flag = 1;
    }
}

// the same for a batch of problems, one workgroup per problem; a problem that
// converges here also counts itself in *converged
__global__ void reduce_norm_batch_kernel(const BatchNorm* tab, double tol, int* converged)
{
    const BatchNorm e = tab[blockIdx.x];
    if (*e.flag != 0) return;
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < e.n; i += blockDim.x) s += e.partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nrm = sqrt(red[0]);
        const int k = *e.counter;
        e.hist[k] = nrm;
        *e.counter = k + 1;
        if (tol >= 0.0 && nrm < tol) {
            *e.flag = 1;
            atomicAdd(converged, 1);
        }
    }
}

hipError_t launch_reduce_norm_batch(const BatchNorm* tab, int count, double tol, int* converged, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_norm_batch_kernel, dim3(count), dim3(256), 0, s, tab, tol, converged);
    return hipGetLastError();
}

template <int K, int ST>
hipError_t launch_batch_ks(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s);

template <int K, int ST>
hipError_t launch_tiled_batch_ks(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s);

template <int K, int ST>
hipError_t launch_wide_batch_ks(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s);

bool tiled_batch_compiled(const KernelCfg& cfg)
{
#define MGK_CASE(C, W) \
    if (cfg.cpt == C && cfg.nw == W && cfg.intervals == 1) return true;
    MGK_TILED_BATCH_CFG_LIST(MGK_CASE)
#undef MGK_CASE
    return false;
}

// every split-line problem of a batch phase in one launch (degree 0..3)
hipError_t launch_tiled_batch(const BatchLaunch& t, const KernelCfg& cfg, int k, int stepper, hipStream_t s)
{
    if (t.nblocks <= 0) return hipSuccess;
    switch (k) {
    case 0: MGK_DISPATCH_KS(launch_tiled_batch_ks, 0, t, cfg, s);
    case 1: MGK_DISPATCH_KS(launch_tiled_batch_ks, 1, t, cfg, s);
    case 2: MGK_DISPATCH_KS(launch_tiled_batch_ks, 2, t, cfg, s);
    case 3: MGK_DISPATCH_KS(launch_tiled_batch_ks, 3, t, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wide_batch(const BatchLaunch& t, const KernelCfg& cfg, int k, int stepper, hipStream_t s)
{
    if (t.nblocks <= 0) return hipSuccess;
    switch (k) {
    case 0: MGK_DISPATCH_KS(launch_wide_batch_ks, 0, t, cfg, s);
    case 1: MGK_DISPATCH_KS(launch_wide_batch_ks, 1, t, cfg, s);
    case 2: MGK_DISPATCH_KS(launch_wide_batch_ks, 2, t, cfg, s);
    case 3: MGK_DISPATCH_KS(launch_wide_batch_ks, 3, t, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch(const BatchLaunch& t, const KernelCfg& cfg, int k, int stepper, hipStream_t s)
{
    if (t.nblocks <= 0) return hipSuccess;
    switch (k) {
    case 0: MGK_DISPATCH_KS(launch_batch_ks, 0, t, cfg, s);
    case 1: MGK_DISPATCH_KS(launch_batch_ks, 1, t, cfg, s);
    case 2: MGK_DISPATCH_KS(launch_batch_ks, 2, t, cfg, s);
    case 3: MGK_DISPATCH_KS(launch_batch_ks, 3, t, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

// smooth test lines for timing runs: u[b][i] = 0.5 + 0.25 sin(2 pi (i + 1/2)/nx + 0.1 b)
__global__ void fill_wave_kernel(double* u, int64_t nx, int64_t nlines)
{
    const int64_t total = nx * nlines;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / nx, c = i - b * nx;
        u[i] = 0.5 + 0.25 * sin(2.0 * M_PI * ((double)c + 0.5) / (double)nx + 0.1 * (double)b);
    }
}

hipError_t launch_fill_wave(double* u, int64_t nx, int64_t nlines, hipStream_t s)
{
    if (nlines <= 0) return hipSuccess;
    int64_t blocks = (nx * nlines + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_wave_kernel, dim3((unsigned)blocks), dim3(256), 0, s, u, nx, nlines);
    return hipGetLastError();
}

hipError_t launch_broadcast(const double* src, double* dst, int64_t nx, int64_t nlines, hipStream_t s)
{
    if (nlines <= 0) return hipSuccess;
    const int64_t total = nx * nlines;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(broadcast_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, nx, nlines);
    return hipGetLastError();
}

hipError_t launch_sumsq_norm(const double* r, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sumsq_norm_kernel, dim3(1), dim3(256), 0, s, r, n, out);
    return hipGetLastError();
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long value, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long value, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const int blocks = want < 1024 ? (int)want : 1024;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_clear_ints(int* p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
    hipLaunchKernelGGL(clear_ints_kernel, dim3(blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_reduce_norm(const double* partial, int n, double* hist, int* counter, int* flag, double tol,
                              hipStream_t s)
{
    hipLaunchKernelGGL(reduce_norm_kernel, dim3(1), dim3(256), 0, s, partial, n, hist, counter, flag, tol);
    return hipGetLastError();
}

}  // namespace mgk
