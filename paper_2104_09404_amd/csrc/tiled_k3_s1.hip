// Tiled-line sweep kernels for reconstruction degree k = 3 and the
// 1-stage Runge-Kutta scheme (one translation unit per scheme so that the
// kernels compile in parallel).
#include "tiled_impl.h"

namespace mgk {
template hipError_t launch_tiled_ks<3, 1>(const SweepArgs& a, const KernelCfg& cfg, hipStream_t s);
template hipError_t launch_tiled_batch_ks<3, 1>(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s);
}  // namespace mgk
