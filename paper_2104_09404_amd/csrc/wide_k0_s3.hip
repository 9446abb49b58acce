// Batch kernels for lines of one workgroup with several cell blocks per
// thread, WENO degree k = 0 and 3-stage Runge-Kutta (one translation unit
// per pair so that they compile in parallel).
#include "wide_impl.h"

namespace mgk {
template hipError_t launch_wide_batch_ks<0, 3>(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s);
}  // namespace mgk
