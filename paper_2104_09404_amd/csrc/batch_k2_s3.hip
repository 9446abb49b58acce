// Batched sweep kernels (many independent problems per launch) for
// reconstruction degree k = 2 and the 3-stage Runge-Kutta scheme.
#include "sweep_impl.h"

namespace mgk {
template hipError_t launch_batch_ks<2, 3>(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s);
}  // namespace mgk
