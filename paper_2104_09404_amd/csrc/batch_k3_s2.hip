// Batched sweep kernels (many independent problems per launch) for
// reconstruction degree k = 3 and the 2-stage Runge-Kutta scheme.
#include "sweep_impl.h"

namespace mgk {
template hipError_t launch_batch_ks<3, 2>(const BatchLaunch& t, const KernelCfg& cfg, hipStream_t s);
}  // namespace mgk
