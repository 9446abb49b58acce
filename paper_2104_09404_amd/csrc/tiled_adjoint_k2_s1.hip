// Adjoint kernels of split lines for reconstruction degree k = 2 and the
// 1-stage Runge-Kutta scheme (one translation unit per scheme).
#include "tiled_adjoint_impl.h"

namespace mgk {
template hipError_t launch_tiled_adjoint_ks<2, 1>(const AdjArgs& a, const KernelCfg& cfg, int store_mode,
                                                          hipStream_t s);
}  // namespace mgk
