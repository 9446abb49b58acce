// Adjoint kernels for reconstruction degree k = 0 and SSPRK3 (one translation
// unit per scheme so that the kernels compile in parallel).
#include "adjoint_impl.h"

namespace mgk {
template hipError_t launch_adjoint_ks<0, 3>(const AdjArgs& a, const KernelCfg& cfg, int store_mode, hipStream_t s);
}  // namespace mgk
