// Sweep kernels for reconstruction degree k = 1 and forward Euler (one translation
// unit per scheme so that the kernels compile in parallel).
#include "sweep_impl.h"

namespace mgk {
template hipError_t launch_sweep_ks<1, 1>(const SweepArgs& a, const KernelCfg& cfg, hipStream_t s);
}  // namespace mgk
