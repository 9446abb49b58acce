// Split-line system sweep kernels for shallow water with reconstruction degree
// k = 0 (one translation unit per system and degree so that they compile in
// parallel).
#include "sys_tiled_impl.h"

namespace mgk {
template hipError_t launch_sys_tiled_sk<2, 0>(const SweepArgs& a, int threads, int stepper, hipStream_t s);
}  // namespace mgk
