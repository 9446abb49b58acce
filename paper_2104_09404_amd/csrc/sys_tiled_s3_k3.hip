// Split-line system sweep kernels for the Euler equations with reconstruction degree
// k = 3 (one translation unit per system and degree so that they compile in
// parallel).
#include "sys_tiled_impl.h"

namespace mgk {
template hipError_t launch_sys_tiled_sk<3, 3>(const SweepArgs& a, int threads, int stepper, hipStream_t s);
}  // namespace mgk
