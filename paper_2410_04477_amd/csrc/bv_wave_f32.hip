// One-wave matrix-core kernels, FP32 instantiations (the kernel is in wave_kernel.hpp).
#include "wave_kernel.hpp"

namespace bv {

hipError_t launch_wave_f32(int g, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  if (mode == 0) return launch_wave_t<float, 0>(g, a, thp, grid, s);
  if (mode == 1) return launch_wave_t<float, 1>(g, a, thp, grid, s);
  if (mode == 5) return launch_wave_t<float, 5>(g, a, thp, grid, s);
  if (mode == 2) return launch_wave_t<float, 2>(g, a, thp, grid, s);
  if (mode == 3) return launch_wave_t<float, 3>(g, a, thp, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace bv
