// One-wave matrix-core kernels with the Bessel-form covariance (any nu), FP64
// instantiations (the kernel is in wave_kernel.hpp).
#include "wave_kernel.hpp"

namespace bv {

hipError_t launch_wave_gen_f64(int g, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  if (mode == 0) return launch_wave_t<double, 0, true>(g, a, thp, grid, s);
  if (mode == 1) return launch_wave_t<double, 1, true>(g, a, thp, grid, s);
  if (mode == 5) return launch_wave_t<double, 5, true>(g, a, thp, grid, s);
  if (mode == 4) return launch_wave_t<double, 4, true>(g, a, thp, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace bv
