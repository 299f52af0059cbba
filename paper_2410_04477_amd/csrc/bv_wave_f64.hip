// One-wave matrix-core kernels, FP64 instantiations (the kernel is in wave_kernel.hpp).
#include "wave_kernel.hpp"

namespace bv {

hipError_t launch_wave_f64(int g, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  if (mode == 0) return launch_wave_t<double, 0>(g, a, thp, grid, s);
  if (mode == 1) return launch_wave_t<double, 1>(g, a, thp, grid, s);
  if (mode == 5) return launch_wave_t<double, 5>(g, a, thp, grid, s);
  if (mode == 4) return launch_wave_t<double, 4>(g, a, thp, grid, s);
  if (mode == 6) return launch_wave_t<double, 6>(g, a, thp, grid, s);
  if (mode == 3) return launch_wave_t<double, 3>(g, a, thp, grid, s);
  return hipErrorInvalidValue;
}

bool wave_fits(int g, bool fp32) { return g >= 1 && g <= (fp32 ? kWaveMaxG32 : kWaveMaxG64); }

hipError_t launch_wave(int g, bool fp32, int mode, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  if (!wave_fits(g, fp32)) return hipErrorInvalidValue;
  if (a.gen) return fp32 ? launch_wave_gen_f32(g, mode, a, thp, grid, s) : launch_wave_gen_f64(g, mode, a, thp, grid, s);
  return fp32 ? launch_wave_f32(g, mode, a, thp, grid, s) : launch_wave_f64(g, mode, a, thp, grid, s);
}

}  // namespace bv
