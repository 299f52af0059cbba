// Univariate conditional simulation from block Vecchia predictions
// (Section 2.4): R draws mean_j + sqrt(var_j) z_rj per new location, their
// sample mean and standard deviation, the 95 % interval, and -- against
// held-out true values -- the prediction-interval coverage (PICP) and the
// mean square prediction error (MSPE) of Section 3.
#include "internal.hpp"

namespace bv {

constexpr double kZ975 = 1.959963984540054;   // standard normal quantile at 0.975
constexpr int kCondsimBlocks = 1024;

// One thread per location (grid-stride); z is read coalesced, draw r of
// location j at z[r * n + j].  Two passes over the draws (mean, then squared
// deviations).  Per-workgroup coverage counts and squared errors go to part.
__global__ void __launch_bounds__(256)
condsim_kernel(const double* __restrict__ mean, const double* __restrict__ var, int64_t n,
               const double* __restrict__ z, int R, const double* __restrict__ y_true, double* __restrict__ smean,
               double* __restrict__ ssd, double* __restrict__ lo, double* __restrict__ hi, double* __restrict__ part) {
  __shared__ double s_in[256], s_err[256];
  double in_acc = 0.0, err_acc = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    const double mu = mean[j], sd = sqrt(var[j]);
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc += mu + sd * z[(size_t)r * n + j];
    const double m = acc / (double)R;
    double ss = 0.0;
    for (int r = 0; r < R; ++r) {
      const double dv = (mu + sd * z[(size_t)r * n + j]) - m;
      ss += dv * dv;
    }
    const double sdv = sqrt(ss / (double)(R - 1));
    const double l = m - kZ975 * sdv, h = m + kZ975 * sdv;
    if (smean) smean[j] = m;
    if (ssd) ssd[j] = sdv;
    if (lo) lo[j] = l;
    if (hi) hi[j] = h;
    if (y_true) {
      const double yt = y_true[j];
      in_acc += (yt >= l && yt <= h) ? 1.0 : 0.0;
      err_acc += (m - yt) * (m - yt);
    }
  }
  s_in[threadIdx.x] = in_acc;
  s_err[threadIdx.x] = err_acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_in[threadIdx.x] += s_in[threadIdx.x + s];
      s_err[threadIdx.x] += s_err[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s_in[0];
    part[2 * blockIdx.x + 1] = s_err[0];
  }
}

// Fixed-order sum of the per-workgroup parts: stats = (PICP, MSPE).
__global__ void __launch_bounds__(256) condsim_final_kernel(const double* __restrict__ part, int nb, int64_t n,
                                                             double* __restrict__ stats) {
  __shared__ double s_in[256], s_err[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  s_in[threadIdx.x] = a;
  s_err[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_in[threadIdx.x] += s_in[threadIdx.x + s];
      s_err[threadIdx.x] += s_err[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = s_in[0] / (double)n;
    stats[1] = s_err[0] / (double)n;
  }
}

}  // namespace bv

using namespace bv;

extern "C" size_t vecchia_condsim_workspace_size(int64_t n) {
  return n > 0 ? sizeof(double) * 2 * kCondsimBlocks : 0;
}

extern "C" int vecchia_condsim(const double* mean, const double* var, int64_t n, const double* z, int32_t R,
                               const double* y_true, double* smean, double* ssd, double* lo, double* hi,
                               double* stats, void* workspace, size_t ws_bytes, void* stream) {
  if (!mean || !var || !z || !workspace || n <= 0 || R < 2 || (y_true && !stats)) return VECCHIA_EINVAL;
  if (ws_bytes < vecchia_condsim_workspace_size(n)) return VECCHIA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  const int64_t want = (n + 255) / 256;
  const int nb = (int)(want < kCondsimBlocks ? want : kCondsimBlocks);
  double* part = static_cast<double*>(workspace);
  hipLaunchKernelGGL(condsim_kernel, dim3(nb), dim3(256), 0, s, mean, var, n, z, (int)R, y_true, smean, ssd, lo, hi,
                     part);
  if (hipGetLastError() != hipSuccess) return VECCHIA_EHIP;
  if (y_true) {
    hipLaunchKernelGGL(condsim_final_kernel, dim3(1), dim3(256), 0, s, part, nb, n, stats);
    if (hipGetLastError() != hipSuccess) return VECCHIA_EHIP;
  }
  return VECCHIA_OK;
}
