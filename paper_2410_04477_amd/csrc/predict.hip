// Univariate conditional simulation from block Vecchia predictions
// (Section 2.4): R draws mean_j + sqrt(var_j) z_rj per new location, their
// sample mean and standard deviation, the 95 % interval, and -- against
// held-out true values -- the prediction-interval coverage (PICP) and the
// mean square prediction error (MSPE) of Section 3.
#include "internal.hpp"

namespace bv {

constexpr double kZ975 = 1.959963984540054;   // standard normal quantile at 0.975
constexpr int kCondsimBlocks = 4096;
constexpr int kSlices = 4;   // waves per workgroup, each summing every kSlices-th draw

// A workgroup takes 64 consecutive locations; wave k of it sums the draws
// r = k, k + kSlices, ... (one coalesced 512-byte row of z per step), so the
// R x n draws are read once with four times the waves in flight.  The draws
// are summed shifted by the mean (d = sqrt(var) z): sample mean
// mean + sum d / R, sample variance (sum d^2 - (sum d)^2 / R) / (R - 1).
// Per-workgroup coverage counts and squared errors go to part.
__global__ void __launch_bounds__(256)
condsim_kernel(const double* __restrict__ mean, const double* __restrict__ var, int64_t n,
               const double* __restrict__ z, int R, const double* __restrict__ y_true, double* __restrict__ smean,
               double* __restrict__ ssd, double* __restrict__ lo, double* __restrict__ hi, double* __restrict__ part) {
  __shared__ double s1s[kSlices][64], s2s[kSlices][64];
  __shared__ double s_in[256], s_err[256];
  const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
  double in_acc = 0.0, err_acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
    const int64_t j = base + lane;
    double a1 = 0.0, a2 = 0.0;
    if (j < n) {
      const double sd = sqrt(var[j]);
      const double* zj = z + j;
#pragma unroll 8
      for (int r = slice; r < R; r += kSlices) {
        const double dv = sd * zj[(size_t)r * n];
        a1 += dv;
        a2 += dv * dv;
      }
    }
    s1s[slice][lane] = a1;
    s2s[slice][lane] = a2;
    __syncthreads();
    if (slice == 0 && j < n) {
      double t1 = 0.0, t2 = 0.0;
#pragma unroll
      for (int k = 0; k < kSlices; ++k) {
        t1 += s1s[k][lane];
        t2 += s2s[k][lane];
      }
      const double m = mean[j] + t1 / (double)R;
      const double sdv = sqrt(fmax(t2 - t1 * t1 / (double)R, 0.0) / (double)(R - 1));
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
    __syncthreads();
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
  const int64_t want = (n + 63) / 64;
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
