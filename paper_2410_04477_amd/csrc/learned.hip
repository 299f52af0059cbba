// Learned warm start for the block Vecchia MLE: binned empirical
// semivariogram features and the kernels that train / run a small MLP
// (96 -> 256 -> 256 -> 3, ReLU) on the GPU.
//
// Variogram: for each data set, all pairs of a subset of k points; pair (i, j),
// i < j, with 0 < h <= h_max falls in bin floor(h / h_max * nbins) (clamped to
// nbins - 1), decided in FP64.  Bin sums of (y_i - y_j)^2 and counts accumulate
// per workgroup in LDS (FP64 sums), workgroup partials are reduced in a fixed
// order, and the
// features are gamma_k / s2 (gamma_k = sum / (2 N_k), s2 = subset variance)
// placed in the data set's smoothness slot (one-hot over nu in {1/2, 3/2, 5/2}).
//
// GEMM: C = op(A) op(B) with BF16 operands on the matrix cores
// (v_mfma_f32_16x16x16_bf16, FP32 accumulation); the epilogue adds a bias,
// applies ReLU, or multiplies by the ReLU mask of a pre-activation (backward).
// Operands are FP32 in memory (master copies) and rounded to BF16 (round to
// nearest even) as they are loaded; mode FP32 uses plain FP32 FMAs instead.
#include <math.h>
#include <string.h>

#include "internal.hpp"

namespace bv {

// ------------------------------------------------------------- variogram --

constexpr int VG_T = 256;
constexpr int VG_MAXBINS = 64;

// grid: (row chunks, data sets).  Workgroup g of data set b handles rows
// i = g, g + gridDim.x, ... against all j > i.
__global__ void __launch_bounds__(VG_T)
variogram_pairs_kernel(const double* __restrict__ locs, int64_t locs_stride, const double* __restrict__ y,
                       int64_t y_stride, int k, int nbins, double hmax, double* __restrict__ part_sum,
                       unsigned* __restrict__ part_cnt) {
  __shared__ double ssum[VG_MAXBINS];
  __shared__ unsigned scnt[VG_MAXBINS];
  const int b = blockIdx.y;
  const double* L = locs + (size_t)b * locs_stride;
  const double* Y = y + (size_t)b * y_stride;
  for (int q = threadIdx.x; q < nbins; q += VG_T) {
    ssum[q] = 0.0;
    scnt[q] = 0u;
  }
  __syncthreads();
  // the bin is an integer decided by floating point: FP64, h / hmax * nbins,
  // no fused multiply-add, exactly as the reference definition evaluates it
  for (int i = blockIdx.x; i < k - 1; i += gridDim.x) {
    const double xi = L[2 * i], yi = L[2 * i + 1];
    const double vi = Y[i];
    for (int j = i + 1 + threadIdx.x; j < k; j += VG_T) {
      int bin;
      double dv2;
      {
#pragma clang fp contract(off)
        const double dx = L[2 * j] - xi, dy = L[2 * j + 1] - yi;
        const double h = sqrt(dx * dx + dy * dy);
        bin = (h > 0.0 && h <= hmax) ? (int)(h / hmax * (double)nbins) : -1;
        const double dv = Y[j] - vi;
        dv2 = dv * dv;
      }
      if (bin >= 0) {
        bin = bin < nbins ? bin : nbins - 1;
        atomicAdd(&ssum[bin], dv2);
        atomicAdd(&scnt[bin], 1u);
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nbins; q += VG_T) {
    const size_t o = ((size_t)b * gridDim.x + blockIdx.x) * nbins + q;
    part_sum[o] = ssum[q];
    part_cnt[o] = scnt[q];
  }
}

// one workgroup per data set: fixed-order reduction of the partials, subset
// variance, normalised features in the nu slot
__global__ void __launch_bounds__(VG_T)
variogram_features_kernel(const double* __restrict__ y, int64_t y_stride, int k, int nbins, int nchunks,
                          const double* __restrict__ part_sum, const unsigned* __restrict__ part_cnt,
                          const int* __restrict__ nu_slot, int nslots, float* __restrict__ feat,
                          double* __restrict__ gamma_out) {
  __shared__ double s1[VG_T], s2[VG_T];
  const int b = blockIdx.x;
  const double* Y = y + (size_t)b * y_stride;
  double a1 = 0.0, a2 = 0.0;
  for (int i = threadIdx.x; i < k; i += VG_T) {
    a1 += Y[i];
    a2 += Y[i] * Y[i];
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int s = VG_T / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  const double mean = s1[0] / k;
  const double var = s2[0] / k - mean * mean;
  const int slot = nu_slot[b];
  for (int q = threadIdx.x; q < nbins * nslots; q += VG_T) feat[(size_t)b * nbins * nslots + q] = 0.f;
  __syncthreads();
  for (int q = threadIdx.x; q < nbins; q += VG_T) {
    double sum = 0.0;
    unsigned long long cnt = 0;
    for (int c = 0; c < nchunks; ++c) {
      const size_t o = ((size_t)b * nchunks + c) * nbins + q;
      sum += part_sum[o];
      cnt += part_cnt[o];
    }
    const double g = cnt ? sum / (2.0 * (double)cnt) : 0.0;
    if (gamma_out) gamma_out[(size_t)b * nbins + q] = g;
    feat[(size_t)b * nbins * nslots + (size_t)slot * nbins + q] = (float)(g / var);
  }
}

// ------------------------------------------------------------------- GEMM --

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f32_to_bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  const float* bias;   // length N or NULL
  const float* mask;   // pre-activation of the same shape as C (ReLU backward) or NULL
  float* Z;            // if non-NULL, pre-activation output (before ReLU)
  int M, N, K;
  int lda, ldb, ldc;
  int ta, tb;          // op(A) = A^T if ta (A stored K x M), op(B) = B^T if tb (B stored N x K)
  int act;             // 0 none, 1 ReLU
  int beta_accum;      // 1: C += result
};

__device__ __forceinline__ float ldA(const GemmArgs& g, int m, int k) {
  if (m >= g.M || k >= g.K) return 0.f;
  return g.ta ? g.A[(size_t)k * g.lda + m] : g.A[(size_t)m * g.lda + k];
}
__device__ __forceinline__ float ldB(const GemmArgs& g, int k, int n) {
  if (n >= g.N || k >= g.K) return 0.f;
  return g.tb ? g.B[(size_t)n * g.ldb + k] : g.B[(size_t)k * g.ldb + n];
}

__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int m, int n, float v) {
  if (m >= g.M || n >= g.N) return;
  const size_t o = (size_t)m * g.ldc + n;
  if (g.bias) v += g.bias[n];
  if (g.Z) g.Z[o] = v;
  if (g.act == 1) v = v > 0.f ? v : 0.f;
  if (g.mask) v = g.mask[o] > 0.f ? v : 0.f;
  if (g.beta_accum) v += g.C[o];
  g.C[o] = v;
}

// one wave per 16 x 16 output tile, BF16 MFMA over K in steps of 16
__global__ void __launch_bounds__(64) gemm_bf16_kernel(GemmArgs g) {
  const int l = threadIdx.x;
  const int n0 = blockIdx.x * 16, m0 = blockIdx.y * 16;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const int row = l & 15, kq = (l >> 4) * 4;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = f32_to_bf16_rne(ldA(g, m0 + row, k0 + kq + j));
      b[j] = f32_to_bf16_rne(ldB(g, k0 + kq + j, n0 + row));
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  // accumulator: lane l holds rows 4*(l/16) + r of column l % 16
#pragma unroll
  for (int r = 0; r < 4; ++r) gemm_epilogue(g, m0 + kq + r, n0 + row, acc[r]);
}

// FP32 reference mode: 16 x 16 tile per 256 threads, plain FMAs
__global__ void __launch_bounds__(256) gemm_f32_kernel(GemmArgs g) {
  const int n = blockIdx.x * 16 + (threadIdx.x & 15);
  const int m = blockIdx.y * 16 + (threadIdx.x >> 4);
  float acc = 0.f;
  for (int k = 0; k < g.K; ++k) acc += ldA(g, m, k) * ldB(g, k, n);
  gemm_epilogue(g, m, n, acc);
}

// --------------------------------------------------------- loss / adam ---

// MSE over all B x D entries: dOut = 2 (out - T) / (B D); loss partials per workgroup
__global__ void __launch_bounds__(256)
mse_kernel(const float* __restrict__ out, const float* __restrict__ tgt, int total, float* __restrict__ dout,
           double* __restrict__ loss_part) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < total; i += gridDim.x * 256) {
    const float d = out[i] - tgt[i];
    dout[i] = 2.f * d / (float)total;
    acc += (double)d * (double)d;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if (threadIdx.x < q) s[threadIdx.x] += s[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = s[0] / (double)total;
}

// column sums of an M x N matrix (bias gradients), one thread per column, fixed order
__global__ void colsum_kernel(const float* __restrict__ X, int M, int N, int ld, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float acc = 0.f;
  for (int m = 0; m < M; ++m) acc += X[(size_t)m * ld + n];
  out[n] = acc;
}

// Adam (Kingma & Ba) with bias correction; t is the 1-based step
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace bv

using namespace bv;

#define LCHECK(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return VECCHIA_EHIP; \
  } while (0)

extern "C" size_t vecchia_variogram_workspace_size(int32_t nsets, int32_t nbins, int32_t nchunks) {
  if (nsets <= 0 || nbins <= 0 || nchunks <= 0) return 0;
  return (size_t)nsets * nchunks * nbins * (sizeof(double) + sizeof(unsigned)) + 256;
}

extern "C" int vecchia_variogram(const double* locs, int64_t locs_stride, const double* y, int64_t y_stride,
                                 int32_t nsets, int32_t k, int32_t nbins, double hmax, const int32_t* nu_slot,
                                 int32_t nslots, float* features, double* gamma, int32_t nchunks, void* workspace,
                                 size_t ws_bytes, void* stream) {
  if (!locs || !y || !nu_slot || !features || !workspace) return VECCHIA_EINVAL;
  if (nsets <= 0 || k < 2 || nbins <= 0 || nbins > VG_MAXBINS || !(hmax > 0) || nslots <= 0 || nchunks <= 0)
    return VECCHIA_EINVAL;
  if (ws_bytes < vecchia_variogram_workspace_size(nsets, nbins, nchunks)) return VECCHIA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  double* ps = static_cast<double*>(workspace);
  unsigned* pc = reinterpret_cast<unsigned*>(ps + (size_t)nsets * nchunks * nbins);
  hipLaunchKernelGGL(variogram_pairs_kernel, dim3(nchunks, nsets), dim3(VG_T), 0, s, locs, locs_stride, y, y_stride,
                     k, nbins, hmax, ps, pc);
  hipLaunchKernelGGL(variogram_features_kernel, dim3(nsets), dim3(VG_T), 0, s, y, y_stride, k, nbins, nchunks, ps,
                     pc, nu_slot, nslots, features, gamma);
  LCHECK(hipGetLastError());
  return VECCHIA_OK;
}

extern "C" int vecchia_gemm(const float* A, const float* B, float* C, const float* bias, const float* mask, float* Z,
                            int32_t M, int32_t N, int32_t K, int32_t lda, int32_t ldb, int32_t ldc, int32_t ta,
                            int32_t tb, int32_t act, int32_t accumulate, int32_t use_bf16, void* stream) {
  if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0) return VECCHIA_EINVAL;
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.C = C;
  g.bias = bias;
  g.mask = mask;
  g.Z = Z;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.ta = ta;
  g.tb = tb;
  g.act = act;
  g.beta_accum = accumulate;
  const dim3 grid((N + 15) / 16, (M + 15) / 16);
  if (use_bf16)
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(64), 0, (hipStream_t)stream, g);
  else
    hipLaunchKernelGGL(gemm_f32_kernel, grid, dim3(256), 0, (hipStream_t)stream, g);
  LCHECK(hipGetLastError());
  return VECCHIA_OK;
}

extern "C" int vecchia_mse(const float* out, const float* target, int32_t total, float* dout, double* loss_part,
                           int32_t nparts, void* stream) {
  if (!out || !target || !dout || !loss_part || total <= 0 || nparts <= 0) return VECCHIA_EINVAL;
  hipLaunchKernelGGL(mse_kernel, dim3(nparts), dim3(256), 0, (hipStream_t)stream, out, target, total, dout, loss_part);
  LCHECK(hipGetLastError());
  return VECCHIA_OK;
}

extern "C" int vecchia_colsum(const float* X, int32_t M, int32_t N, int32_t ld, float* out, void* stream) {
  if (!X || !out || M <= 0 || N <= 0) return VECCHIA_EINVAL;
  hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, X, M, N, ld, out);
  LCHECK(hipGetLastError());
  return VECCHIA_OK;
}

extern "C" int vecchia_adam(float* param, const float* grad, float* m, float* v, int64_t n, double lr, double beta1,
                            double beta2, double eps, int64_t step, void* stream) {
  if (!param || !grad || !m || !v || n <= 0 || step < 1) return VECCHIA_EINVAL;
  const float c1 = (float)(1.0 - pow(beta1, (double)step));
  const float c2 = (float)(1.0 - pow(beta2, (double)step));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, param, grad,
                     m, v, (int)n, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
  LCHECK(hipGetLastError());
  return VECCHIA_OK;
}
