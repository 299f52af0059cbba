// Small device kernels around the fused block kernels: size-class schedule,
// FP32-guard compaction, and the deterministic FP64 cross-block reduction
// (the final loop of Alg. 1: l = sum_i l_i).
#include "internal.hpp"

namespace bv {

// Per block: joint size p_i = m_i + l_i, its tile configuration, and
// workload statistics (exact integer sums, so they are deterministic).
__global__ void classify_kernel(const int* __restrict__ block_ptr, const int* __restrict__ nbr_ptr, int bc,
                                int* __restrict__ cfg_of, int* __restrict__ counts, unsigned long long* __restrict__ stats,
                                int* __restrict__ maxes, int* __restrict__ lmax_cfg, int engine, int mpad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  const int l = block_ptr[b + 1] - block_ptr[b];
  const int m0 = nbr_ptr[b + 1] - nbr_ptr[b];
  const int m = m0 < 0 ? m0 : (m0 + mpad - 1) / mpad * mpad;
  const int p = l + m;
  int c = engine == kEngineTiles ? cfg_for_joint(p) : cfg_mfma_for_joint(p);
  if (c < 0 && p <= 16383) c = kLargeCfg;   // served by the global-workspace kernel
  if (l <= 0 || m < 0) c = -2;
  cfg_of[b] = c;
  if (c >= 0) {
    atomicAdd(&counts[c], 1);
    atomicMax(&lmax_cfg[c], l);
  }
  const unsigned long long pp = (unsigned long long)p;
  atomicAdd(&stats[0], pp * pp * pp);
  atomicAdd(&stats[1], pp * pp);
  atomicAdd(&stats[2], pp * (pp + 1ull) / 2ull);
  atomicAdd(&stats[3], (unsigned long long)(l > 0 ? l : 0));
  atomicMax(&maxes[0], p);
  atomicMax(&maxes[1], l);
  atomicMax(&maxes[2], m);
  if (c < 0) atomicAdd(&maxes[3], 1);  // blocks no configuration covers
}

__global__ void scatter_kernel(const int* __restrict__ cfg_of, int bc, const int* __restrict__ cfg_off,
                               int* __restrict__ cursor, int* __restrict__ sched) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  const int c = cfg_of[b];
  if (c < 0) return;
  const int pos = atomicAdd(&cursor[c], 1);
  sched[cfg_off[c] + pos] = b;
}

// Size-class merge: cfg_of[b] <- remap[cfg_of[b]] (classes >= 0 only).
__global__ void remap_kernel(int* __restrict__ cfg_of, int bc, const int* __restrict__ remap) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  const int c = cfg_of[b];
  if (c >= 0) cfg_of[b] = remap[c];
}

__global__ void fill_int_kernel(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Collect the (theta, block) pairs of one size class whose FP32 pivots tripped the guard.
__global__ void compact_flagged_kernel(const int* __restrict__ sched, int nsched, int ntheta, int bc,
                                       const int* __restrict__ flag, int* __restrict__ list,
                                       int* __restrict__ count) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nsched * ntheta) return;
  const int tt = w / nsched;
  const int b = sched[w - tt * nsched];
  const int e = tt * bc + b;
  if (flag[e] & 1) {
    const int pos = atomicAdd(count, 1);
    list[pos] = e;
  }
}

// Deterministic FP64 sum of per-block terms for one theta per workgroup:
// thread j sums entries j, j+kRed, ... in order, then a fixed LDS tree
// (kRed = 1024 threads: the loop is bound by load latency, so the more loads
// in flight the better).
// counters[2t] = blocks re-factorised in FP64, counters[2t+1] = non-PD blocks.
constexpr int kRed = 1024;
__global__ void __launch_bounds__(kRed)
reduce_partials_kernel(const double* __restrict__ partial, const int* __restrict__ flag, int bc, int fp64_only,
                       double* __restrict__ out, int* __restrict__ counters) {
  __shared__ double ssum[kRed];
  __shared__ int sref[kRed], sbad[kRed];
  const int tt = blockIdx.x;
  const double* pp = partial + (size_t)tt * bc;
  const int* ff = flag + (size_t)tt * bc;
  double acc = 0.0;
  int nref = 0, nbad = 0;
  // unrolled so that several loads are in flight; the additions keep their order
#pragma unroll 8
  for (int i = threadIdx.x; i < bc; i += kRed) {
    acc += pp[i];
    const int f = ff[i];
    nref += (f & 4) ? 1 : 0;
    nbad += ((f & 2) && (fp64_only || (f & 4))) ? 1 : 0;
  }
  ssum[threadIdx.x] = acc;
  sref[threadIdx.x] = nref;
  sbad[threadIdx.x] = nbad;
  __syncthreads();
  for (int s = kRed / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      ssum[threadIdx.x] += ssum[threadIdx.x + s];
      sref[threadIdx.x] += sref[threadIdx.x + s];
      sbad[threadIdx.x] += sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[tt] = sbad[0] ? __builtin_nan("") : ssum[0];
    if (counters) {
      counters[2 * tt] = sref[0];
      counters[2 * tt + 1] = sbad[0];
    }
  }
}

// Same tree for k-component per-block vectors (gradients): out[t*k + c].
__global__ void __launch_bounds__(kRed)
reduce_vec_kernel(const double* __restrict__ vec, int bc, int k, double* __restrict__ out) {
  __shared__ double ssum[kRed];
  const int tt = blockIdx.x / k;
  const int c = blockIdx.x - tt * k;
  const double* pp = vec + (size_t)tt * bc * k;
  double acc = 0.0;
#pragma unroll 8
  for (int i = threadIdx.x; i < bc; i += kRed) acc += pp[(size_t)i * k + c];
  ssum[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRed / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) ssum[threadIdx.x] += ssum[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = ssum[0];
}

}  // namespace bv

namespace bv {

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

hipError_t launch_classify(const int* block_ptr, const int* nbr_ptr, int bc, int* cfg_of, int* counts,
                           unsigned long long* stats, int* maxes, int* lmax_cfg, int engine, int mpad,
                           hipStream_t s) {
  hipLaunchKernelGGL(classify_kernel, dim3(cdiv(bc, 256)), dim3(256), 0, s, block_ptr, nbr_ptr, bc, cfg_of, counts,
                     stats, maxes, lmax_cfg, engine, mpad);
  return hipGetLastError();
}

hipError_t launch_scatter(const int* cfg_of, int bc, const int* cfg_off, int* cursor, int* sched, hipStream_t s) {
  hipLaunchKernelGGL(scatter_kernel, dim3(cdiv(bc, 256)), dim3(256), 0, s, cfg_of, bc, cfg_off, cursor, sched);
  return hipGetLastError();
}

hipError_t launch_remap(int* cfg_of, int bc, const int* remap, hipStream_t s) {
  hipLaunchKernelGGL(remap_kernel, dim3(cdiv(bc, 256)), dim3(256), 0, s, cfg_of, bc, remap);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_compact_flagged(const int* sched, int nsched, int ntheta, int bc, const int* flag, int* list,
                                  int* count, hipStream_t s) {
  const int n = nsched * ntheta;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_flagged_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, sched, nsched, ntheta, bc, flag,
                     list, count);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, const int* flag, int bc, int ntheta, int fp64_only,
                                  double* out, int* counters, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(ntheta), dim3(kRed), 0, s, partial, flag, bc, fp64_only, out,
                     counters);
  return hipGetLastError();
}

hipError_t launch_reduce_vec(const double* vec, int bc, int k, int ntheta, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_vec_kernel, dim3(ntheta * k), dim3(kRed), 0, s, vec, bc, k, out);
  return hipGetLastError();
}

}  // namespace bv
