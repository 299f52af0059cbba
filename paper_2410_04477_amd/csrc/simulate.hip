// Sequential Vecchia simulator (data generator for the synthetic workloads):
// points in a given (random) order, point i drawn from N(c_i^T y_N(i), s_i)
// given its nearest earlier points N(i).  The weights c_i and variances s_i
// come from the adjoint kernel's coefficient mode (one workgroup per point,
// FP64).  The recursion runs in passes: a point is drawn in the first pass in
// which all of its neighbours were drawn in earlier passes, so each value is a
// fixed function of the inputs (bit-for-bit reproducible).
#include <string.h>

#include <vector>

#include "internal.hpp"

namespace bv {

__global__ void unit_blocks_kernel(int* __restrict__ bp, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) bp[i] = i;
}

// grid.y runs over the data sets that share the design (same neighbour lists)
__global__ void sim_pass_kernel(const int* __restrict__ nbr_ptr, const int* __restrict__ nbr_idx,
                                const double* __restrict__ coef, int64_t coef_stride, const double* __restrict__ cvar,
                                const double* __restrict__ z, double* __restrict__ y, int* __restrict__ done, int n,
                                int pass, int* __restrict__ ndone) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (i >= n) return;
  int* dn = done + (size_t)t * (n + 8);
  if (dn[i] != 0) return;
  const int o0 = nbr_ptr[i], o1 = nbr_ptr[i + 1];
  const double* cf = coef + (size_t)t * coef_stride;
  const double* yy = y + (size_t)t * n;
  double acc = 0.0;
  for (int q = o0; q < o1; ++q) {
    const int j = nbr_idx[q];
    const int dj = dn[j];
    if (dj == 0 || dj >= pass) return;  // a neighbour is not drawn yet
    acc += cf[q] * yy[j];
  }
  y[(size_t)t * n + i] = acc + sqrt(cvar[(size_t)t * n + i]) * z[(size_t)t * n + i];
  dn[i] = pass;
  atomicAdd(ndone, 1);
}

}  // namespace bv

using namespace bv;

namespace {
inline size_t al256s(size_t x) { return (x + 255) & ~(size_t)255; }
struct SimLayout {
  size_t bp, cfg, sched, counts, stats, coef, cvar, flag, done, total;
};
SimLayout sim_layout(int64_t n, int64_t nnz, int64_t nt) {
  SimLayout L;
  size_t o = 0;
  L.bp = o;     o = al256s(o + sizeof(int) * (n + 1));
  L.cfg = o;    o = al256s(o + sizeof(int) * n);
  L.sched = o;  o = al256s(o + sizeof(int) * n);
  L.counts = o; o = al256s(o + sizeof(int) * 64);
  L.stats = o;  o = al256s(o + sizeof(unsigned long long) * 8 + sizeof(int) * (16 + 32));
  L.coef = o;   o = al256s(o + sizeof(double) * (nnz > 0 ? nnz : 1) * nt);
  L.cvar = o;   o = al256s(o + sizeof(double) * n * nt);
  L.flag = o;   o = al256s(o + sizeof(int) * n * nt);
  L.done = o;   o = al256s(o + sizeof(int) * (n + 8) * nt + 64);
  L.total = o;
  return L;
}
template <typename P> P* at(void* base, size_t off) { return reinterpret_cast<P*>(static_cast<char*>(base) + off); }
}  // namespace

#define SCHECK(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return VECCHIA_EHIP; \
  } while (0)

extern "C" size_t vecchia_simulate_workspace_size(int64_t n, int64_t nnz, int32_t ntheta) {
  if (n <= 0 || nnz < 0 || ntheta <= 0) return 0;
  return sim_layout(n, nnz, ntheta).total;
}

extern "C" int vecchia_simulate(const double* locs_ord, int64_t n, int32_t d, const int32_t* nbr_ptr,
                                const int32_t* nbr_idx, const vecchia_theta* theta, int32_t ntheta, const double* z,
                                double* y, void* workspace, size_t ws_bytes, void* stream) {
  if (!locs_ord || !nbr_ptr || !nbr_idx || !theta || !z || !y || !workspace) return VECCHIA_EINVAL;
  if (n <= 0 || d < 1 || d > 3 || n >= ((int64_t)1 << 31)) return VECCHIA_EINVAL;
  if (ntheta < 1 || ntheta > kMaxThetaPerLaunch || (int64_t)ntheta * (n + 8) >= ((int64_t)1 << 31))
    return VECCHIA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int hnnz = 0;
  SCHECK(hipMemcpyAsync(&hnnz, nbr_ptr + n, sizeof(int), hipMemcpyDeviceToHost, s));
  SCHECK(hipStreamSynchronize(s));
  const SimLayout L = sim_layout(n, hnnz, ntheta);
  if (ws_bytes < L.total) return VECCHIA_ENOMEM;
  ThetaPack thp;
  memset(&thp, 0, sizeof(thp));
  for (int q = 0; q < ntheta; ++q) {
    const vecchia_theta& t = theta[q];
    if (!(t.sigma2 > 0) || !(t.range > 0) || !(t.nugget >= 0)) return VECCHIA_EINVAL;
    ThetaDev& o = thp.t[q];
    if (t.nu == 0.5) o.nu_code = 0;
    else if (t.nu == 1.5) o.nu_code = 1;
    else if (t.nu == 2.5) o.nu_code = 2;
    else return VECCHIA_EUNSUPPORTED;
    o.sigma2 = t.sigma2;
    o.nugget = t.nugget;
    o.inv_range = 1.0 / t.range;
    for (int k = 0; k < 3; ++k) o.inv_scale[k] = k < d ? 1.0 / (t.range * t.aniso[k]) : 0.0;
  }
  int* bp = at<int>(workspace, L.bp);
  int* cfg = at<int>(workspace, L.cfg);
  int* sched = at<int>(workspace, L.sched);
  int* counts = at<int>(workspace, L.counts);
  unsigned long long* stats = at<unsigned long long>(workspace, L.stats);
  int* maxes = reinterpret_cast<int*>(stats + 8);
  const int ni = (int)n;
  hipLaunchKernelGGL(unit_blocks_kernel, dim3((ni + 256) / 256), dim3(256), 0, s, bp, ni);
  SCHECK(launch_fill_int(counts, 64, 0, s));
  int* lmax_cfg = maxes + 16;
  SCHECK(launch_fill_int(reinterpret_cast<int*>(stats), 16 + 16 + 32, 0, s));
  SCHECK(launch_classify(bp, nbr_ptr, ni, cfg, counts, stats, maxes, lmax_cfg, kEngineMfmaWg, 1, s));
  int hc[32], hmax[4];
  SCHECK(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s));
  SCHECK(hipMemcpyAsync(hmax, maxes, sizeof(hmax), hipMemcpyDeviceToHost, s));
  SCHECK(hipStreamSynchronize(s));
  if (hmax[3] > 0) return hmax[0] > VECCHIA_MAX_JOINT ? VECCHIA_EUNSUPPORTED : VECCHIA_EINVAL;
  int hoff[32], acc = 0;
  for (int c = 0; c < kMfmaMaxG; ++c) {
    hoff[c] = acc;
    acc += hc[c];
  }
  SCHECK(hipMemcpyAsync(counts + 32, hoff, sizeof(int) * kMfmaMaxG, hipMemcpyHostToDevice, s));
  SCHECK(launch_fill_int(counts, 32, 0, s));
  SCHECK(launch_scatter(cfg, ni, counts + 32, counts, sched, s));
  AdjArgs a;
  memset(&a, 0, sizeof(a));
  a.locs = locs_ord;
  a.y = nullptr;
  a.block_ptr = bp;
  a.nbr_ptr = nbr_ptr;
  a.nbr_idx = nbr_idx;
  a.ntheta = ntheta;
  a.bc = ni;
  a.coef_stride = hnnz;
  a.d = d;
  a.ldx = mfma_ldx(1);
  a.flag = at<int>(workspace, L.flag);
  a.coef = at<double>(workspace, L.coef);
  a.cvar = at<double>(workspace, L.cvar);
  for (int c = 0; c < kMfmaMaxG; ++c) {
    if (hc[c] == 0) continue;
    a.sched = sched + hoff[c];
    a.nsched = hc[c];
    SCHECK(launch_mfma(c + 1, false, 2, a, thp, hc[c] * ntheta, s));
  }
  // recursion in passes
  int* done = at<int>(workspace, L.done);
  int* ndone = done + (size_t)(n + 8) * ntheta;
  SCHECK(launch_fill_int(done, (ni + 8) * ntheta + 8, 0, s));
  const int target = ni * ntheta;
  int total = 0;
  for (int pass = 1; total < target; pass += 16) {
    for (int q = 0; q < 16; ++q)
      hipLaunchKernelGGL(sim_pass_kernel, dim3((ni + 255) / 256, ntheta), dim3(256), 0, s, nbr_ptr, nbr_idx, a.coef,
                         (int64_t)hnnz, a.cvar, z, y, done, ni, pass + q, ndone);
    SCHECK(hipGetLastError());
    int prev = total;
    SCHECK(hipMemcpyAsync(&total, ndone, sizeof(int), hipMemcpyDeviceToHost, s));
    SCHECK(hipStreamSynchronize(s));
    if (total == prev) return VECCHIA_EINVAL;  // no progress: a neighbour index is not earlier
  }
  return VECCHIA_OK;
}
