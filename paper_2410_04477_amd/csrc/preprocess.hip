// Preprocessing of Alg. 1 on the device: clustering g (K-means, Section 2.1),
// block permutation zeta, and the m nearest earlier neighbours of each block
// centroid (Alg. 1, nearest neighbours).  Untimed in the paper's convention.
//
// K-means: Lloyd iterations in FP64.  Assignment is exhaustive over the
// centroids (staged through LDS, ascending index, strict '<' so ties go to
// the lower index).  Centroid sums use 64-bit fixed point (exact integer
// atomics), so every run produces the same centroids bit for bit.
//
// Neighbours: exact search on a uniform grid of cells over the metric-scaled
// points.  Points are sorted by cell with ascending index inside a cell, so
// "earlier than block i" is a prefix of each cell's list.  For each block the
// search grows a cube of cells around the centroid until at least m earlier
// points lie within the cube's guaranteed radius, collects every earlier point
// inside that radius, sorts by (squared distance, index) in LDS and keeps the
// first m.  Blocks with few earlier points are searched exhaustively.
#include <math.h>
#include <string.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace bv {

static inline int cdiv64(int64_t a, int b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------- utilities --

__global__ void fill_i32_kernel(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void permute_rows_kernel(const double* __restrict__ src, int64_t n, int d, const int64_t* __restrict__ perm,
                                    double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t s = perm[i];
  for (int k = 0; k < d; ++k) dst[i * d + k] = src[s * d + k];
}

// per-workgroup min / max of the metric-scaled coordinates
__global__ void __launch_bounds__(256) bbox_kernel(const double* __restrict__ locs, int64_t n, int d, double w0, double w1,
                                                   double w2, double* __restrict__ part) {
  __shared__ double smn[3][256], smx[3][256];
  const double w[3] = {w0, w1, w2};
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    for (int k = 0; k < d; ++k) {
      const double v = locs[i * d + k] * w[k];
      mn[k] = fmin(mn[k], v);
      mx[k] = fmax(mx[k], v);
    }
  for (int k = 0; k < 3; ++k) {
    smn[k][threadIdx.x] = mn[k];
    smx[k][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) {
        smn[k][threadIdx.x] = fmin(smn[k][threadIdx.x], smn[k][threadIdx.x + s]);
        smx[k][threadIdx.x] = fmax(smx[k][threadIdx.x], smx[k][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      part[blockIdx.x * 6 + k] = smn[k][0];
      part[blockIdx.x * 6 + 3 + k] = smx[k][0];
    }
}

// ---------------------------------------------------------------- kmeans --

struct KmArgs {
  const double* locs;
  int64_t n;
  int d;
  double w[3];
  double lo[3];      // fixed-point origin
  double fscale;     // fixed-point units per coordinate unit
  int bc;
  double* cent;      // bc x 3 (unused dims 0)
  int* label;        // n
  int* changed;      // 1 int
  unsigned long long* fsum;  // bc x 3 fixed-point sums
  int* cnt;          // bc
  double* dist;      // n: squared distance to own centroid (for re-seeding)
};

__global__ void km_init_kernel(KmArgs a, const int64_t* __restrict__ init_idx) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.bc) return;
  const int64_t p = init_idx[c];
  for (int k = 0; k < 3; ++k) a.cent[c * 3 + k] = k < a.d ? a.locs[p * a.d + k] * a.w[k] : 0.0;
}

// nearest centroid of each point; centroids staged through LDS in chunks
constexpr int KM_CHUNK = 512;
__global__ void __launch_bounds__(256) km_assign_kernel(KmArgs a, int first) {
#pragma clang fp contract(off)
  __shared__ double sc[KM_CHUNK * 3];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double x[3] = {0, 0, 0};
  if (i < a.n)
    for (int k = 0; k < a.d; ++k) x[k] = a.locs[i * a.d + k] * a.w[k];
  double best = INFINITY;
  int bi = 0;
  for (int c0 = 0; c0 < a.bc; c0 += KM_CHUNK) {
    const int nc = min(KM_CHUNK, a.bc - c0);
    __syncthreads();
    for (int t = threadIdx.x; t < nc * 3; t += 256) sc[t] = a.cent[c0 * 3 + t];
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      const double t0 = x[0] - sc[c * 3], t1 = x[1] - sc[c * 3 + 1], t2 = x[2] - sc[c * 3 + 2];
      const double dd = t0 * t0 + t1 * t1 + t2 * t2;
      if (dd < best) {
        best = dd;
        bi = c0 + c;
      }
    }
  }
  if (i < a.n) {
    if (!first && a.label[i] != bi) atomicOr(a.changed, 1);
    a.label[i] = bi;
    a.dist[i] = best;
  }
}

// Large block counts: a uniform grid of cubic cells (side h, in the scaled
// coordinates, over the points' bounding box) holds the centroids, about two
// per cell, and each point searches rings of cells around its own until the
// next ring is farther than the best distance found.  A centroid in a cell r+1
// rings away is at least r h from the point, so the search is exact; ties go
// to the lowest centroid index, as in the exhaustive kernel.
constexpr int64_t kKmGridMinBlocks = 65536;

struct KmGrid {
  double lo[3];
  double h, inv_h;
  int nc[3];
  int ncell;
  int* cstart;   // ncell + 1 (exclusive scan of the counts)
  int* ccur;     // ncell + 1: counts, then insertion cursors
  int* cidx;     // bc centroid indices grouped by cell
};

__device__ inline int km_grid_cell(const KmGrid& g, const double* x, int d, int* pc) {
  int cell = 0, stride = 1;
  for (int k = 0; k < 3; ++k) {
    int c = 0;
    if (k < d) {
      const double t = floor((x[k] - g.lo[k]) * g.inv_h);
      c = !(t >= 0.0) ? 0 : (t >= (double)g.nc[k] ? g.nc[k] - 1 : (int)t);
    }
    pc[k] = c;
    cell += c * stride;
    stride *= g.nc[k];
  }
  return cell;
}

__global__ void km_grid_count_kernel(KmArgs a, KmGrid g) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.bc) return;
  int pc[3];
  atomicAdd(&g.ccur[km_grid_cell(g, a.cent + (size_t)c * 3, a.d, pc)], 1);
}

__global__ void km_grid_cursor_kernel(KmGrid g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= g.ncell) g.ccur[i] = g.cstart[i];
}

__global__ void km_grid_place_kernel(KmArgs a, KmGrid g) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.bc) return;
  int pc[3];
  const int pos = atomicAdd(&g.ccur[km_grid_cell(g, a.cent + (size_t)c * 3, a.d, pc)], 1);
  g.cidx[pos] = c;
}

__global__ void __launch_bounds__(256) km_assign_grid_kernel(KmArgs a, KmGrid g, int first) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  double x[3] = {0, 0, 0};
  for (int k = 0; k < a.d; ++k) x[k] = a.locs[i * a.d + k] * a.w[k];
  int pc[3];
  km_grid_cell(g, x, a.d, pc);
  const int rmax = max(g.nc[0], max(g.nc[1], g.nc[2]));
  double best = INFINITY;
  int bi = 0x7fffffff;
  for (int r = 0; r <= rmax; ++r) {
    const int r1 = a.d > 1 ? r : 0, r2 = a.d > 2 ? r : 0;
    for (int o2 = -r2; o2 <= r2; ++o2) {
      const int c2 = pc[2] + o2;
      if (c2 < 0 || c2 >= g.nc[2]) continue;
      for (int o1 = -r1; o1 <= r1; ++o1) {
        const int c1 = pc[1] + o1;
        if (c1 < 0 || c1 >= g.nc[1]) continue;
        for (int o0 = -r; o0 <= r; ++o0) {
          const int c0 = pc[0] + o0;
          if (c0 < 0 || c0 >= g.nc[0]) continue;
          if (max(abs(o0), max(abs(o1), abs(o2))) != r) continue;   // this ring only
          const int cell = c0 + g.nc[0] * (c1 + g.nc[1] * c2);
          const int q1 = g.cstart[cell + 1];
          for (int q = g.cstart[cell]; q < q1; ++q) {
            const int c = g.cidx[q];
            const double t0 = x[0] - a.cent[c * 3], t1 = x[1] - a.cent[c * 3 + 1], t2 = x[2] - a.cent[c * 3 + 2];
            const double dd = t0 * t0 + t1 * t1 + t2 * t2;
            if (dd < best || (dd == best && c < bi)) {
              best = dd;
              bi = c;
            }
          }
        }
      }
    }
    const double reach = (double)r * g.h;
    if (reach * reach * (1.0 - 1e-9) > best) break;
  }
  if (!first && a.label[i] != bi) atomicOr(a.changed, 1);
  a.label[i] = bi;
  a.dist[i] = best;
}

__global__ void km_zero_kernel(KmArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.bc) return;
  a.cnt[c] = 0;
  for (int k = 0; k < 3; ++k) a.fsum[c * 3 + k] = 0ull;
}

__global__ void km_accum_kernel(KmArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int c = a.label[i];
  atomicAdd(&a.cnt[c], 1);
  for (int k = 0; k < a.d; ++k) {
    const double v = (a.locs[i * a.d + k] * a.w[k] - a.lo[k]) * a.fscale;
    atomicAdd(&a.fsum[c * 3 + k], (unsigned long long)llrint(v));
  }
}

// centroid = fixed-point mean; empty clusters keep their centroid (re-seeded on the host side)
__global__ void km_update_kernel(KmArgs a, int* __restrict__ nempty) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.bc) return;
  const int m = a.cnt[c];
  if (m == 0) {
    atomicAdd(nempty, 1);
    return;
  }
  for (int k = 0; k < a.d; ++k)
    a.cent[c * 3 + k] = a.lo[k] + ((double)a.fsum[c * 3 + k] / a.fscale) / (double)m;
}

// squared distance of each point to its (updated) centroid, for re-seeding
// empty clusters; the same unfused arithmetic as the assignment
__global__ void km_dist_kernel(KmArgs a) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int c = a.label[i];
  double x[3] = {0, 0, 0};
  for (int k = 0; k < a.d; ++k) x[k] = a.locs[i * a.d + k] * a.w[k];
  const double t0 = x[0] - a.cent[c * 3], t1 = x[1] - a.cent[c * 3 + 1], t2 = x[2] - a.cent[c * 3 + 2];
  a.dist[i] = t0 * t0 + t1 * t1 + t2 * t2;
}

// farthest point from its centroid (ties: lowest index), two-level
__global__ void __launch_bounds__(256) argmax_kernel(const double* __restrict__ v, int64_t n,
                                                     double* __restrict__ pv, int64_t* __restrict__ pi) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  double best = -INFINITY;
  int64_t bi = INT64_MAX;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    if (v[i] > best) {
      best = v[i];
      bi = i;
    }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double ov = sv[threadIdx.x + s];
      const int64_t oi = si[threadIdx.x + s];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}

__global__ void reseed_kernel(KmArgs a, int c, int64_t p) {
  if (threadIdx.x == 0) {
    for (int k = 0; k < a.d; ++k) a.cent[c * 3 + k] = a.locs[p * a.d + k] * a.w[k];
    a.dist[p] = -1.0;  // never chosen twice
  }
}

// block position of each point: key = position of its cluster in block_perm
__global__ void pos_key_kernel(const int* __restrict__ label, int64_t n, const int* __restrict__ pos_of_label,
                               int* __restrict__ key, int64_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = pos_of_label[label[i]];
  val[i] = i;
}

__global__ void pos_of_label_kernel(const int64_t* __restrict__ block_perm, int bc, int* __restrict__ pos_of_label,
                                    int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bc) return;
  const int64_t c = block_perm[i];
  if (c < 0 || c >= bc) {
    atomicOr(bad, 1);
    return;
  }
  // pos_of_label starts at -1: a second claim of the same cluster is a duplicate
  if (atomicCAS(&pos_of_label[c], -1, i) != -1) atomicOr(bad, 1);
}

__global__ void count_keys_kernel(const int* __restrict__ key, int64_t n, int nkeys, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int k = key[i];
    if (k >= 0 && k < nkeys) atomicAdd(&cnt[k], 1);
  }
}

// ------------------------------------------------------------- neighbours --

struct GridInfo {
  double lo[3];
  double inv_h;   // 1 / cell size
  double h;
  int dims[3];
  int ncell;
};

__device__ __forceinline__ int cell_coord(double x, double lo, double inv_h, int dim) {
  int c = (int)floor((x - lo) * inv_h);
  return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

__global__ void cell_key_kernel(const double* __restrict__ locs, int64_t n, int d, double w0, double w1, double w2,
                                GridInfo g, int* __restrict__ key, int* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w[3] = {w0, w1, w2};
  int cc[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) cc[k] = cell_coord(locs[i * d + k] * w[k], g.lo[k], g.inv_h, g.dims[k]);
  key[i] = (cc[2] * g.dims[1] + cc[1]) * g.dims[0] + cc[0];
  val[i] = (int)i;
}

__global__ void cell_start_kernel(const int* __restrict__ sorted_key, int64_t n, int ncell, int* __restrict__ start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int kcur = i < n ? sorted_key[i] : ncell;
  const int kprev = i > 0 ? sorted_key[i - 1] : -1;
  for (int c = kprev + 1; c <= kcur; ++c) start[c] = (int)i;
}

constexpr int KNN_CAP = 2048;   // LDS candidate capacity (power of two)
constexpr int KNN_T = 256;

struct KnnArgs {
  const double* locs;   // block order
  int d;
  double w[3];
  const int* block_ptr;
  const int* nbr_ptr;
  int* nbr_idx;
  int m;
  GridInfo g;
  const int* cell_start;
  const int* cell_pts;
  int* status;          // set to 1 if a block could not be resolved within capacity
  int brute_first;      // blocks [0, brute_first) use the exhaustive path (set by host ordering)
  int nref;             // candidates are the points below min(block start, nref)
};

// squared distance with a fixed evaluation order and no fused multiply-add
__device__ __forceinline__ double sqdist_fixed(const double* c, const double* __restrict__ locs, int j, int d,
                                               const double* w) {
#pragma clang fp contract(off)
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    const double x = locs[(size_t)j * d + k] * w[k];
    const double t = c[k] - x;
    acc = (k == 0) ? t * t : acc + t * t;
  }
  return acc;
}

__device__ __forceinline__ void block_centroid(const double* __restrict__ locs, int d, const double* w, int b0, int b1,
                                               double* c) {
#pragma clang fp contract(off)
  double acc[3] = {0.0, 0.0, 0.0};
  for (int j = b0; j < b1; ++j)
    for (int k = 0; k < d; ++k) {
      const double x = locs[(size_t)j * d + k] * w[k];
      acc[k] = acc[k] + x;
    }
  for (int k = 0; k < 3; ++k) c[k] = k < d ? acc[k] / (double)(b1 - b0) : 0.0;
}

__device__ __forceinline__ bool key_less(double da, int ia, double db, int ib) {
  return da < db || (da == db && ia < ib);
}

// bitonic sort of N (power of two) keys in LDS
__device__ void bitonic_sort(double* sd, int* si, int N) {
  for (int k = 2; k <= N; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const bool sw = up ? key_less(sd[ixj], si[ixj], sd[i], si[i]) : key_less(sd[i], si[i], sd[ixj], si[ixj]);
          if (sw) {
            const double td = sd[i];
            sd[i] = sd[ixj];
            sd[ixj] = td;
            const int ti = si[i];
            si[i] = si[ixj];
            si[ixj] = ti;
          }
        }
      }
      __syncthreads();
    }
}

__device__ int block_sum_int(int v, int* sred) {
  __syncthreads();
  sred[threadIdx.x] = v;
  __syncthreads();
  for (int s = KNN_T / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sred[threadIdx.x] += sred[threadIdx.x + s];
    __syncthreads();
  }
  const int r = sred[0];
  __syncthreads();
  return r;
}

// visit every earlier point (index < limit) in the cube of cells of Chebyshev radius r around cc
template <typename F>
__device__ void for_cube(const KnnArgs& a, const int* cc, int r, int limit, F&& f) {
  int lo[3], hi[3], ext[3];
  for (int k = 0; k < 3; ++k) {
    lo[k] = max(cc[k] - r, 0);
    hi[k] = min(cc[k] + r, a.g.dims[k] - 1);
    ext[k] = hi[k] - lo[k] + 1;
  }
  const int total = ext[0] * ext[1] * ext[2];
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int ix = lo[0] + q % ext[0];
    const int iy = lo[1] + (q / ext[0]) % ext[1];
    const int iz = lo[2] + q / (ext[0] * ext[1]);
    const int cell = (iz * a.g.dims[1] + iy) * a.g.dims[0] + ix;
    const int s0 = a.cell_start[cell], s1 = a.cell_start[cell + 1];
    for (int s = s0; s < s1; ++s) {
      const int j = a.cell_pts[s];
      if (j >= limit) break;  // ascending inside a cell
      f(j);
    }
  }
}

__global__ void __launch_bounds__(KNN_T) knn_kernel(KnnArgs a, int bc) {
  __shared__ double sd[KNN_CAP];
  __shared__ int si[KNN_CAP];
  __shared__ int sred[KNN_T];
  __shared__ int scount;
  __shared__ double scen[3];
  const int b = blockIdx.x;
  if (b >= bc) return;
  const int limit = min(a.block_ptr[b], a.nref);
  const int out0 = a.nbr_ptr[b];
  const int mi = a.nbr_ptr[b + 1] - out0;
  if (mi == 0) return;
  if (threadIdx.x == 0) {
    double c[3];
    block_centroid(a.locs, a.d, a.w, a.block_ptr[b], a.block_ptr[b + 1], c);
    for (int k = 0; k < 3; ++k) scen[k] = c[k];
    scount = 0;
  }
  __syncthreads();
  const double c[3] = {scen[0], scen[1], scen[2]};
  int K;
  if (limit <= KNN_CAP) {
    // exhaustive over all earlier points
    for (int j = threadIdx.x; j < limit; j += blockDim.x) {
      sd[j] = sqdist_fixed(c, a.locs, j, a.d, a.w);
      si[j] = j;
    }
    K = limit;
  } else {
    int cc[3] = {0, 0, 0};
    for (int k = 0; k < a.d; ++k) cc[k] = cell_coord(c[k], a.g.lo[k], a.g.inv_h, a.g.dims[k]);
    // initial radius from the density of earlier points
    const double frac = (double)limit / (double)a.g.ncell;  // earlier points per cell
    const double need = (double)mi / fmax(frac, 1e-30);
    int r = (int)floor(0.55 * pow(need, 1.0 / (double)a.d));
    if (r < 1) r = 1;
    const int rmax = max(a.g.dims[0], max(a.g.dims[1], a.g.dims[2]));
    double rad2;
    for (;;) {
      const double rad = fmax((double)r * a.g.h * (1.0 - 1e-9), 0.0);
      rad2 = r >= rmax ? INFINITY : rad * rad;
      int cnt = 0;
      for_cube(a, cc, r, limit, [&](int j) {
        if (sqdist_fixed(c, a.locs, j, a.d, a.w) <= rad2) ++cnt;
      });
      cnt = block_sum_int(cnt, sred);
      if (cnt >= mi || r >= rmax) {
        if (cnt <= KNN_CAP) break;
        // too many points inside the radius: shrink the threshold by bisection
        double lo2 = 0.0, hi2 = rad2;
        if (!isfinite(hi2)) hi2 = 1e300;
        int it = 0;
        for (; it < 200; ++it) {
          const double mid = 0.5 * (lo2 + hi2);
          int c2 = 0;
          for_cube(a, cc, r, limit, [&](int j) {
            if (sqdist_fixed(c, a.locs, j, a.d, a.w) <= mid) ++c2;
          });
          c2 = block_sum_int(c2, sred);
          if (c2 < mi) lo2 = mid;
          else if (c2 > KNN_CAP) hi2 = mid;
          else {
            rad2 = mid;
            break;
          }
        }
        if (it == 200) {
          if (threadIdx.x == 0) atomicOr(a.status, 1);
          return;
        }
        break;
      }
      ++r;
    }
    for_cube(a, cc, r, limit, [&](int j) {
      const double dd = sqdist_fixed(c, a.locs, j, a.d, a.w);
      if (dd <= rad2) {
        const int pos = atomicAdd(&scount, 1);
        if (pos < KNN_CAP) {
          sd[pos] = dd;
          si[pos] = j;
        }
      }
    });
    __syncthreads();
    K = min(scount, KNN_CAP);
  }
  int N = 1;
  while (N < K) N <<= 1;
  for (int j = K + threadIdx.x; j < N; j += blockDim.x) {
    sd[j] = INFINITY;
    si[j] = 0x7fffffff;
  }
  __syncthreads();
  bitonic_sort(sd, si, N);
  for (int j = threadIdx.x; j < mi; j += blockDim.x) a.nbr_idx[out0 + j] = si[j];
}

__global__ void all_previous_kernel(const int* __restrict__ block_ptr, const int* __restrict__ nbr_ptr,
                                    int* __restrict__ nbr_idx, int bc) {
  const int b = blockIdx.x;
  if (b >= bc) return;
  const int o = nbr_ptr[b], mi = nbr_ptr[b + 1] - o;
  for (int j = threadIdx.x; j < mi; j += blockDim.x) nbr_idx[o + j] = j;
}

}  // namespace bv

using namespace bv;

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

#define PCHECK(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return VECCHIA_EHIP; \
  } while (0)

namespace {
template <typename P> P* at(void* base, size_t off) { return reinterpret_cast<P*>(static_cast<char*>(base) + off); }

// rocPRIM device primitives: stable LSD radix sort of (key, value) pairs on
// bits [b0, b1), and an exclusive prefix sum of int32.  A null `tmp` asks for
// the temporary storage size in `bytes`.
template <typename K, typename V>
hipError_t radix_sort(void* tmp, size_t& bytes, const K* kin, K* kout, const V* vin, V* vout, int n, int b0, int b1,
                      hipStream_t s) {
  return rocprim::radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, (unsigned int)n, (unsigned int)b0,
                                   (unsigned int)b1, s);
}
hipError_t exclusive_sum(void* tmp, size_t& bytes, const int* in, int* out, int n, hipStream_t s) {
  return rocprim::exclusive_scan(tmp, bytes, in, out, 0, (size_t)n, rocprim::plus<int>(), s);
}

size_t sort_temp_bytes_i32_i64(int64_t n, int nbits = 32) {
  size_t sz = 0;
  (void)radix_sort((void*)nullptr, sz, (const int*)nullptr, (int*)nullptr, (const int64_t*)nullptr,
                                     (int64_t*)nullptr, (int)n, 0, nbits, (hipStream_t)0);
  return sz;
}
size_t sort_temp_bytes_i32_i32(int64_t n, int nbits = 32) {
  size_t sz = 0;
  (void)radix_sort((void*)nullptr, sz, (const int*)nullptr, (int*)nullptr, (const int*)nullptr,
                                     (int*)nullptr, (int)n, 0, nbits, (hipStream_t)0);
  return sz;
}

struct BlocksLayout {
  size_t cent, label, fsum, cnt, dist, changed, key, val, key2, val2, pol, kcnt, part, parti, sort, total;
  size_t gstart, gcur, gidx, gscan;   // centroid grid (large block counts only)
  int64_t gcells;                     // cell capacity of the grid
};
BlocksLayout blocks_layout(int64_t n, int64_t bc) {
  BlocksLayout L;
  size_t o = 0;
  L.cent = o;    o = al256(o + sizeof(double) * 3 * bc);
  L.label = o;   o = al256(o + sizeof(int) * n);
  L.fsum = o;    o = al256(o + sizeof(unsigned long long) * 3 * bc);
  L.cnt = o;     o = al256(o + sizeof(int) * bc);
  L.dist = o;    o = al256(o + sizeof(double) * n);
  L.changed = o; o = al256(o + sizeof(int) * 8);
  L.key = o;     o = al256(o + sizeof(int) * n);
  L.val = o;     o = al256(o + sizeof(int64_t) * n);
  L.key2 = o;    o = al256(o + sizeof(int) * n);
  L.val2 = o;    o = al256(o + sizeof(int64_t) * n);
  L.pol = o;     o = al256(o + sizeof(int) * bc);
  L.kcnt = o;    o = al256(o + sizeof(int) * (bc + 1));
  L.part = o;    o = al256(o + sizeof(double) * 6 * 1024);
  L.parti = o;   o = al256(o + sizeof(int64_t) * 1024);
  L.sort = o;    o = al256(o + sort_temp_bytes_i32_i64(n));
  L.gcells = 0;
  L.gstart = L.gcur = L.gidx = L.gscan = o;
  if (bc >= kKmGridMinBlocks) {
    L.gcells = 2 * bc + 64;
    L.gstart = o; o = al256(o + sizeof(int) * (L.gcells + 1));
    L.gcur = o;   o = al256(o + sizeof(int) * (L.gcells + 1));
    L.gidx = o;   o = al256(o + sizeof(int) * bc);
    size_t sc = 0;
    (void)exclusive_sum((void*)nullptr, sc, (const int*)nullptr, (int*)nullptr, (int)(L.gcells + 1),
                                     (hipStream_t)0);
    L.gscan = o;  o = al256(o + sc);
  }
  L.total = o;
  return L;
}

// Centroid grid for vecchia_blocks: cubic cells of side h over the scaled
// bounding box [lo, hi], about two centroids per cell, at most L.gcells cells.
void km_grid_setup(const BlocksLayout& L, void* ws, int64_t bc, int d, const double* lo, const double* hi, KmGrid& g) {
  memset(&g, 0, sizeof(g));
  double ext[3] = {0, 0, 0}, vol = 1.0;
  int deff = 0;
  for (int k = 0; k < 3; ++k) {
    g.lo[k] = k < d ? lo[k] : 0.0;
    ext[k] = k < d ? hi[k] - lo[k] : 0.0;
    if (ext[k] > 0) {
      vol *= ext[k];
      ++deff;
    }
  }
  const double target = std::max(1.0, (double)bc / 2.0);
  double h = deff ? std::pow(vol / target, 1.0 / deff) : 1.0;
  if (!(h > 0) || !std::isfinite(h)) h = 1.0;
  for (;;) {
    int64_t total = 1;
    for (int k = 0; k < 3; ++k) {
      const double c = ext[k] > 0 ? std::ceil(ext[k] / h) : 1.0;
      g.nc[k] = (int)std::max(1.0, std::min(c, 1e9));
      total *= g.nc[k];
      if (total > L.gcells) break;
    }
    if (total <= L.gcells) {
      g.ncell = (int)total;
      break;
    }
    h *= 1.03;   // coarsen until the cell count fits
  }
  g.h = h;
  g.inv_h = 1.0 / h;
  g.cstart = at<int>(ws, L.gstart);
  g.ccur = at<int>(ws, L.gcur);
  g.cidx = at<int>(ws, L.gidx);
}

// nearest centroid of every point: exhaustive for small block counts, through
// the centroid grid (rebuilt from the current centroids) for large ones
int km_assign(const KmArgs& a, const BlocksLayout& L, void* ws, const KmGrid* g, int first, hipStream_t s) {
  const int gn = cdiv64(a.n, 256);
  if (!g) {
    hipLaunchKernelGGL(km_assign_kernel, dim3(gn), dim3(256), 0, s, a, first);
    PCHECK(hipGetLastError());
    return VECCHIA_OK;
  }
  const int gb = cdiv64(a.bc, 256);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(cdiv64(g->ncell + 1, 256)), dim3(256), 0, s, g->ccur, g->ncell + 1, 0);
  hipLaunchKernelGGL(km_grid_count_kernel, dim3(gb), dim3(256), 0, s, a, *g);
  PCHECK(hipGetLastError());
  size_t tmp = L.total - L.gscan;
  PCHECK(exclusive_sum(at<void>(ws, L.gscan), tmp, g->ccur, g->cstart, g->ncell + 1, s));
  hipLaunchKernelGGL(km_grid_cursor_kernel, dim3(cdiv64(g->ncell + 1, 256)), dim3(256), 0, s, *g);
  hipLaunchKernelGGL(km_grid_place_kernel, dim3(gb), dim3(256), 0, s, a, *g);
  hipLaunchKernelGGL(km_assign_grid_kernel, dim3(gn), dim3(256), 0, s, a, *g, first);
  PCHECK(hipGetLastError());
  return VECCHIA_OK;
}

int bbox(const double* locs, int64_t n, int d, const double* w, double* part, double* lo, double* hi, hipStream_t s) {
  const int grid = std::min(1024, std::max(1, cdiv64(n, 256)));
  hipLaunchKernelGGL(bbox_kernel, dim3(grid), dim3(256), 0, s, locs, n, d, w[0], w[1], w[2], part);
  PCHECK(hipGetLastError());
  std::vector<double> h(6 * grid);
  PCHECK(hipMemcpyAsync(h.data(), part, sizeof(double) * 6 * grid, hipMemcpyDeviceToHost, s));
  PCHECK(hipStreamSynchronize(s));
  for (int k = 0; k < 3; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
  }
  for (int g = 0; g < grid; ++g)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], h[g * 6 + k]);
      hi[k] = std::max(hi[k], h[g * 6 + 3 + k]);
    }
  for (int k = d; k < 3; ++k) lo[k] = hi[k] = 0.0;
  return VECCHIA_OK;
}
}  // namespace

extern "C" int vecchia_permute(const double* src, int64_t n, int32_t d, const int64_t* perm, double* dst,
                               void* stream) {
  if (!src || !perm || !dst || n <= 0 || d < 1) return VECCHIA_EINVAL;
  hipLaunchKernelGGL(permute_rows_kernel, dim3(cdiv64(n, 256)), dim3(256), 0, (hipStream_t)stream, src, n, d, perm,
                     dst);
  PCHECK(hipGetLastError());
  return VECCHIA_OK;
}

extern "C" size_t vecchia_blocks_workspace_size(int64_t n, int64_t bc, int32_t d) {
  (void)d;
  if (n <= 0 || bc <= 0) return 0;
  return blocks_layout(n, bc).total;
}

extern "C" int vecchia_blocks(const double* locs, int64_t n, int32_t d, const double* metric_scale,
                              const int64_t* init_idx, const int64_t* block_perm, int64_t bc, int32_t max_iter,
                              int64_t* perm, int32_t* block_ptr, int64_t* bc_out, int32_t* iters_out,
                              void* workspace, size_t ws_bytes, void* stream) {
  if (!locs || !init_idx || !block_perm || !perm || !block_ptr || !bc_out || !workspace) return VECCHIA_EINVAL;
  if (n <= 0 || bc <= 0 || bc > n || d < 1 || d > 3 || max_iter < 0 || n >= ((int64_t)1 << 31)) return VECCHIA_EINVAL;
  const BlocksLayout L = blocks_layout(n, bc);
  if (ws_bytes < L.total) return VECCHIA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  double w[3] = {1.0, 1.0, 1.0};
  for (int k = 0; k < d; ++k) {
    w[k] = metric_scale ? metric_scale[k] : 1.0;
    if (!(w[k] > 0) || !isfinite(w[k])) return VECCHIA_EINVAL;
  }
  double lo[3], hi[3];
  int st = bbox(locs, n, d, w, at<double>(workspace, L.part), lo, hi, s);
  if (st) return st;
  double ext = 0.0;
  for (int k = 0; k < d; ++k) ext = std::max(ext, hi[k] - lo[k]);
  if (!(ext > 0)) ext = 1.0;
  KmArgs a;
  memset(&a, 0, sizeof(a));
  a.locs = locs;
  a.n = n;
  a.d = d;
  for (int k = 0; k < 3; ++k) {
    a.w[k] = w[k];
    a.lo[k] = lo[k];
  }
  // every per-cluster fixed-point sum stays below 2^62
  a.fscale = std::ldexp(1.0, 62) / ((double)n * ext * 1.0000001);
  a.bc = (int)bc;
  a.cent = at<double>(workspace, L.cent);
  a.label = at<int>(workspace, L.label);
  a.changed = at<int>(workspace, L.changed);
  a.fsum = at<unsigned long long>(workspace, L.fsum);
  a.cnt = at<int>(workspace, L.cnt);
  a.dist = at<double>(workspace, L.dist);
  const int gb = cdiv64(bc, 256), gn = cdiv64(n, 256);
  KmGrid grid;
  const KmGrid* gp = nullptr;
  if (L.gcells > 0) {
    km_grid_setup(L, workspace, bc, d, lo, hi, grid);
    gp = &grid;
  }
  hipLaunchKernelGGL(km_init_kernel, dim3(gb), dim3(256), 0, s, a, init_idx);
  PCHECK(hipGetLastError());
  st = km_assign(a, L, workspace, gp, 1, s);
  if (st) return st;
  int it = 0;
  for (; it < max_iter; ++it) {
    hipLaunchKernelGGL(km_zero_kernel, dim3(gb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, a.changed, 8, 0);
    hipLaunchKernelGGL(km_accum_kernel, dim3(gn), dim3(256), 0, s, a);
    hipLaunchKernelGGL(km_update_kernel, dim3(gb), dim3(256), 0, s, a, a.changed + 1);
    PCHECK(hipGetLastError());
    int hflags[2];
    PCHECK(hipMemcpyAsync(hflags, a.changed, sizeof(hflags), hipMemcpyDeviceToHost, s));
    PCHECK(hipStreamSynchronize(s));
    const int nempty = hflags[1];
    if (nempty > 0) {
      // re-seed each empty cluster, in cluster order, with the point farthest
      // from its updated centroid (each point at most once)
      hipLaunchKernelGGL(km_dist_kernel, dim3(gn), dim3(256), 0, s, a);
      PCHECK(hipGetLastError());
      std::vector<int> hc(bc);
      PCHECK(hipMemcpyAsync(hc.data(), a.cnt, sizeof(int) * bc, hipMemcpyDeviceToHost, s));
      PCHECK(hipStreamSynchronize(s));
      const int grid = std::min(1024, gn);
      for (int64_t c = 0; c < bc; ++c) {
        if (hc[c] != 0) continue;
        hipLaunchKernelGGL(argmax_kernel, dim3(grid), dim3(256), 0, s, a.dist, n, at<double>(workspace, L.part),
                           at<int64_t>(workspace, L.parti));
        std::vector<double> pv(grid);
        std::vector<int64_t> pi(grid);
        PCHECK(hipMemcpyAsync(pv.data(), at<double>(workspace, L.part), sizeof(double) * grid, hipMemcpyDeviceToHost, s));
        PCHECK(hipMemcpyAsync(pi.data(), at<int64_t>(workspace, L.parti), sizeof(int64_t) * grid,
                              hipMemcpyDeviceToHost, s));
        PCHECK(hipStreamSynchronize(s));
        double bv = -INFINITY;
        int64_t bi = 0;
        for (int g = 0; g < grid; ++g)
          if (pv[g] > bv || (pv[g] == bv && pi[g] < bi)) {
            bv = pv[g];
            bi = pi[g];
          }
        if (bi < 0 || bi >= n) return VECCHIA_EUNSUPPORTED;  // no point left to re-seed with
        hipLaunchKernelGGL(reseed_kernel, dim3(1), dim3(64), 0, s, a, (int)c, bi);
      }
    }
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, a.changed, 1, 0);
    st = km_assign(a, L, workspace, gp, 0, s);
    if (st) return st;
    int hch = 0;
    PCHECK(hipMemcpyAsync(&hch, a.changed, sizeof(int), hipMemcpyDeviceToHost, s));
    PCHECK(hipStreamSynchronize(s));
    if (!hch && nempty == 0) {
      ++it;
      break;
    }
  }
  if (iters_out) *iters_out = it;
  // order: stable radix sort of points by block position (ascending index inside a block)
  int* pol = at<int>(workspace, L.pol);
  int* bad = a.changed + 2;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, bad, 1, 0);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(gb), dim3(256), 0, s, pol, (int)bc, -1);
  hipLaunchKernelGGL(pos_of_label_kernel, dim3(gb), dim3(256), 0, s, block_perm, (int)bc, pol, bad);
  PCHECK(hipGetLastError());
  {
    // a block_perm that is not a permutation of 0..bc-1 stops here, before any
    // kernel uses the positions as indices
    int hbad = 0;
    PCHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    PCHECK(hipStreamSynchronize(s));
    if (hbad) return VECCHIA_EINVAL;
  }
  int* key = at<int>(workspace, L.key);
  int64_t* val = at<int64_t>(workspace, L.val);
  hipLaunchKernelGGL(pos_key_kernel, dim3(gn), dim3(256), 0, s, a.label, n, pol, key, val);
  PCHECK(hipGetLastError());
  int nbits = 1;
  while (((int64_t)1 << nbits) < bc) ++nbits;
  size_t tmp = sort_temp_bytes_i32_i64(n, nbits);
  if (L.sort + tmp > ws_bytes) return VECCHIA_ENOMEM;
  PCHECK(radix_sort(at<void>(workspace, L.sort), tmp, key, at<int>(workspace, L.key2), val,
                                            perm, (int)n, 0, nbits, s));
  int* kcnt = at<int>(workspace, L.kcnt);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(cdiv64(bc + 1, 256)), dim3(256), 0, s, kcnt, (int)bc + 1, 0);
  hipLaunchKernelGGL(count_keys_kernel, dim3(gn), dim3(256), 0, s, key, n, (int)bc, kcnt);
  PCHECK(hipGetLastError());
  std::vector<int> hk(bc);
  PCHECK(hipMemcpyAsync(hk.data(), kcnt, sizeof(int) * bc, hipMemcpyDeviceToHost, s));
  PCHECK(hipStreamSynchronize(s));
  std::vector<int> hp;
  hp.reserve(bc + 1);
  hp.push_back(0);
  for (int64_t i = 0; i < bc; ++i)
    if (hk[i] > 0) hp.push_back(hp.back() + hk[i]);
  PCHECK(hipMemcpyAsync(block_ptr, hp.data(), sizeof(int) * hp.size(), hipMemcpyHostToDevice, s));
  PCHECK(hipStreamSynchronize(s));
  *bc_out = (int64_t)hp.size() - 1;
  return VECCHIA_OK;
}

// ------------------------------------------------------------ neighbours --

namespace {
struct NbrLayout {
  size_t key, val, key2, val2, cstart, part, status, sort, total;
};
NbrLayout nbr_layout(int64_t n, int ncell) {
  NbrLayout L;
  size_t o = 0;
  L.key = o;    o = al256(o + sizeof(int) * n);
  L.val = o;    o = al256(o + sizeof(int) * n);
  L.key2 = o;   o = al256(o + sizeof(int) * n);
  L.val2 = o;   o = al256(o + sizeof(int) * n);
  L.cstart = o; o = al256(o + sizeof(int) * ((size_t)ncell + 1));
  L.part = o;   o = al256(o + sizeof(double) * 6 * 1024);
  L.status = o; o = al256(o + sizeof(int) * 8);
  L.sort = o;   o = al256(o + sort_temp_bytes_i32_i32(n));
  L.total = o;
  return L;
}
int max_cells(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(n / 2, 1), (int64_t)1 << 26); }
}  // namespace

extern "C" size_t vecchia_neighbors_workspace_size(int64_t n, int64_t bc, int32_t d, int32_t m) {
  (void)bc;
  (void)d;
  (void)m;
  if (n <= 0) return 0;
  // the grid is coarsened until it has at most max_cells(n) cells
  return nbr_layout(n, max_cells(n)).total;
}

// Neighbour search over the points of `locs` (n x d) for the blocks of
// block_ptr (device; hb is its host copy): candidates of block i are the
// points below min(hb[i], nref).
static int neighbors_impl(const double* locs, int64_t n, int32_t d, const double* w, const int32_t* block_ptr,
                          const std::vector<int>& hb, int64_t bc, int32_t m, int nref, int32_t* nbr_ptr,
                          int32_t* nbr_idx, int64_t nbr_cap, void* workspace, size_t ws_bytes, hipStream_t s) {
  // conditioning-set sizes m_i = min(m, candidates of block i)
  std::vector<int> hn(bc + 1);
  int64_t tot = 0;
  hn[0] = 0;
  for (int64_t i = 0; i < bc; ++i) {
    if (hb[i + 1] <= hb[i]) return VECCHIA_EINVAL;
    const int64_t lim = std::min<int64_t>(hb[i], nref);
    const int64_t mi = m < 0 ? lim : std::min<int64_t>(m, lim);
    tot += mi;
    if (tot >= ((int64_t)1 << 31)) return VECCHIA_ENOMEM;
    hn[i + 1] = (int)tot;
  }
  if (tot > nbr_cap) return VECCHIA_ENOMEM;
  PCHECK(hipMemcpyAsync(nbr_ptr, hn.data(), sizeof(int) * (bc + 1), hipMemcpyHostToDevice, s));
  if (m < 0) {
    hipLaunchKernelGGL(all_previous_kernel, dim3((unsigned)bc), dim3(256), 0, s, block_ptr, nbr_ptr, nbr_idx, (int)bc);
    PCHECK(hipGetLastError());
    PCHECK(hipStreamSynchronize(s));
    return VECCHIA_OK;
  }
  // uniform grid over the scaled bounding box, about two points per cell
  NbrLayout L0 = nbr_layout(n, 1);
  if (ws_bytes < L0.total) return VECCHIA_ENOMEM;
  double lo[3], hi[3];
  int st = bbox(locs, n, d, w, at<double>(workspace, L0.part), lo, hi, s);
  if (st) return st;
  double vol = 1.0;
  double extk[3];
  for (int k = 0; k < d; ++k) {
    extk[k] = std::max(hi[k] - lo[k], 1e-12);
    vol *= extk[k];
  }
  const int target = max_cells(n);
  double h = std::pow(vol / (double)target, 1.0 / d);
  GridInfo g;
  memset(&g, 0, sizeof(g));
  int64_t nc = 1;
  for (int attempt = 0; attempt < 200; ++attempt) {
    nc = 1;
    for (int k = 0; k < 3; ++k) {
      g.dims[k] = k < d ? (int)std::min<double>(std::max(1.0, std::ceil(extk[k] / h)), 4096.0) : 1;
      g.lo[k] = lo[k];
      nc *= g.dims[k];
    }
    if (nc <= target) break;
    h *= 1.03;  // coarsen until the cell count fits the workspace bound
  }
  if (nc > target) return VECCHIA_EUNSUPPORTED;
  // the cell size must cover every axis with the chosen counts
  for (int k = 0; k < d; ++k) h = std::max(h, extk[k] / g.dims[k] * (1.0 + 1e-12));
  g.h = h;
  g.inv_h = 1.0 / h;
  g.ncell = (int)nc;
  const NbrLayout L = nbr_layout(n, g.ncell);
  if (ws_bytes < L.total) return VECCHIA_ENOMEM;
  int* key = at<int>(workspace, L.key);
  int* val = at<int>(workspace, L.val);
  int* key2 = at<int>(workspace, L.key2);
  int* cell_pts = at<int>(workspace, L.val2);
  int* cstart = at<int>(workspace, L.cstart);
  hipLaunchKernelGGL(cell_key_kernel, dim3(cdiv64(n, 256)), dim3(256), 0, s, locs, n, d, w[0], w[1], w[2], g, key,
                     val);
  PCHECK(hipGetLastError());
  int nbits = 1;
  while (((int64_t)1 << nbits) < (int64_t)g.ncell + 1) ++nbits;
  size_t tmp = sort_temp_bytes_i32_i32(n, nbits);
  if (L.sort + tmp > ws_bytes) return VECCHIA_ENOMEM;
  PCHECK(radix_sort(at<void>(workspace, L.sort), tmp, key, key2, val, cell_pts, (int)n, 0,
                                            nbits, s));
  hipLaunchKernelGGL(cell_start_kernel, dim3(cdiv64(n + 1, 256)), dim3(256), 0, s, key2, n, g.ncell, cstart);
  int* status = at<int>(workspace, L.status);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, status, 8, 0);
  KnnArgs a;
  memset(&a, 0, sizeof(a));
  a.locs = locs;
  a.d = d;
  for (int k = 0; k < 3; ++k) a.w[k] = w[k];
  a.block_ptr = block_ptr;
  a.nbr_ptr = nbr_ptr;
  a.nbr_idx = nbr_idx;
  a.m = m;
  a.g = g;
  a.cell_start = cstart;
  a.cell_pts = cell_pts;
  a.status = status;
  a.nref = nref;
  hipLaunchKernelGGL(knn_kernel, dim3((unsigned)bc), dim3(KNN_T), 0, s, a, (int)bc);
  PCHECK(hipGetLastError());
  int hs = 0;
  PCHECK(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, s));
  PCHECK(hipStreamSynchronize(s));
  return hs ? VECCHIA_EUNSUPPORTED : VECCHIA_OK;
}

static int metric_weights(const double* metric_scale, int d, double* w) {
  for (int k = 0; k < 3; ++k) w[k] = 1.0;
  for (int k = 0; k < d; ++k) {
    w[k] = metric_scale ? metric_scale[k] : 1.0;
    if (!(w[k] > 0) || !isfinite(w[k])) return VECCHIA_EINVAL;
  }
  return VECCHIA_OK;
}

extern "C" int vecchia_neighbors(const double* locs_perm, int64_t n, int32_t d, const double* metric_scale,
                                 const int32_t* block_ptr, int64_t bc, int32_t m, int32_t* nbr_ptr, int32_t* nbr_idx,
                                 int64_t nbr_cap, void* workspace, size_t ws_bytes, void* stream) {
  if (!locs_perm || !block_ptr || !nbr_ptr || !nbr_idx || !workspace) return VECCHIA_EINVAL;
  if (n <= 0 || bc <= 0 || d < 1 || d > 3 || m < -1 || n >= ((int64_t)1 << 31)) return VECCHIA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  double w[3];
  if (metric_weights(metric_scale, d, w)) return VECCHIA_EINVAL;
  std::vector<int> hb(bc + 1);
  PCHECK(hipMemcpyAsync(hb.data(), block_ptr, sizeof(int) * (bc + 1), hipMemcpyDeviceToHost, s));
  PCHECK(hipStreamSynchronize(s));
  if (hb[0] != 0 || hb[bc] > n) return VECCHIA_EINVAL;
  return neighbors_impl(locs_perm, n, d, w, block_ptr, hb, bc, m, 0x7fffffff, nbr_ptr, nbr_idx, nbr_cap, workspace,
                        ws_bytes, s);
}

// Prediction: the observations and the new locations side by side in the
// workspace, the blocks shifted past the observations, every observation a
// candidate of every block.
namespace {
struct PredNbrLayout {
  size_t locs, bp, nbr, total;
};
PredNbrLayout pred_nbr_layout(int64_t n_obs, int64_t n_new, int64_t bc, int d) {
  PredNbrLayout L;
  const int64_t nt = n_obs + n_new;
  size_t o = 0;
  L.locs = o; o = al256(o + sizeof(double) * (size_t)nt * d);
  L.bp = o;   o = al256(o + sizeof(int) * (size_t)(bc + 1));
  L.nbr = o;  o = al256(o + nbr_layout(nt, max_cells(nt)).total);
  L.total = o;
  return L;
}
}  // namespace

extern "C" size_t vecchia_pred_neighbors_workspace_size(int64_t n_obs, int64_t n_new, int64_t bc, int32_t d,
                                                        int32_t m) {
  (void)m;
  if (n_obs <= 0 || n_new <= 0 || bc <= 0 || d < 1 || d > 3) return 0;
  return pred_nbr_layout(n_obs, n_new, bc, d).total;
}

extern "C" int vecchia_pred_neighbors(const double* locs_obs, int64_t n_obs, const double* locs_new, int64_t n_new,
                                      int32_t d, const double* metric_scale, const int32_t* block_ptr, int64_t bc,
                                      int32_t m, int32_t* nbr_ptr, int32_t* nbr_idx, int64_t nbr_cap,
                                      void* workspace, size_t ws_bytes, void* stream) {
  if (!locs_obs || !locs_new || !block_ptr || !nbr_ptr || !nbr_idx || !workspace) return VECCHIA_EINVAL;
  if (n_obs <= 0 || n_new <= 0 || bc <= 0 || bc > n_new || d < 1 || d > 3 || m < -1 ||
      n_obs + n_new >= ((int64_t)1 << 31))
    return VECCHIA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  double w[3];
  if (metric_weights(metric_scale, d, w)) return VECCHIA_EINVAL;
  const PredNbrLayout L = pred_nbr_layout(n_obs, n_new, bc, d);
  if (ws_bytes < L.total) return VECCHIA_ENOMEM;
  std::vector<int> hb(bc + 1);
  PCHECK(hipMemcpyAsync(hb.data(), block_ptr, sizeof(int) * (bc + 1), hipMemcpyDeviceToHost, s));
  PCHECK(hipStreamSynchronize(s));
  if (hb[0] != 0 || hb[bc] != n_new) return VECCHIA_EINVAL;
  for (int64_t i = 0; i <= bc; ++i) hb[i] += (int)n_obs;
  double* cat = at<double>(workspace, L.locs);
  int* bp = at<int>(workspace, L.bp);
  PCHECK(hipMemcpyAsync(cat, locs_obs, sizeof(double) * (size_t)n_obs * d, hipMemcpyDeviceToDevice, s));
  PCHECK(hipMemcpyAsync(cat + (size_t)n_obs * d, locs_new, sizeof(double) * (size_t)n_new * d,
                        hipMemcpyDeviceToDevice, s));
  PCHECK(hipMemcpyAsync(bp, hb.data(), sizeof(int) * (bc + 1), hipMemcpyHostToDevice, s));
  return neighbors_impl(cat, n_obs + n_new, d, w, bp, hb, bc, m, (int)n_obs, nbr_ptr, nbr_idx, nbr_cap,
                        at<void>(workspace, L.nbr), ws_bytes - L.nbr, s);
}

// ------------------------------------------------------------ block order --
// Morton, Hilbert, KD-tree and maxmin orderings of the blocks (Section 2.1)
// by their centroids.

namespace bv {

__global__ void centroids_kernel(const double* __restrict__ locs, int d, double w0, double w1, double w2,
                                 const int* __restrict__ block_ptr, int bc, double* __restrict__ cen) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  const double w[3] = {w0, w1, w2};
  double c[3];
  block_centroid(locs, d, w, block_ptr[b], block_ptr[b + 1], c);
  for (int k = 0; k < d; ++k) cen[(size_t)b * d + k] = c[k];
}

// Interleaved cell bits (axis 0 lowest) on a 2^B grid over the bounding box.
__global__ void morton_kernel(const double* __restrict__ cen, int bc, int d, double lo0, double lo1, double lo2,
                              double ex0, double ex1, double ex2, unsigned long long* __restrict__ key,
                              int64_t* __restrict__ idx) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  const int bits = d == 1 ? 63 : (d == 2 ? 32 : 21);
  const double scale = (double)(1ull << bits);
  const double lo[3] = {lo0, lo1, lo2}, ex[3] = {ex0, ex1, ex2};
  unsigned long long cell[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    const double t = floor((cen[(size_t)b * d + k] - lo[k]) / ex[k] * scale);
    cell[k] = (unsigned long long)fmin(t, scale - 1.0);
  }
  unsigned long long v = 0;
  for (int i = 0; i < bits; ++i)
    for (int k = 0; k < d; ++k) v |= ((cell[k] >> i) & 1ull) << (i * d + k);
  key[b] = v;
  idx[b] = b;
}

// Distance along the Hilbert curve of order B of the same cells (Skilling's
// transform, AIP Conf. Proc. 707, 2004): walking from the top bit down, the
// low bits are reflected (axis 0) or swapped between axis 0 and axis i,
// then Gray-encoded; the index reads the bits level by level, axis 0 most
// significant within a level.  In 1-D the curve is the cell order.
__global__ void hilbert_kernel(const double* __restrict__ cen, int bc, int d, double lo0, double lo1, double lo2,
                               double ex0, double ex1, double ex2, unsigned long long* __restrict__ key,
                               int64_t* __restrict__ idx) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  const int bits = d == 1 ? 63 : (d == 2 ? 32 : 21);
  const double scale = (double)(1ull << bits);
  const double lo[3] = {lo0, lo1, lo2}, ex[3] = {ex0, ex1, ex2};
  unsigned long long X[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    const double t = floor((cen[(size_t)b * d + k] - lo[k]) / ex[k] * scale);
    X[k] = (unsigned long long)fmin(t, scale - 1.0);
  }
  unsigned long long v = X[0];
  if (d > 1) {
    for (unsigned long long q = 1ull << (bits - 1); q > 1; q >>= 1) {
      const unsigned long long p = q - 1;
      for (int i = 0; i < d; ++i) {
        if (X[i] & q) {
          X[0] ^= p;
        } else {
          const unsigned long long t = (X[0] ^ X[i]) & p;
          X[0] ^= t;
          X[i] ^= t;
        }
      }
    }
    for (int i = 1; i < d; ++i) X[i] ^= X[i - 1];
    unsigned long long t = 0;
    for (unsigned long long q = 1ull << (bits - 1); q > 1; q >>= 1)
      if (X[d - 1] & q) t ^= q - 1;
    for (int i = 0; i < d; ++i) X[i] ^= t;
    v = 0;
    for (int l = bits - 1; l >= 0; --l)
      for (int i = 0; i < d; ++i) v = (v << 1) | ((X[i] >> l) & 1ull);
  }
  key[b] = v;
  idx[b] = b;
}

// KD-tree order, one tree level per pass (axis = level mod d): the blocks are
// sorted by their coordinate on the axis (stable, so ties keep the block
// index), then stably by the node that holds each block's current position,
// which sorts every node's blocks by coordinate; the node of a position at
// depth L follows from halving [0, bc) L times (left child: the first half,
// rounded down), so no tree is stored.
__device__ inline unsigned long long ordered_bits(double x) {
  // total order of finite doubles as unsigned integers (-0 folded into +0)
  const unsigned long long u = (unsigned long long)__double_as_longlong(x + 0.0);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}

__global__ void kd_init_kernel(int bc, int64_t* __restrict__ pos, int64_t* __restrict__ order) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  pos[b] = b;
  order[b] = b;
}

__global__ void kd_coord_kernel(const double* __restrict__ cen, int bc, int d, int axis,
                                unsigned long long* __restrict__ key, int64_t* __restrict__ idx) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= bc) return;
  key[b] = ordered_bits(cen[(size_t)b * d + axis]);
  idx[b] = b;
}

__global__ void kd_node_kernel(const int64_t* __restrict__ by_coord, const int64_t* __restrict__ pos, int bc,
                               int level, unsigned long long* __restrict__ key, int64_t* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bc) return;
  const int64_t b = by_coord[i];
  const int64_t p = pos[b];
  int64_t lo = 0, hi = bc;
  unsigned long long node = 0;
  for (int l = 0; l < level; ++l) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (p < mid) {
      hi = mid;
      node = 2 * node;
    } else {
      lo = mid;
      node = 2 * node + 1;
    }
  }
  key[i] = node;
  idx[i] = b;
}

__global__ void kd_pos_kernel(const int64_t* __restrict__ order, int bc, int64_t* __restrict__ pos) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= bc) return;
  pos[order[p]] = p;
}

// Greedy maxmin by one workgroup: the first block is the one nearest the mean
// centroid; each next one maximises the minimum squared distance to the
// blocks placed (ties: lowest index).  mind < 0 marks placed blocks.
constexpr int kMaxminThreads = 1024;
__global__ void __launch_bounds__(kMaxminThreads)
maxmin_kernel(const double* __restrict__ cen, int bc, int d, double* __restrict__ mind, int64_t* __restrict__ order,
              int steps, int* __restrict__ cur_out) {
#pragma clang fp contract(off)
  __shared__ double sv[kMaxminThreads];
  __shared__ int si[kMaxminThreads];
  __shared__ double sc[3];
  const double one[3] = {1.0, 1.0, 1.0};
  const int t = threadIdx.x;
  if (t == 0) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < bc; ++b)
      for (int k = 0; k < d; ++k) acc[k] = acc[k] + cen[(size_t)b * d + k];
    for (int k = 0; k < 3; ++k) sc[k] = k < d ? acc[k] / (double)bc : 0.0;
  }
  __syncthreads();
  // pick = argmin (first) or argmax (later) of a per-block value, ties to the lowest index
  auto reduce_pick = [&](double v, int i, bool want_max) {
    sv[t] = v;
    si[t] = i;
    __syncthreads();
    for (int s = kMaxminThreads / 2; s > 0; s >>= 1) {
      if (t < s) {
        const double a = sv[t], b = sv[t + s];
        const int ia = si[t], ib = si[t + s];
        const bool take = ib >= 0 && (ia < 0 || (want_max ? (b > a || (b == a && ib < ia)) : (b < a || (b == a && ib < ia))));
        if (take) {
          sv[t] = b;
          si[t] = ib;
        }
      }
      __syncthreads();
    }
    const int r = si[0];
    __syncthreads();
    return r;
  };
  double bv0 = INFINITY;
  int bi = -1;
  {
    const double c[3] = {sc[0], sc[1], sc[2]};
    for (int j = t; j < bc; j += kMaxminThreads) {
      const double v = sqdist_fixed(c, cen, j, d, one);
      if (bi < 0 || v < bv0) {
        bv0 = v;
        bi = j;
      }
    }
  }
  int cur = reduce_pick(bv0, bi, false);
  if (t == 0) cur_out[0] = cur;
  for (int step = 0; step < steps; ++step) {
    if (t == 0) order[step] = cur;
    if (step == steps - 1) break;
    const double c[3] = {cen[(size_t)cur * d], d > 1 ? cen[(size_t)cur * d + 1] : 0.0, d > 2 ? cen[(size_t)cur * d + 2] : 0.0};
    double best = -1.0;
    int besti = -1;
    for (int j = t; j < bc; j += kMaxminThreads) {
      double m;
      if (j == cur) {
        m = -1.0;
      } else {
        const double dj = sqdist_fixed(c, cen, j, d, one);
        const double old = mind[j];
        m = step == 0 ? dj : (old < 0.0 ? old : fmin(old, dj));
      }
      mind[j] = m;
      if (m >= 0.0 && (besti < 0 || m > best)) {
        best = m;
        besti = j;
      }
    }
    cur = reduce_pick(best, besti, true);
  }
}

// Maxmin for many blocks: one launch pair per step over the whole device.
// Step: every thread updates one block's minimum distance with the block just
// placed (cur[0]) and the workgroup's best candidate goes to part; pick: one
// workgroup reduces the parts (ties: lowest index) and places the winner.
constexpr int kMaxminStepThreads = 256;
__global__ void __launch_bounds__(kMaxminStepThreads)
maxmin_step_kernel(const double* __restrict__ cen, int bc, int d, double* __restrict__ mind,
                   const int* __restrict__ cur, int first_step, double* __restrict__ part_val,
                   int* __restrict__ part_idx) {
#pragma clang fp contract(off)
  __shared__ double sv[kMaxminStepThreads];
  __shared__ int si[kMaxminStepThreads];
  const double one[3] = {1.0, 1.0, 1.0};
  const int t = threadIdx.x, j = blockIdx.x * kMaxminStepThreads + t;
  const int c0 = cur[0];
  double m = -1.0;
  int mi = -1;
  if (j < bc) {
    if (j == c0) {
      m = -1.0;
    } else {
      const double c[3] = {cen[(size_t)c0 * d], d > 1 ? cen[(size_t)c0 * d + 1] : 0.0,
                           d > 2 ? cen[(size_t)c0 * d + 2] : 0.0};
      const double dj = sqdist_fixed(c, cen, j, d, one);
      const double old = mind[j];
      m = first_step ? dj : (old < 0.0 ? old : fmin(old, dj));
    }
    mind[j] = m;
    if (m >= 0.0) mi = j;
  }
  sv[t] = m;
  si[t] = mi;
  __syncthreads();
  for (int s = kMaxminStepThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double a = sv[t], b = sv[t + s];
      const int ia = si[t], ib = si[t + s];
      if (ib >= 0 && (ia < 0 || b > a || (b == a && ib < ia))) {
        sv[t] = b;
        si[t] = ib;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    part_val[blockIdx.x] = sv[0];
    part_idx[blockIdx.x] = si[0];
  }
}

__global__ void __launch_bounds__(kMaxminThreads)
maxmin_pick_kernel(const double* __restrict__ part_val, const int* __restrict__ part_idx, int nb,
                   int* __restrict__ cur, int64_t* __restrict__ order, int step) {
  __shared__ double sv[kMaxminThreads];
  __shared__ int si[kMaxminThreads];
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = -1;
  for (int k = t; k < nb; k += kMaxminThreads) {
    const double v = part_val[k];
    const int i = part_idx[k];
    if (i >= 0 && (bi < 0 || v > best || (v == best && i < bi))) {
      best = v;
      bi = i;
    }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int s = kMaxminThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double a = sv[t], b = sv[t + s];
      const int ia = si[t], ib = si[t + s];
      if (ib >= 0 && (ia < 0 || b > a || (b == a && ib < ia))) {
        sv[t] = b;
        si[t] = ib;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    cur[0] = si[0];
    order[step] = si[0];
  }
}

__global__ void block_sizes_kernel(const int* __restrict__ block_ptr, const int64_t* __restrict__ order, int bc,
                                   int* __restrict__ sizes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < bc) sizes[i] = block_ptr[order[i] + 1] - block_ptr[order[i]];
  if (i == bc) sizes[i] = 0;
}

__global__ void gather_blocks_kernel(const int* __restrict__ block_ptr, const int64_t* __restrict__ order,
                                     const int* __restrict__ new_ptr, int64_t* __restrict__ perm) {
  const int i = blockIdx.x;
  const int b0 = block_ptr[order[i]], l = block_ptr[order[i] + 1] - b0, o = new_ptr[i];
  for (int j = threadIdx.x; j < l; j += blockDim.x) perm[o + j] = b0 + j;
}

}  // namespace bv

namespace {
struct OrderLayout {
  size_t cen, key, key2, idx, idx2, mind, sizes, pval, pidx, part, sort, scan, total;
};
OrderLayout order_layout(int64_t bc, int d) {
  OrderLayout L;
  size_t o = 0;
  L.cen = o;   o = al256(o + sizeof(double) * (size_t)bc * d);
  L.key = o;   o = al256(o + sizeof(unsigned long long) * (size_t)bc);
  L.key2 = o;  o = al256(o + sizeof(unsigned long long) * (size_t)bc);
  L.idx = o;   o = al256(o + sizeof(int64_t) * (size_t)bc);
  L.idx2 = o;  o = al256(o + sizeof(int64_t) * (size_t)bc);
  L.mind = o;  o = al256(o + sizeof(double) * (size_t)bc);
  L.sizes = o; o = al256(o + sizeof(int) * (size_t)(bc + 1));
  L.pval = o;  o = al256(o + sizeof(double) * (size_t)(bc / kMaxminStepThreads + 1));
  L.pidx = o;  o = al256(o + sizeof(int) * (size_t)(bc / kMaxminStepThreads + 1) + 64);
  L.part = o;  o = al256(o + sizeof(double) * 6 * 1024);
  size_t st = 0, sc = 0;
  (void)radix_sort((void*)nullptr, st, (const unsigned long long*)nullptr,
                                     (unsigned long long*)nullptr, (const int64_t*)nullptr, (int64_t*)nullptr,
                                     (int)bc, 0, 64, (hipStream_t)0);
  (void)exclusive_sum((void*)nullptr, sc, (const int*)nullptr, (int*)nullptr, (int)(bc + 1),
                                   (hipStream_t)0);
  L.sort = o;  o = al256(o + st);
  L.scan = o;  o = al256(o + sc);
  L.total = o;
  return L;
}
}  // namespace

extern "C" size_t vecchia_reorder_blocks_workspace_size(int64_t n, int64_t bc, int32_t d) {
  (void)n;
  if (bc <= 0 || d < 1 || d > 3) return 0;
  return order_layout(bc, d).total;
}

extern "C" int vecchia_reorder_blocks(const double* locs_perm, int64_t n, int32_t d, const double* metric_scale,
                                      const int32_t* block_ptr, int64_t bc, int32_t method, int64_t* block_order,
                                      int64_t* point_perm, int32_t* block_ptr_out, void* workspace, size_t ws_bytes,
                                      void* stream) {
  if (!locs_perm || !block_ptr || !block_order || !point_perm || !block_ptr_out || !workspace) return VECCHIA_EINVAL;
  if (n <= 0 || bc <= 0 || bc > n || d < 1 || d > 3 || n >= ((int64_t)1 << 31)) return VECCHIA_EINVAL;
  if (method != VECCHIA_ORDER_MORTON && method != VECCHIA_ORDER_MAXMIN && method != VECCHIA_ORDER_HILBERT &&
      method != VECCHIA_ORDER_KDTREE)
    return VECCHIA_EINVAL;
  double w[3];
  if (metric_weights(metric_scale, d, w)) return VECCHIA_EINVAL;
  const OrderLayout L = order_layout(bc, d);
  if (ws_bytes < L.total) return VECCHIA_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  double* cen = at<double>(workspace, L.cen);
  const int ib = (int)bc;
  hipLaunchKernelGGL(centroids_kernel, dim3(cdiv64(bc, 256)), dim3(256), 0, s, locs_perm, d, w[0], w[1], w[2],
                     block_ptr, ib, cen);
  PCHECK(hipGetLastError());
  int64_t* order = block_order;
  if (method == VECCHIA_ORDER_MORTON || method == VECCHIA_ORDER_HILBERT) {
    const double one[3] = {1.0, 1.0, 1.0};
    double lo[3], hi[3], ex[3];
    int st = bbox(cen, bc, d, one, at<double>(workspace, L.part), lo, hi, s);
    if (st) return st;
    for (int k = 0; k < 3; ++k) ex[k] = (k < d && hi[k] > lo[k]) ? hi[k] - lo[k] : 1.0;
    unsigned long long* key = at<unsigned long long>(workspace, L.key);
    int64_t* idx = at<int64_t>(workspace, L.idx);
    hipLaunchKernelGGL(method == VECCHIA_ORDER_MORTON ? morton_kernel : hilbert_kernel, dim3(cdiv64(bc, 256)),
                       dim3(256), 0, s, cen, ib, d, lo[0], lo[1], lo[2], ex[0], ex[1], ex[2], key, idx);
    PCHECK(hipGetLastError());
    size_t tmp = L.scan - L.sort;
    // radix sort is stable: equal keys keep the ascending block index
    PCHECK(radix_sort(at<void>(workspace, L.sort), tmp, key,
                                              at<unsigned long long>(workspace, L.key2), idx, order, ib, 0, 64, s));
  } else if (method == VECCHIA_ORDER_KDTREE) {
    unsigned long long* key = at<unsigned long long>(workspace, L.key);
    unsigned long long* key2 = at<unsigned long long>(workspace, L.key2);
    int64_t* idx = at<int64_t>(workspace, L.idx);
    int64_t* idx2 = at<int64_t>(workspace, L.idx2);
    int64_t* pos = at<int64_t>(workspace, L.mind);   // bc slots of 8 bytes
    const unsigned g = (unsigned)cdiv64(bc, 256);
    hipLaunchKernelGGL(kd_init_kernel, dim3(g), dim3(256), 0, s, ib, pos, order);
    PCHECK(hipGetLastError());
    int levels = 0;
    while (((int64_t)1 << levels) < bc) ++levels;
    for (int level = 0; level < levels; ++level) {
      size_t tmp = L.scan - L.sort;
      hipLaunchKernelGGL(kd_coord_kernel, dim3(g), dim3(256), 0, s, cen, ib, d, level % d, key, idx);
      PCHECK(hipGetLastError());
      PCHECK(radix_sort(at<void>(workspace, L.sort), tmp, key, key2, idx, idx2, ib, 0, 64, s));
      hipLaunchKernelGGL(kd_node_kernel, dim3(g), dim3(256), 0, s, idx2, pos, ib, level, key, idx);
      PCHECK(hipGetLastError());
      tmp = L.scan - L.sort;
      PCHECK(radix_sort(at<void>(workspace, L.sort), tmp, key, key2, idx, order, ib, 0, 64, s));
      hipLaunchKernelGGL(kd_pos_kernel, dim3(g), dim3(256), 0, s, order, ib, pos);
      PCHECK(hipGetLastError());
    }
  } else {
    // up to 8192 blocks one workgroup does every step; above, one launch pair
    // per step spreads the O(bc) distance updates over the device
    double* mind = at<double>(workspace, L.mind);
    double* pval = at<double>(workspace, L.pval);
    int* pidx = at<int>(workspace, L.pidx);
    int* cur = pidx + (bc / kMaxminStepThreads + 1);
    const bool one_wg = bc <= 8192;
    hipLaunchKernelGGL(maxmin_kernel, dim3(1), dim3(kMaxminThreads), 0, s, cen, ib, d, mind, order,
                       one_wg ? ib : 1, cur);
    PCHECK(hipGetLastError());
    if (!one_wg) {
      const int nb = cdiv64(bc, kMaxminStepThreads);
      for (int step = 1; step < ib; ++step) {
        hipLaunchKernelGGL(maxmin_step_kernel, dim3(nb), dim3(kMaxminStepThreads), 0, s, cen, ib, d, mind, cur,
                           step == 1 ? 1 : 0, pval, pidx);
        hipLaunchKernelGGL(maxmin_pick_kernel, dim3(1), dim3(kMaxminThreads), 0, s, pval, pidx, nb, cur, order, step);
      }
      PCHECK(hipGetLastError());
    }
  }
  int* sizes = at<int>(workspace, L.sizes);
  hipLaunchKernelGGL(block_sizes_kernel, dim3(cdiv64(bc + 1, 256)), dim3(256), 0, s, block_ptr, order, ib, sizes);
  PCHECK(hipGetLastError());
  size_t stmp = L.total - L.scan;
  PCHECK(exclusive_sum(at<void>(workspace, L.scan), stmp, sizes, block_ptr_out, ib + 1, s));
  hipLaunchKernelGGL(gather_blocks_kernel, dim3(ib), dim3(64), 0, s, block_ptr, order, block_ptr_out, point_perm);
  PCHECK(hipGetLastError());
  return VECCHIA_OK;
}
