// One-wave matrix-core kernels for the per-block chain of Alg. 1.
//
// A single wave (64 lanes, the whole workgroup) evaluates one block for one
// theta.  The bordered joint matrix [[K_J, .], [y_J^T, .]] (p + 1 rows, padded
// to P = 16 G with identity) lives in the wave's accumulator registers as the
// G (G + 1) / 2 lower-triangular 16 x 16 tiles of the v_mfma_*_16x16x4
// instructions; every lane generates its own Matern entries.  With the tile
// loops unrolled (G is a template parameter) every tile index is static, so
// the matrix never leaves the register file.
//
// Factorisation: right-looking Cholesky in panels of four columns.  Per panel,
// the lanes holding its columns write them to LDS; every lane factors the
// 4 x 4 diagonal block (all lanes compute the same values in lockstep, so the
// redundancy costs nothing); each lane solves up to ceil((P - 16 K) / 64)
// panel rows (the TRSM / TRSV of Alg. 1; the border row becomes
// w = L^-1 y_J); the trailing tiles take one rank-4 MFMA each (the Schur
// update).  Workgroup barriers of a single wave reduce to LDS fences, so a
// panel costs no cross-wave synchronisation.  Pivots d_k and border entries
// w_k (k >= m) give log det and the quadratic form, summed in FP64.
//
// Adjoint (MODE 1): the finished factor columns are restored into the tiles,
// then X = L^-T [ w | [z; 0] | [0; I_l] ] is solved tile row by tile row
// (16-row triangular solve per right-hand side, MFMA updates of the rows
// above), and W = alpha alpha^T - b b^T - X_R X_R^T is formed tile by tile with
// MFMA and contracted against dK regenerated entry by entry (FP64 sums):
// d l_i = 1/2 <W, dK>.
#pragma once

#include <utility>

#include "internal.hpp"

namespace bv {

// Compile-time loops: the body receives std::integral_constant<int, i>, so
// accumulator tile indices are constants whatever the unroller decides.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
template <int B, int E, typename F>  // E - 1 down to B
__device__ __forceinline__ void static_for_down(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, E - 1>{});
    static_for_down<B, E - 1>(f);
  }
}
#define BV_CI(name) [&](auto name##_c) __attribute__((always_inline))
#define BV_CV(name) constexpr int name = decltype(name##_c)::value

typedef float w32x4_t __attribute__((ext_vector_type(4)));
typedef double w64x4_t __attribute__((ext_vector_type(4)));

template <typename T> struct WMma;
template <> struct WMma<float> {
  typedef w32x4_t acc;
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // tile row held by accumulator register r of lane group g
  static __device__ __forceinline__ constexpr int row(int g, int r) { return 4 * g + r; }
  static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
};
template <> struct WMma<double> {
  typedef w64x4_t acc;
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int g, int r) { return g + 4 * r; }
  static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / sqrt(x); }
};

// lower-triangular tile (I, J), J <= I, in row-major packed order
__host__ __device__ constexpr int tix(int I, int J) { return I * (I + 1) / 2 + J; }

__host__ __device__ constexpr int wave_lds_elems(int G, int mode) {
  // su (3 P), sy, sdk, swk (P each), then the panel (4 P) or, for the adjoint,
  // one chunk of right-hand sides (P x (kWaveChunk + 1)), a published tile
  // row of L (16 x P) and the reciprocals of its diagonal (16)
  return 6 * 16 * G + (mode == 0 ? 4 * 16 * G : 16 * G * (kWaveChunk + 1) + 16 * 16 * G + 16);
}

// Two waves per SIMD where the register file holds them without spilling
// (FP32 up to G = 9); one otherwise.
template <typename T, int G>
constexpr int wave_min_waves() { return sizeof(T) == 4 && G <= 9 ? 2 : 1; }

template <typename T, int G, int MODE>
__global__ void __launch_bounds__(64, (wave_min_waves<T, G>())) bv_wave_kernel(AdjArgs a, ThetaPack thp) {
  constexpr int P = 16 * G;
  constexpr int NT = G * (G + 1) / 2;
  typedef WMma<T> M;
  typedef typename M::acc acc_t;
  extern __shared__ __align__(16) unsigned char smem[];
  T* su = reinterpret_cast<T*>(smem);  // scaled coordinates relative to the block's first point, su[k * P + i]
  T* sy = su + 3 * P;                  // border row y_J
  T* sdk = sy + P;                     // pivots d_k
  T* swk = sdk + P;                    // border entries w_k
  T* work = swk + P;

  const int ln = threadIdx.x, lr = ln & 15, lg = ln >> 4;
  const int total = a.list ? *a.list_count : a.nsched * a.ntheta;
  const int wi = blockIdx.x + a.item_base;
  if (wi >= total) return;
  int b, tt;
  if (a.list) {
    const int e = a.list[wi];
    tt = e / a.bc;
    b = e - tt * a.bc;
  } else {
    tt = wi / a.nsched;
    b = a.sched[wi - tt * a.nsched];
  }
  const ThetaDev& th = thp.t[tt];
  const int b0 = a.block_ptr[b], b1 = a.block_ptr[b + 1];
  const int n0 = a.nbr_ptr[b], n1 = a.nbr_ptr[b + 1];
  const int l = b1 - b0, m = n1 - n0, p = m + l;

  for (int i = ln; i < P; i += 64) {
    if (i < p) {
      const int g = (i < m) ? a.nbr_idx[n0 + i] : (b0 + i - m);
      sy[i] = T(a.y[g]);
      for (int k = 0; k < 3; ++k)
        su[k * P + i] = k < a.d ? T((a.locs[(size_t)g * a.d + k] - a.locs[(size_t)b0 * a.d + k]) * th.inv_scale[k]) : T(0);
    } else {
      sy[i] = T(0);
      for (int k = 0; k < 3; ++k) su[k * P + i] = T(0);
    }
  }
  __syncthreads();

  // ---- generate the bordered joint matrix in the accumulator tiles ----------
  const T sig2 = T(th.sigma2), nug = T(th.nugget);
  const MaternCoef<T> mc(th.nu_code);
  acc_t acc[NT];
  static_for<0, G>(BV_CI(I) {
    BV_CV(I);
    T ri[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I * 16 + M::row(lg, r);
      ri[r][0] = su[i];
      ri[r][1] = su[P + i];
      ri[r][2] = su[2 * P + i];
    }
    static_for<0, I + 1>(BV_CI(J) {
      BV_CV(J);
      const int j = J * 16 + lr;
      const T sj0 = su[j], sj1 = su[P + j], sj2 = su[2 * P + j];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * 16 + M::row(lg, r);
        const T dx = ri[r][0] - sj0, dy = ri[r][1] - sj1, dz = ri[r][2] - sj2;
        const T x = sqrt_fast<T>(dx * dx + dy * dy + dz * dz);
        T v = sig2 * mc.rho(x) + ((i == j) ? nug : T(0));
        if (!(i < p && j < p)) v = (i == j) ? T(1) : T(0);
        acc[tix(I, J)][r] = v;
      }
      if (I == (p >> 4)) {  // border row p: y_J
        const T yb = sy[j];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (I * 16 + M::row(lg, r) == p && j < p) acc[tix(I, J)][r] = yb;
      }
      // D = 0 * 0 + C: hands the finished tile to the accumulator registers now,
      // so the generated values do not pile up in VGPRs until the first update
      acc[tix(I, J)] = M::op(T(0), T(0), acc[tix(I, J)]);
    });
  });

  // ---- factorisation, four columns per step -----------------------------------
  T* pan = work;  // pan[c * P + row], c < 4
  static_for<0, G>(BV_CI(K) {
    BV_CV(K);
    if (K * 16 >= p) return;
#pragma nounroll
    for (int c0 = 0; c0 < 16; c0 += 4) {
      const int k0 = K * 16 + c0;
      if (k0 >= p) break;
      if (lr >= c0 && lr < c0 + 4) {
        static_for<K, G>(BV_CI(I) {
          BV_CV(I);
#pragma unroll
          for (int r = 0; r < 4; ++r) pan[(lr - c0) * P + I * 16 + M::row(lg, r)] = acc[tix(I, K)][r];
        });
      }
      __syncthreads();
      // 4 x 4 diagonal block (same values in every lane)
      T Ld[4][4], rinv[4], piv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) Ld[r][c] = r >= c ? pan[c * P + k0 + r] : T(0);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool real = k0 + c < p;
        T dsum = Ld[c][c];
#pragma unroll
        for (int j = 0; j < c; ++j) dsum -= Ld[c][j] * Ld[c][j];
        piv[c] = real ? dsum : T(1);
        const T ri = real ? M::rsqrt(dsum) : T(1);
        rinv[c] = ri;
        Ld[c][c] = real ? dsum * ri : T(1);
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
          T v = Ld[r][c];
#pragma unroll
          for (int j = 0; j < c; ++j) v -= Ld[r][j] * Ld[c][j];
          Ld[r][c] = real ? v * ri : T(0);
        }
      }
      // panel rows of tile K and below: zero above the block, L_dd in it, TRSM below
#pragma unroll
      for (int q = 0; q < (P - K * 16 + 63) / 64; ++q) {
        const int i = K * 16 + ln + 64 * q;
        if (i < P) {
          // branch-free: every lane runs the substitution, then rows above the
          // block take zero and rows inside it take L_dd
          const int di = i - k0;
          T x[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            T v = pan[c * P + i];
#pragma unroll
            for (int j = 0; j < c; ++j) v -= x[j] * Ld[c][j];
            const T t = (k0 + c < p) ? v * rinv[c] : T(0);
            T v2 = t;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) v2 = di == rr ? Ld[rr][c] : v2;
            x[c] = di < 0 ? T(0) : v2;
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) pan[c * P + i] = x[c];
          if (i == p) {
#pragma unroll
            for (int c = 0; c < 4; ++c) swk[k0 + c] = x[c];
          }
        }
      }
      if (ln == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sdk[k0 + c] = piv[c];
      }
      __syncthreads();
      // rank-4 update of the trailing tiles: D -= L_I L_J^T
      T v[G];
      static_for<K, G>(BV_CI(I) {
        BV_CV(I);
        v[I] = pan[lg * P + I * 16 + lr];
      });
      static_for<K, G>(BV_CI(I) {
        BV_CV(I);
        const T nv = -v[I];
        static_for<K, I + 1>(BV_CI(J) {
          BV_CV(J);
          acc[tix(I, J)] = M::op(nv, v[J], acc[tix(I, J)]);
        });
      });
      if (MODE != 0 && lr >= c0 && lr < c0 + 4) {
        // keep the finished factor columns in the tiles
        static_for<K, G>(BV_CI(I) {
          BV_CV(I);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[tix(I, K)][r] = pan[(lr - c0) * P + I * 16 + M::row(lg, r)];
        });
      }
      __syncthreads();
    }
  });

  // ---- log-determinant, quadratic form and pivot guard (FP64) -----------------
  const double guard = a.fp32_guard == 2 ? INFINITY
      : a.fp32_guard ? fmax(0.5 * th.nugget, (double)p * 1.1920928955078125e-07 * (th.sigma2 + th.nugget))
      : 0.0;
  double acc_ll = 0.0;
  int flag = 0;
  for (int k = ln; k < p; k += 64) {
    const double dd = (double)sdk[k];
    if (!(dd > guard)) flag |= a.fp32_guard ? 1 : 2;
    if (!(dd > 0.0)) flag |= 2;
    if (k >= m) {
      const double wk = (double)swk[k];
      acc_ll += log(dd) + wk * wk;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc_ll += __shfl_down(acc_ll, off, 64);
    flag |= __shfl_down(flag, off, 64);
  }
  const size_t o = (size_t)tt * a.bc + b;
  if (MODE == 0) {
    if (ln == 0) {
      a.partial[o] = (flag & 2) && !a.fp32_guard ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
      a.flag[o] = flag | a.flag_or;
    }
    return;
  }
  // the factor leaves the registers for this item's slot of the tile buffer
  // (accumulator order, 256 elements per tile); the adjoint reads it back one
  // tile row at a time, so its phases do not hold the tiles in registers
  T* Lg = reinterpret_cast<T*>(a.tiles) + (size_t)(wi - a.item_base) * (NT * 256);
  static_for<0, NT>(BV_CI(t) {
    BV_CV(t);
#pragma unroll
    for (int r = 0; r < 4; ++r) Lg[t * 256 + ln * 4 + r] = acc[t][r];
  });
  __syncthreads();

  // ---- adjoint: X <- L^-T X and the contraction, kWaveChunk right-hand sides at a time
  // (the factor stays in the tiles, so a chunk only repeats the triangular solves)
  constexpr int LDX = kWaveChunk + 1;
  const int nr = l + 2;
  T* X = work;               // X[row * LDX + col], one chunk of right-hand sides
  T* lrow = work + P * LDX;  // published tile row of L, lrow[r * P + col]
  T* rdiag = lrow + 16 * P;  // reciprocals of its diagonal
  const int Ip = p >> 4, rp = p & 15;
  const int Gp = (p + 15) >> 4;
  const T irange = T(th.inv_range);
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int cb = 0; cb < nr; cb += kWaveChunk) {
    const int nc = nr - cb < kWaveChunk ? nr - cb : kWaveChunk;
    const int nq = (nc + 15) >> 4;
    __syncthreads();
    for (int e = ln; e < P * LDX; e += 64) X[e] = T(0);
    __syncthreads();
    // column cb + c of [ w | [z; 0] | [0; I_l] ]
    for (int c = ln; c < nc; c += 64)
      if (cb + c >= 2) X[(m + cb + c - 2) * LDX + c] = T(1);
    if (cb == 0) {
      for (int J = 0; J <= Ip; ++J) {
        const int j = J * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (M::row(lg, r) == rp && j < p) {
            const T v = Lg[tix(Ip, J) * 256 + ln * 4 + r];
            X[j * LDX] = v;                  // w
            if (j < m) X[j * LDX + 1] = v;   // [z; 0]
          }
      }
    }
    __syncthreads();
    for (int K = Gp - 1; K >= 0; --K) {
      // publish tile row K of L (only this step indexes the tiles)
      for (int J = 0; J <= K; ++J)
#pragma unroll
        for (int r = 0; r < 4; ++r) lrow[M::row(lg, r) * P + J * 16 + lr] = Lg[tix(K, J) * 256 + ln * 4 + r];
      {
        __syncthreads();
        if (K == Gp - 1) {
          // the tiles hold L (zeros above the diagonal) on rows and columns < p;
          // the border row and the padding become identity rows here
          for (int e = ln; e < 16 * (K + 1) * 16; e += 64) {
            const int rw = e / (16 * (K + 1)), j = e - rw * 16 * (K + 1), i = K * 16 + rw;
            if (i >= p || j >= p) lrow[rw * P + j] = (i == j) ? T(1) : T(0);
          }
          __syncthreads();
        }
        if (ln < 16) rdiag[ln] = T(1) / lrow[ln * P + K * 16 + ln];
        __syncthreads();
        // diagonal tile: X_K <- L_KK^-T X_K, one lane per right-hand side
        if (ln < nc) {
          T x[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) x[r] = X[(K * 16 + r) * LDX + ln];
          // column-oriented: finish x[rr], then remove it from the rows above
#pragma unroll
          for (int rr = 15; rr >= 0; --rr) {
            x[rr] = x[rr] * rdiag[rr];
#pragma unroll
            for (int r2 = 0; r2 < rr; ++r2) x[r2] -= lrow[rr * P + K * 16 + r2] * x[rr];
            // compiler-only memory barrier: keeps the next row's L_KK loads from being
            // hoisted above this step (bounds the registers they occupy)
            __asm__ volatile("" ::: "memory");
          }
#pragma unroll
          for (int r = 0; r < 16; ++r) X[(K * 16 + r) * LDX + ln] = x[r];
        }
        __syncthreads();
        // rows above: X_J -= L_KJ^T X_K
        for (int J = 0; J < K; ++J)
          for (int q = 0; q < nq; ++q) {
            acc_t c;
#pragma unroll
            for (int r = 0; r < 4; ++r) c[r] = X[(J * 16 + M::row(lg, r)) * LDX + q * 16 + lr];
#pragma unroll
            for (int sub = 0; sub < 4; ++sub) {
              const T av = -lrow[(4 * sub + lg) * P + J * 16 + lr];
              const T bv = X[(K * 16 + 4 * sub + lg) * LDX + q * 16 + lr];
              c = M::op(av, bv, c);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) X[(J * 16 + M::row(lg, r)) * LDX + q * 16 + lr] = c[r];
          }
        __syncthreads();
      }
    }

    // W = alpha alpha^T - b b^T - X_R X_R^T (this chunk's columns), contracted with dK
    const int nk = (nc + 3) >> 2;
    for (int I = 0; I < Gp; ++I)
      for (int J = 0; J <= I; ++J) {
        acc_t c;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = T(0);
        const int iI = I * 16, jJ = J * 16;
        for (int kq = 0; kq < nk; ++kq) {
          const int q = 4 * kq + lg;
          const T sg = cb + q == 0 ? T(1) : T(-1);
          c = M::op(sg * X[(iI + lr) * LDX + q], X[(jJ + lr) * LDX + q], c);
        }
        // the tile's four entries in T, then FP64 across tiles and lanes
        T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = iI + M::row(lg, r), j = jJ + lr;
          if (i < p && j < p) {
            const T dx = su[i] - su[j];
            const T dy = su[P + i] - su[P + j];
            const T dz = su[2 * P + i] - su[2 * P + j];
            const T x = sqrt_fast<T>(dx * dx + dy * dy + dz * dz);
            T rho, drho;
            mc.rho_drange(x, irange, rho, drho);
            s0 += c[r] * rho;
            s1 += c[r] * drho;
            if (i == j) s2 += c[r];
          }
        }
        const double wgt = I == J ? 1.0 : 2.0;
        g0 += wgt * (double)s0;
        g1 += wgt * (double)s1;
        g2 += (double)s2;
      }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    g0 += __shfl_down(g0, off, 64);
    g1 += __shfl_down(g1, off, 64);
    g2 += __shfl_down(g2, off, 64);
  }
  if (ln == 0) {
    const bool bad = (flag & 2) && !a.fp32_guard;
    a.partial[o] = bad ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
    a.gpart[3 * o + 0] = bad ? __builtin_nan("") : 0.5 * g0;
    a.gpart[3 * o + 1] = bad ? __builtin_nan("") : 0.5 * th.sigma2 * g1;
    a.gpart[3 * o + 2] = bad ? __builtin_nan("") : 0.5 * g2;
    a.flag[o] = flag | a.flag_or;
  }
}

template <typename T, int G, int MODE>
static hipError_t launch_wave_g(const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  const size_t lds = sizeof(T) * (size_t)wave_lds_elems(G, MODE);
  hipLaunchKernelGGL((bv_wave_kernel<T, G, MODE>), dim3(grid), dim3(64), lds, s, a, thp);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_wave_t(int g, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  switch (g) {
    case 1: return launch_wave_g<T, 1, MODE>(a, thp, grid, s);
    case 2: return launch_wave_g<T, 2, MODE>(a, thp, grid, s);
    case 3: return launch_wave_g<T, 3, MODE>(a, thp, grid, s);
    case 4: return launch_wave_g<T, 4, MODE>(a, thp, grid, s);
    case 5: return launch_wave_g<T, 5, MODE>(a, thp, grid, s);
    case 6: return launch_wave_g<T, 6, MODE>(a, thp, grid, s);
    case 7: return launch_wave_g<T, 7, MODE>(a, thp, grid, s);
    case 8: return launch_wave_g<T, 8, MODE>(a, thp, grid, s);
    case 9: return launch_wave_g<T, 9, MODE>(a, thp, grid, s);
    case 10: return launch_wave_g<T, 10, MODE>(a, thp, grid, s);
    case 11: return launch_wave_g<T, 11, MODE>(a, thp, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bv
