// Blocks whose joint size exceeds the register capacity (m_i + l_i > 175), e.g.
// conditioning on every earlier point.  One workgroup (four waves) per block:
// the bordered matrix [[K_J, .], [y_J^T, .]] (p + 1 rows, padded with identity to
// P = 16 G) is generated into a global workspace (column-major, lower part),
// then factored left-looking in 16-column panels:
//   C_IJ = A_IJ - sum_{K<J} L_IK L_JK^T      (MFMA, one output tile per wave at a time)
//   L_JJ = chol(C_JJ)                        (one wave, rows in lane registers)
//   L_IJ = C_IJ L_JJ^-T                      (one thread per row)
// The matrix is generated with each thread owning a row and the columns staged
// in LDS.  The log-determinant and quadratic form come from the panel pivots
// and the border row, as in the register kernels.  Operands stream through L2: about
// P^3 / 96 elements are read per block.  The gradient variant then
// back-substitutes the right-hand sides [w | [w_N; 0] | [0; I_l]] through L^T
// tile row by tile row (16 x 16 triangular solves, MFMA updates of the rows
// above) and contracts W with d K / d range regenerated from the staged
// coordinates, as the one-wave kernels do.
#include "internal.hpp"

namespace bv {

typedef float lf32x4_t __attribute__((ext_vector_type(4)));
typedef double lf64x4_t __attribute__((ext_vector_type(4)));

template <typename T> struct LMma;
template <> struct LMma<float> {
  typedef lf32x4_t acc;
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // tile row held by accumulator register r of lane group g (the FP32 and
  // FP64 16x16x4 instructions interleave their output rows differently)
  static __device__ __forceinline__ constexpr int row(int g, int r) { return 4 * g + r; }
};
template <> struct LMma<double> {
  typedef lf64x4_t acc;
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int g, int r) { return g + 4 * r; }
};

// Orders one wave's LDS accesses across its lanes: a wavefront-scope fence
// keeps the compiler from moving loads and stores across it (the hardware
// already processes a wave's LDS operations in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Value of v held by lane `lane` (a compile-time or wave-uniform index).
template <typename T> __device__ __forceinline__ T lane_read(T v, int lane);
template <> __device__ __forceinline__ float lane_read<float>(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
template <> __device__ __forceinline__ double lane_read<double>(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Per-block slot layout (elements of T, P = 16 G for the block's own p):
// the bordered matrix, column-major lower part, P x P; in gradient launches
// the right-hand sides X (P rows, 16 ceil((l + 2) / 16) columns, column-major)
// follow it; then the scaled coordinates of the p points (3 x P).
// Waves per SIMD at least: FP32 6 (80 VGPRs, 6 workgroups of 4 waves per
// compute unit, up to 1536 blocks in flight hiding each other's latency);
// FP64 4 (128 VGPRs), which holds two output tiles per wave in the panel
// update (each load of the panel operand feeds two products)
#ifndef BV_LARGE_WAVES32
#define BV_LARGE_WAVES32 6
#endif
#ifndef BV_LARGE_WAVES64
#define BV_LARGE_WAVES64 4
#endif
#ifndef BV_LARGE_TPW64
#define BV_LARGE_TPW64 2    // FP64 output tiles per wave in one pass of the panel update
#endif
#ifndef BV_LARGE_DEPTH32
#define BV_LARGE_DEPTH32 2  // panel-update steps whose operand loads are issued together
#endif
#ifndef BV_LARGE_DEPTH64
#define BV_LARGE_DEPTH64 2
#endif
template <typename T, bool GRAD>
__global__ void __launch_bounds__(256, sizeof(T) == 8 ? BV_LARGE_WAVES64 : BV_LARGE_WAVES32)
    bv_large_kernel(LargeArgs a, ThetaPack thp) {
  constexpr int TPW = sizeof(T) == 8 ? BV_LARGE_TPW64 : 1;
  constexpr int DEPTH = sizeof(T) == 8 ? BV_LARGE_DEPTH64 : BV_LARGE_DEPTH32;
  typedef typename LMma<T>::acc acc_t;
  __shared__ T dtile[16][17];
  __shared__ T colc[4][256];   // generation: coordinates and y of 256 columns
  __shared__ double sred[2][256];
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63, lr = ln & 15, lg = ln >> 4;
  const int total = a.list ? *a.list_count : a.nsched * a.ntheta;
  T* M = reinterpret_cast<T*>(a.ws) + (size_t)blockIdx.x * a.slot_elems;
  for (int wi = blockIdx.x; wi < total; wi += gridDim.x) {
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
    const int G = (p + 1 + 15) >> 4, P = 16 * G;
    const size_t ld = (size_t)P;
    const int nr = l + 2, NRP = 16 * ((nr + 15) >> 4);   // right-hand sides, padded to whole tiles
    T* X = M + ld * ld;
    T* cs = GRAD ? X + ld * NRP : X;                      // cs[k * P + i]: scaled coordinates
    const int d = a.d;
    const MaternCoef<T> mc(th.nu_code);
    const T sig2 = T(th.sigma2), nug = T(th.nugget);
    // ---- scaled coordinates relative to the block's first point -------------
    __syncthreads();
    for (int i = tid; i < P; i += 256) {
      const int gi = i < m ? a.nbr_idx[n0 + i] : (b0 + i - m);
      for (int k = 0; k < 3; ++k)
        cs[k * ld + i] = (i < p && k < d) ? T((a.locs[(size_t)gi * d + k] - a.locs[(size_t)b0 * d + k]) * th.inv_scale[k])
                                          : T(0);
    }
    __syncthreads();
    // ---- generate the lower part: each thread owns a row (its coordinates in
    // registers) and walks the columns, staged 256 at a time in LDS with their
    // y values; for a fixed column the stores of a wave are contiguous -------
    for (int ib = 0; ib < P; ib += 256) {
      const int i = ib + tid;
      const T ci0 = i < P ? cs[i] : T(0), ci1 = i < P ? cs[ld + i] : T(0), ci2 = i < P ? cs[2 * ld + i] : T(0);
      for (int jb = 0; jb <= ib; jb += 256) {
        __syncthreads();
        {
          const int j = jb + tid;
          if (j < P) {
            colc[0][tid] = cs[j];
            colc[1][tid] = cs[ld + j];
            colc[2][tid] = cs[2 * ld + j];
            colc[3][tid] = j < p ? T(a.y[j < m ? a.nbr_idx[n0 + j] : (b0 + j - m)]) : T(0);
          }
        }
        __syncthreads();
        const int jn = P - jb < 256 ? P - jb : 256;
        if (i < P) {
          for (int jj = 0; jj < jn; ++jj) {
            const int j = jb + jj;
            if (j <= i) {
              T v;
              if (i < p) {
                const T d0 = ci0 - colc[0][jj], d1 = ci1 - colc[1][jj], d2 = ci2 - colc[2][jj];
                v = sig2 * mc.rho(sqrt_<T>(d0 * d0 + d1 * d1 + d2 * d2)) + (i == j ? nug : T(0));
              } else if (i == p && j < p) {
                v = colc[3][jj];
              } else {
                v = i == j ? T(1) : T(0);
              }
              M[(size_t)j * ld + i] = v;
            }
          }
        }
      }
    }
    __syncthreads();
    const double guard = a.fp32_guard == 2 ? INFINITY
        : a.fp32_guard ? fmax(0.5 * th.nugget, (double)p * 1.1920928955078125e-07 * (th.sigma2 + th.nugget))
        : 0.0;
    double acc_ll = 0.0, qb = 0.0;
    int flag = 0;
    T mypiv = T(1);
    const int Gp = (p + 15) >> 4;  // panels holding real columns
    for (int J = 0; J < Gp; ++J) {
      // panel update C_IJ = A_IJ - sum_{K<J} L_IK L_JK^T, output tiles I >= J dealt to waves
      if constexpr (TPW == 1) {
        for (int I = J + wv; I < G; I += 4) {
          acc_t c;
#pragma unroll
          for (int r = 0; r < 4; ++r) c[r] = M[(size_t)(J * 16 + lr) * ld + I * 16 + LMma<T>::row(lg, r)];
          // DEPTH steps of operands are loaded before their products, so
          // that 8 DEPTH loads are in flight; the steps past J - 1 of the
          // last group re-load step J - 1 and multiply by zero (no branch, so the
          // loads stay in one scheduling region)
          for (int K0 = 0; K0 < J; K0 += DEPTH) {
            T av[DEPTH][4], bv[DEPTH][4];
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
              const int K = K0 + d < J ? K0 + d : J - 1;
              const T sg = K0 + d < J ? T(-1) : T(0);
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                const int col = K * 16 + 4 * s + lg;
                av[d][s] = sg * M[(size_t)col * ld + I * 16 + lr];
                bv[d][s] = M[(size_t)col * ld + J * 16 + lr];
              }
            }
            // all loads of the group issue before the first product (left to
            // itself the scheduler interleaves FP32 loads with the products)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int d = 0; d < DEPTH; ++d)
#pragma unroll
              for (int s = 0; s < 4; ++s) c = LMma<T>::op(av[d][s], bv[d][s], c);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) M[(size_t)(J * 16 + lr) * ld + I * 16 + LMma<T>::row(lg, r)] = c[r];
        }
      } else {
        // TPW output tiles I0, I0 + 4, ... per wave share each load of
        // the panel operand; DEPTH steps of operands are loaded before
        // their products.  Steps past J - 1 of the last group re-load step J - 1
        // and tiles past G - 1 re-load tile I0, both multiplied by zero (no
        // branch, so the loads stay in one scheduling region)
        for (int I0 = J + wv; I0 < G; I0 += 4 * TPW) {
          acc_t c[TPW];
          int It[TPW];
          T tz[TPW];
#pragma unroll
          for (int t = 0; t < TPW; ++t) {
            It[t] = I0 + 4 * t < G ? I0 + 4 * t : I0;
            tz[t] = I0 + 4 * t < G ? T(-1) : T(0);
#pragma unroll
            for (int r = 0; r < 4; ++r) c[t][r] = M[(size_t)(J * 16 + lr) * ld + It[t] * 16 + LMma<T>::row(lg, r)];
          }
          for (int K0 = 0; K0 < J; K0 += DEPTH) {
            T av[DEPTH][TPW][4], bv[DEPTH][4];
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
              const int K = K0 + d < J ? K0 + d : J - 1;
              const T sg = K0 + d < J ? T(1) : T(0);
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                const int col = K * 16 + 4 * s + lg;
                bv[d][s] = M[(size_t)col * ld + J * 16 + lr];
#pragma unroll
                for (int t = 0; t < TPW; ++t) av[d][t][s] = (sg * tz[t]) * M[(size_t)col * ld + It[t] * 16 + lr];
              }
            }
            // all loads of the group issue before the first product (left to
            // itself the scheduler interleaves FP32 loads with the products)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int d = 0; d < DEPTH; ++d)
#pragma unroll
              for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < TPW; ++t) c[t] = LMma<T>::op(av[d][t][s], bv[d][s], c[t]);
          }
#pragma unroll
          for (int t = 0; t < TPW; ++t)
            if (I0 + 4 * t < G) {
#pragma unroll
              for (int r = 0; r < 4; ++r) M[(size_t)(J * 16 + lr) * ld + It[t] * 16 + LMma<T>::row(lg, r)] = c[t][r];
            }
        }
      }
      __threadfence_block();
      __syncthreads();
      // diagonal tile: unblocked Cholesky by wave 0 in registers (lane r < 16
      // holds row r; the entries of row k come by lane reads), then to LDS
      if (wv == 0) {
        const int r = ln & 15;
        T x[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) x[c] = M[(size_t)(J * 16 + c) * ld + J * 16 + r];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const T dk = lane_read(x[k], k);
          const bool real = J * 16 + k < p;
          const T lkk = real ? sqrt_<T>(dk) : T(1);
          if (r == k) mypiv = real ? dk : T(1);
          x[k] = r > k ? (real ? x[k] / lkk : T(0)) : (r == k ? lkk : x[k]);
#pragma unroll
          for (int c = k + 1; c < 16; ++c) {
            const T lck = lane_read(x[k], c);
            if (r >= c) x[c] -= x[k] * lck;
          }
        }
        if (ln < 16) {
#pragma unroll
          for (int c = 0; c < 16; ++c) dtile[r][c] = c <= r ? x[c] : T(0);
        }
      }
      __syncthreads();
      // rows of the panel: L_IJ = C_IJ L_JJ^-T (rows below the tile), L_JJ in the tile
      for (int i = J * 16 + tid; i < P; i += 256) {
        // the factor tile is re-read from LDS per row rather than held in
        // 136 registers across the loop
        asm volatile("" ::: "memory");
        T x[16];
        if (i < J * 16 + 16) {
#pragma unroll
          for (int c = 0; c < 16; ++c) x[c] = (c <= i - J * 16) ? dtile[i - J * 16][c] : T(0);
        } else {
#pragma unroll
          for (int c = 0; c < 16; ++c) {
            T v = M[(size_t)(J * 16 + c) * ld + i];
#pragma unroll
            for (int q = 0; q < c; ++q) v -= x[q] * dtile[c][q];
            x[c] = (J * 16 + c < p) ? v / dtile[c][c] : T(0);
          }
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) M[(size_t)(J * 16 + c) * ld + i] = x[c];
      }
      __threadfence_block();
      __syncthreads();
      // pivot k = 16 J + tid of the panel: lanes 0..15 of wave 0 keep running sums
      if (tid < 16) {
        const int k = J * 16 + tid;
        if (k < p) {
          const double dd = (double)mypiv;
          if (!(dd > guard)) flag |= a.fp32_guard ? 1 : 2;
          if (!(dd > 0.0)) flag |= 2;
          if (k >= m) {
            const double wk = (double)M[(size_t)k * ld + p];
            acc_ll += log(dd) + wk * wk;
            qb += wk * wk;
          }
        }
      }
      __syncthreads();
    }
    if (wv == 0) {
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        acc_ll += __shfl_xor(acc_ll, off);
        qb += __shfl_xor(qb, off);
        flag |= __shfl_xor(flag, off);
      }
    }
    const size_t o = (size_t)tt * a.bc + b;
    if (tid == 0) {
      a.partial[o] = (flag & 2) && !a.fp32_guard ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
      a.flag[o] = flag | a.flag_or;
    }
    if constexpr (GRAD) {
      // ---- adjoint: X = L^-T [w | [w_N; 0] | [0; I_l]], then the contraction of
      // W = alpha alpha^T - b b^T - X_R X_R^T with d K / d range (d / d sigma2
      // from the quadratic forms and tr W, d / d nugget = tr W / 2), as in the
      // one-wave kernels.  The border row of the factor (row p) holds w.
      for (size_t e = tid; e < ld * NRP; e += 256) {
        const int c = (int)(e / ld), row = (int)(e - (size_t)c * ld);
        T v = T(0);
        if (row < p) {
          if (c == 0 || (c == 1 && row < m)) v = M[(size_t)row * ld + p];
          else if (c >= 2 && row == m + c - 2) v = T(1);
        }
        X[e] = v;
      }
      __threadfence_block();
      __syncthreads();
      for (int K = Gp - 1; K >= 0; --K) {
        // L_KK to LDS (padding columns of the factor are identity)
        for (int e = tid; e < 256; e += 256) {
          const int r = e & 15, c = e >> 4;
          dtile[r][c] = r >= c ? M[(size_t)(K * 16 + c) * ld + K * 16 + r] : T(0);
        }
        __syncthreads();
        // X_K <- L_KK^-T X_K, one column per thread (back-substitution)
        for (int c = tid; c < NRP; c += 256) {
          asm volatile("" ::: "memory");   // re-read the tile from LDS per column
          T x[16];
#pragma unroll
          for (int r = 0; r < 16; ++r) x[r] = X[(size_t)c * ld + K * 16 + r];
#pragma unroll
          for (int r = 15; r >= 0; --r) {
            T v = x[r];
#pragma unroll
            for (int t = r + 1; t < 16; ++t) v -= dtile[t][r] * x[t];
            x[r] = v / dtile[r][r];
          }
#pragma unroll
          for (int r = 0; r < 16; ++r) X[(size_t)c * ld + K * 16 + r] = x[r];
        }
        __threadfence_block();
        __syncthreads();
        // X_J -= L_KJ^T X_K for J < K: 16 x 16 output tiles (J, q) dealt to the waves
        const int nq = NRP >> 4;
        for (int e = wv; e < K * nq; e += 4) {
          const int J = e / nq, q = e - J * nq;
          acc_t c;
#pragma unroll
          for (int r = 0; r < 4; ++r) c[r] = X[(size_t)(q * 16 + lr) * ld + J * 16 + LMma<T>::row(lg, r)];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int t = K * 16 + 4 * s + lg;
            const T av = -M[(size_t)(J * 16 + lr) * ld + t];   // L[t][J*16 + i]
            const T bv = X[(size_t)(q * 16 + lr) * ld + t];
            c = LMma<T>::op(av, bv, c);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) X[(size_t)(q * 16 + lr) * ld + J * 16 + LMma<T>::row(lg, r)] = c[r];
        }
        __threadfence_block();
        __syncthreads();
      }
      // contraction over the tile pairs (I, J), J <= I < Gp, dealt to the waves
      const T irange = T(th.inv_range);
      double g1 = 0.0, g2 = 0.0;
      const int npair = Gp * (Gp + 1) / 2;
      for (int e = wv; e < npair; e += 4) {
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= e) ++I;
        const int J = e - I * (I + 1) / 2;
        acc_t w;
#pragma unroll
        for (int r = 0; r < 4; ++r) w[r] = T(0);
        for (int c0 = 0; c0 < NRP; c0 += 4) {
          const int c = c0 + lg;
          const T av = (c == 0 ? T(1) : T(-1)) * X[(size_t)c * ld + I * 16 + lr];
          const T bv = X[(size_t)c * ld + J * 16 + lr];
          w = LMma<T>::op(av, bv, w);
        }
        const int j = J * 16 + lr;
        const T sj0 = cs[j], sj1 = cs[ld + j], sj2 = cs[2 * ld + j];
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = I * 16 + LMma<T>::row(lg, r);
          if (i < p && j < p) {
            const T d0 = cs[i] - sj0, d1 = cs[ld + i] - sj1, d2 = cs[2 * ld + i] - sj2;
            s1 += w[r] * mc.drange(sqrt_<T>(d0 * d0 + d1 * d1 + d2 * d2), irange);
            if (i == j) s2 += w[r];
          }
        }
        g1 += (I == J ? 1.0 : 2.0) * (double)s1;
        g2 += (double)s2;
      }
      sred[0][tid] = g1;
      sred[1][tid] = g2;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
          sred[0][tid] += sred[0][tid + h];
          sred[1][tid] += sred[1][tid + h];
        }
        __syncthreads();
      }
      if (tid == 0) {
        const bool bad = (flag & 2) && !a.fp32_guard;
        const double tr = sred[1][0];
        a.gpart[3 * o + 0] = bad ? __builtin_nan("") : 0.5 * (qb - (double)l - th.nugget * tr) / th.sigma2;
        a.gpart[3 * o + 1] = bad ? __builtin_nan("") : 0.5 * th.sigma2 * sred[0][0];
        a.gpart[3 * o + 2] = bad ? __builtin_nan("") : 0.5 * tr;
      }
      __syncthreads();
    }
  }
}

// slot elements of a large block with pmax joint rows and lmax block rows,
// with the gradient's right-hand sides
size_t large_slot_elems(int pmax, int lmax) {
  const size_t P = 16 * (size_t)((pmax + 1 + 15) / 16);
  const size_t nrp = 16 * (size_t)((lmax + 2 + 15) / 16);
  return P * (P + nrp) + 3 * P;
}

hipError_t launch_large(bool fp32, bool grad, const LargeArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  if (fp32) {
    if (grad) hipLaunchKernelGGL((bv_large_kernel<float, true>), dim3(grid), dim3(256), 0, s, a, thp);
    else hipLaunchKernelGGL((bv_large_kernel<float, false>), dim3(grid), dim3(256), 0, s, a, thp);
  } else {
    if (grad) hipLaunchKernelGGL((bv_large_kernel<double, true>), dim3(grid), dim3(256), 0, s, a, thp);
    else hipLaunchKernelGGL((bv_large_kernel<double, false>), dim3(grid), dim3(256), 0, s, a, thp);
  }
  return hipGetLastError();
}

}  // namespace bv
