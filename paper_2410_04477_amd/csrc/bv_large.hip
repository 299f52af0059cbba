// Blocks whose joint size exceeds the register capacity (m_i + l_i > 175), e.g.
// conditioning on every earlier point.  One workgroup (four waves) per block:
// the bordered matrix [[K_J, .], [y_J^T, .]] (p + 1 rows, padded with identity to
// P = 16 G) is generated into a global workspace (column-major, lower part),
// then factored left-looking in 16-column panels:
//   C_IJ = A_IJ - sum_{K<J} L_IK L_JK^T      (MFMA, one output tile per wave at a time)
//   L_JJ = chol(C_JJ), L_IJ = C_IJ L_JJ^-T  (one thread per row)
// The log-determinant and quadratic form come from the panel pivots and the
// border row, as in the register kernels.  Operands stream through L2: about
// P^3 / 96 elements are read per block.
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

template <typename T>
__global__ void __launch_bounds__(256) bv_large_kernel(LargeArgs a, ThetaPack thp) {
  typedef typename LMma<T>::acc acc_t;
  __shared__ T dtile[16][17];
  __shared__ T piv[16];
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
    const int d = a.d;
    const MaternCoef<T> mc(th.nu_code);
    const T sig2 = T(th.sigma2), nug = T(th.nugget);
    // ---- generate the lower part, column by column (rows over threads) -----
    __syncthreads();
    for (int j = 0; j < P; ++j) {
      const int gj = j < m ? a.nbr_idx[n0 + j] : (b0 + j - m);
      T cj[3] = {T(0), T(0), T(0)};
      if (j < p)
        for (int k = 0; k < d; ++k) cj[k] = T((a.locs[(size_t)gj * d + k] - a.locs[(size_t)b0 * d + k]) * th.inv_scale[k]);
      const T yj = j < p ? T(a.y[gj]) : T(0);
      for (int i = j + tid; i < P; i += 256) {
        T v;
        if (i < p && j < p) {
          const int gi = i < m ? a.nbr_idx[n0 + i] : (b0 + i - m);
          T h2 = T(0);
          for (int k = 0; k < d; ++k) {
            const T ci = T((a.locs[(size_t)gi * d + k] - a.locs[(size_t)b0 * d + k]) * th.inv_scale[k]);
            h2 += (ci - cj[k]) * (ci - cj[k]);
          }
          v = sig2 * mc.rho(sqrt_<T>(h2)) + (i == j ? nug : T(0));
        } else if (i == p && j < p) {
          v = yj;
        } else {
          v = i == j ? T(1) : T(0);
        }
        M[(size_t)j * ld + i] = v;
      }
    }
    __syncthreads();
    const double guard = a.fp32_guard == 2 ? INFINITY
        : a.fp32_guard ? fmax(0.5 * th.nugget, (double)p * 1.1920928955078125e-07 * (th.sigma2 + th.nugget))
        : 0.0;
    double acc_ll = 0.0;
    int flag = 0;
    const int Gp = (p + 15) >> 4;  // panels holding real columns
    for (int J = 0; J < Gp; ++J) {
      // panel update C_IJ = A_IJ - sum_{K<J} L_IK L_JK^T, output tiles I >= J dealt to waves
      for (int I = J + wv; I < G; I += 4) {
        acc_t c;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = M[(size_t)(J * 16 + lr) * ld + I * 16 + LMma<T>::row(lg, r)];
        for (int K = 0; K < J; ++K) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int col = K * 16 + 4 * s + lg;
            const T av = -M[(size_t)col * ld + I * 16 + lr];
            const T bv = M[(size_t)col * ld + J * 16 + lr];
            c = LMma<T>::op(av, bv, c);
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) M[(size_t)(J * 16 + lr) * ld + I * 16 + LMma<T>::row(lg, r)] = c[r];
      }
      __threadfence_block();
      __syncthreads();
      // diagonal tile: unblocked Cholesky by wave 0 in LDS
      if (wv == 0) {
        for (int e = ln; e < 256; e += 64) {
          const int r = e & 15, c = e >> 4;
          dtile[r][c] = M[(size_t)(J * 16 + c) * ld + J * 16 + r];
        }
      }
      __syncthreads();
      if (wv == 0) {
        for (int k = 0; k < 16; ++k) {
          const T dk = dtile[k][k];
          const bool real = J * 16 + k < p;
          const T lkk = real ? sqrt_<T>(dk) : T(1);
          if (ln == 0) piv[k] = real ? dk : T(1);
          if (ln > k && ln < 16) dtile[ln][k] = real ? dtile[ln][k] / lkk : T(0);
          wave_sync();
          if (ln == 0) dtile[k][k] = lkk;
          if (ln > k && ln < 16)
            for (int c = k + 1; c <= ln; ++c) dtile[ln][c] -= dtile[ln][k] * dtile[c][k];
          wave_sync();
        }
      }
      __syncthreads();
      // rows of the panel: L_IJ = C_IJ L_JJ^-T (rows below the tile), L_JJ in the tile
      for (int i = J * 16 + tid; i < P; i += 256) {
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
      if (tid == 0) {
        for (int c = 0; c < 16; ++c) {
          const int k = J * 16 + c;
          if (k < p) {
            const double dd = (double)piv[c];
            if (!(dd > guard)) flag |= a.fp32_guard ? 1 : 2;
            if (!(dd > 0.0)) flag |= 2;
            if (k >= m) {
              const double wk = (double)M[(size_t)k * ld + p];
              acc_ll += log(dd) + wk * wk;
            }
          }
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const size_t o = (size_t)tt * a.bc + b;
      a.partial[o] = (flag & 2) && !a.fp32_guard ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
      a.flag[o] = flag | a.flag_or;
    }
  }
}

hipError_t launch_large(bool fp32, const LargeArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL((bv_large_kernel<float>), dim3(grid), dim3(256), 0, s, a, thp);
  else
    hipLaunchKernelGGL((bv_large_kernel<double>), dim3(grid), dim3(256), 0, s, a, thp);
  return hipGetLastError();
}

}  // namespace bv
