// Matrix-core (MFMA) kernels for the per-block chain of Alg. 1.
//
// One workgroup of four waves evaluates one block for one theta.  The
// bordered joint matrix [[K_J, .], [y_J^T, .]] (p + 1 rows, padded to P = 16 G
// with identity) is held in registers as 16 x 16 accumulator tiles of the
// v_mfma_*_16x16x4 instructions, the lower-triangular tiles dealt round-robin
// to the four waves.  Every lane generates its own Matern entries.
//
// Factorisation: right-looking Cholesky in panels of four columns.  The
// owners of the panel write it to LDS; all threads factor its 4 x 4 diagonal
// block redundantly and solve one panel row each (the TRSM / TRSV of Alg. 1
// for those columns; the border row becomes w = L^-1 y_J); the trailing matrix
// is then updated by one rank-4 MFMA per tile (the Schur update of Alg. 1).
// Two barriers per panel.  Pivots d_k (k >= m) and border entries w_k give the
// log-determinant and quadratic form of the block, accumulated in FP64.
//
// Adjoint (MODE 1): the factor is kept in the tiles (each finished panel is
// written back over the columns its own update touched), then
//   X = L^-T [ w | [z; 0] | [0; I_l] ]
// is solved tile row by tile row in LDS -- the owners publish the tile row, a
// 16-row triangular solve per right-hand side, and the rows above are updated
// with MFMA products -- and W = alpha alpha^T - b b^T - X_R X_R^T is formed tile by
// tile with MFMA and contracted against dK regenerated entry by entry (FP64
// sums):  d l_i = 1/2 <W, dK>.
// Coefficient mode (MODE 2): border e_last, X = alpha = K_J^-1 e_last gives the
// sequential simulator's conditional-mean weights and variance.
//
// MFMA 16x16x4 operand layout (lane l, r = 0..3): A[l % 16][l / 16],
// B[l / 16][l % 16]; accumulator register r holds column l % 16 of row
// 4 (l / 16) + r for FP32 but of row l / 16 + 4 r for FP64 (Mma<T>::row).
#include "internal.hpp"

namespace bv {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef f32x4_t acc;
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // tile row held by accumulator register r of lane group g
  static __device__ __forceinline__ constexpr int row(int g, int r) { return 4 * g + r; }
};
template <> struct Mma<double> {
  typedef f64x4_t acc;
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int g, int r) { return g + 4 * r; }
};

__host__ __device__ constexpr int mfma_pan_elems(int G) { return 2 * 4 * 16 * G; }

template <typename T, int G, int MODE>
__global__ void __launch_bounds__(256)
bv_mfma_kernel(AdjArgs a, ThetaPack thp) {
  constexpr int P = 16 * G;
  constexpr int GA = (G + 1) / 2;            // tile pairs per dimension
  constexpr int TPW = GA * (GA + 1) / 2;     // slots (a, b), a >= b, per wave
  typedef typename Mma<T>::acc acc_t;
  extern __shared__ __align__(16) unsigned char smem[];
  T* su = reinterpret_cast<T*>(smem);  // scaled coordinates relative to the block's first point, su[k * P + i]
  T* sy = su + 3 * P;       // border row: y_J (e_last in coefficient mode)
  T* work = sy + P;
  __shared__ double sred[3][4];
  __shared__ T dcopy[2][16];     // 4 x 4 diagonal block of the current / next panel, [c * 4 + r]
  __shared__ T sdk[P], swk[P];   // pivots d_k and border entries w_k (log-det / quadratic form)

  const int tid = threadIdx.x;
  const int wv = tid >> 6, ln = tid & 63;
  const int lr = ln & 15, lg = ln >> 4;
  const int ldx = a.ldx;

  // The four waves form a 2 x 2 grid: wave (wr, wc) owns tile (2a + wr, 2b + wc)
  // for every slot (a, b), a >= b, that lies in the lower triangle.  Slot
  // offsets are then compile-time constants plus one wave-uniform term.
  const int wuni = __builtin_amdgcn_readfirstlane(wv);
  const int wr = wuni & 1, wc = wuni >> 1;
  int tI[TPW], tJ[TPW];
#pragma unroll
  for (int aa = 0, s = 0; aa < GA; ++aa)
#pragma unroll
    for (int bb = 0; bb <= aa; ++bb, ++s) {
      const int I = 2 * aa + wr, J = 2 * bb + wc;
      const bool ok = I < G && J < G && (aa > bb || wr >= wc);
      tI[s] = ok ? I : 0;   // empty slots point at tile row 0 so every index stays in range
      tJ[s] = ok ? J : G;   // J == G marks an empty slot
    }

  // one work item per workgroup (no loop: nothing is hoisted across items)
  const int total = a.list ? *a.list_count : a.nsched * a.ntheta;
  const int wi = blockIdx.x;
  if (wi < total) {
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

    __syncthreads();
    for (int i = tid; i < p; i += 256) {
      const int g = (i < m) ? a.nbr_idx[n0 + i] : (b0 + i - m);
      sy[i] = MODE == 2 ? ((i == p - 1) ? T(1) : T(0)) : T(a.y[g]);
      for (int k = 0; k < 3; ++k) {
        T v = T(0);
        if (k < a.d) v = T((a.locs[(size_t)g * a.d + k] - a.locs[(size_t)b0 * a.d + k]) * th.inv_scale[k]);
        su[k * P + i] = v;
      }
    }
    __syncthreads();

    // ---- generate the bordered joint matrix in the accumulator tiles --------
    const T sig2 = T(th.sigma2), nug = T(th.nugget);
    const MaternCoef<T> mc(th.nu_code);
    // border value of column j (this lane's column in every tile column)
    acc_t acc[TPW];
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      const int j = (tJ[s] < G ? tJ[s] : 0) * 16 + lr;
      const T sj0 = su[j], sj1 = su[P + j], sj2 = su[2 * P + j];
      const T yb = sy[j];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = tI[s] * 16 + Mma<T>::row(lg, r);
        const T dx = su[i] - sj0;
        const T dy = su[P + i] - sj1;
        const T dz = su[2 * P + i] - sj2;
        const T x = sqrt_fast<T>(dx * dx + dy * dy + dz * dz);
        T v = sig2 * mc.rho(x) + ((i == j) ? nug : T(0));
        if (!(i < p && j < p)) v = (i == p && j < p) ? yb : ((i == j) ? T(1) : T(0));
        acc[s][r] = tJ[s] < G ? v : T(0);
      }
      __builtin_amdgcn_sched_barrier(0);  // one slot at a time: bounds the live Matern temporaries
    }

    const double guard = a.fp32_guard == 2 ? INFINITY
        : a.fp32_guard ? fmax(0.5 * th.nugget, (double)p * 1.1920928955078125e-07 * (th.sigma2 + th.nugget))
        : 0.0;
    double acc_ll = 0.0;
    int flag = 0;

    // extract panel 0 (columns 0..3) and a copy of its diagonal block
    {
      T* pan = work;
#pragma unroll
      for (int s = 0; s < TPW; ++s)
        if (tJ[s] == 0 && lr < 4) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rw = Mma<T>::row(lg, r);
            pan[lr * P + tI[s] * 16 + rw] = acc[s][r];
            if (tI[s] == 0 && rw < 4) dcopy[0][lr * 4 + rw] = acc[s][r];
          }
        }
    }

    // ---- factorisation, four columns per step ---------------------------------
    for (int k0 = 0; k0 < p; k0 += 4) {
      const int K = k0 >> 4, c0 = k0 & 15;
      const int pb = (k0 >> 2) & 1;
      T* pan = work + pb * 4 * P;
      T* pnext = work + (pb ^ 1) * 4 * P;
      const T* dblk = dcopy[pb];
      __syncthreads();
      // 4 x 4 diagonal block (every thread, redundantly)
      T Ld[4][4];
      T piv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Ld[r][c] = T(0);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool real = k0 + c < p;
        T dsum = dblk[c * 4 + c];
#pragma unroll
        for (int j = 0; j < c; ++j) dsum -= Ld[c][j] * Ld[c][j];
        piv[c] = real ? dsum : T(1);
        const T lcc = real ? sqrt_<T>(dsum) : T(1);
        Ld[c][c] = lcc;
        const T inv = T(1) / lcc;
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
          T v = dblk[c * 4 + r];
#pragma unroll
          for (int j = 0; j < c; ++j) v -= Ld[r][j] * Ld[c][j];
          Ld[r][c] = real ? v * inv : T(0);
        }
      }
      // panel rows of tile K and below: zero above the block, L_dd in it, TRSM below
      {
        const int i = K * 16 + tid;
        if (i < P) {
          T x[4];
          if (i < k0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) x[c] = T(0);
          } else if (i < k0 + 4) {
#pragma unroll
            for (int c = 0; c < 4; ++c) x[c] = Ld[i - k0][c];
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              T v = pan[c * P + i];
#pragma unroll
              for (int j = 0; j < c; ++j) v -= x[j] * Ld[c][j];
              x[c] = (k0 + c < p) ? v / Ld[c][c] : T(0);
            }
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) pan[c * P + i] = x[c];
          if (i == p) {
#pragma unroll
            for (int c = 0; c < 4; ++c) swk[k0 + c] = x[c];
          }
        }
      }
      if (tid == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sdk[k0 + c] = piv[c];
      }
      __syncthreads();
      // rank-4 update of the trailing tiles: D -= L_I L_J^T
#pragma unroll
      for (int s = 0; s < TPW; ++s) {
        if (tJ[s] < G && tJ[s] >= K) {
          const T av = -pan[lg * P + tI[s] * 16 + lr];
          const T bv = pan[lg * P + tJ[s] * 16 + lr];
          acc[s] = Mma<T>::op(av, bv, acc[s]);
        }
      }
      if (MODE != 0) {
        // keep the finished factor columns in the tiles
#pragma unroll
        for (int s = 0; s < TPW; ++s)
          if (tJ[s] == K && lr >= c0 && lr < c0 + 4) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[s][r] = pan[(lr - c0) * P + tI[s] * 16 + Mma<T>::row(lg, r)];
          }
      }
      // publish the next panel
      const int k1 = k0 + 4;
      if (k1 < p) {
        const int K1 = k1 >> 4, c1 = k1 & 15;
#pragma unroll
        for (int s = 0; s < TPW; ++s)
          if (tJ[s] == K1 && lr >= c1 && lr < c1 + 4) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int rw = Mma<T>::row(lg, r);
              pnext[(lr - c1) * P + tI[s] * 16 + rw] = acc[s][r];
              if (tI[s] == K1 && rw >= c1 && rw < c1 + 4) dcopy[pb ^ 1][(lr - c1) * 4 + rw - c1] = acc[s][r];
            }
          }
      }
    }

    // log-determinant, quadratic form and pivot guard, one pivot per thread (FP64)
    {
      __syncthreads();
      double v = 0.0;
      int f = 0;
      for (int k = tid; k < p; k += 256) {
        const double dd = (double)sdk[k];
        if (!(dd > guard)) f |= a.fp32_guard ? 1 : 2;
        if (!(dd > 0.0)) f |= 2;
        if (MODE != 2 && k >= m) {
          const double wk = (double)swk[k];
          v += log(dd) + wk * wk;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        v += __shfl_down(v, off, 64);
        f |= __shfl_down(f, off, 64);
      }
      if (ln == 0) {
        sred[0][wv] = v;
        sred[1][wv] = (double)f;
      }
      __syncthreads();
      acc_ll = ((sred[0][0] + sred[0][1]) + sred[0][2]) + sred[0][3];
      flag = (int)sred[1][0] | (int)sred[1][1] | (int)sred[1][2] | (int)sred[1][3];
    }

    if (MODE == 0) {
      if (tid == 0) {
        const size_t o = (size_t)tt * a.bc + b;
        a.partial[o] = (flag & 2) && !a.fp32_guard ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
        a.flag[o] = flag | a.flag_or;
      }
      return;
    }

    // ---- back-substitution X <- L^-T X --------------------------------------
    const int nr = MODE == 1 ? l + 2 : 1;
    const int nq = (nr + 15) >> 4;
    T* X = work;              // P x ldx
    T* lrow = work + P * ldx; // 16 x P: the published tile row
    __syncthreads();
    for (int e = tid; e < P * ldx; e += 256) X[e] = T(0);
    __syncthreads();
    if (MODE == 1)
      for (int q = tid; q < l; q += 256) X[(m + q) * ldx + 2 + q] = T(1);
    {
      const int Ip = p >> 4, rp = p & 15;
#pragma unroll
      for (int s = 0; s < TPW; ++s)
        if (tJ[s] < G && tI[s] == Ip) {
          const int j = tJ[s] * 16 + lr;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (Mma<T>::row(lg, r) == rp && j < p) {
              X[j * ldx] = acc[s][r];                              // w
              if (MODE == 1 && j < m) X[j * ldx + 1] = acc[s][r];  // [z; 0]
            }
        }
    }
    const int Gp = (p + 15) >> 4;
    for (int K = Gp - 1; K >= 0; --K) {
      __syncthreads();
#pragma unroll
      for (int s = 0; s < TPW; ++s)
        if (tJ[s] < G && tI[s] == K) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rw = Mma<T>::row(lg, r);
            const int i = K * 16 + rw, j = tJ[s] * 16 + lr;
            T v = acc[s][r];
            if (i >= p || j >= p) v = (i == j) ? T(1) : T(0);
            else if (j > i) v = T(0);
            lrow[rw * P + j] = v;
          }
        }
      __syncthreads();
      // diagonal tile: X_K <- L_KK^-T X_K, one thread per right-hand side
      if (tid < nr) {
        T x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = X[(K * 16 + r) * ldx + tid];
#pragma unroll
        for (int rr = 15; rr >= 0; --rr) {
          T v = x[rr];
#pragma unroll
          for (int r2 = rr + 1; r2 < 16; ++r2) v -= lrow[r2 * P + K * 16 + rr] * x[r2];
          x[rr] = v / lrow[rr * P + K * 16 + rr];
          __builtin_amdgcn_sched_barrier(0);  // bound the live L_KK loads
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) X[(K * 16 + r) * ldx + tid] = x[r];
      }
      __syncthreads();
      // rows above: X_J -= L_KJ^T X_K, output tiles (J, q) dealt to the waves
      const int nout = K * nq;
      for (int e = wv; e < nout; e += 4) {
        const int J = e / nq, q = e - (e / nq) * nq;
        acc_t c;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = X[(J * 16 + Mma<T>::row(lg, r)) * ldx + q * 16 + lr];
#pragma unroll
        for (int sub = 0; sub < 4; ++sub) {
          const T av = -lrow[(4 * sub + lg) * P + J * 16 + lr];
          const T bv = X[(K * 16 + 4 * sub + lg) * ldx + q * 16 + lr];
          c = Mma<T>::op(av, bv, c);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) X[(J * 16 + Mma<T>::row(lg, r)) * ldx + q * 16 + lr] = c[r];
      }
    }
    __syncthreads();

    if (MODE == 2) {
      const double al = (double)X[(p - 1) * ldx];
      for (int j = tid; j < m; j += 256) a.coef[(size_t)tt * a.coef_stride + n0 + j] = -(double)X[j * ldx] / al;
      if (tid == 0) {
        a.cvar[(size_t)tt * a.bc + b] = 1.0 / al;
        a.flag[(size_t)tt * a.bc + b] = flag;
      }
      return;
    }

    // ---- W = alpha alpha^T - b b^T - X_R X_R^T tile by tile, contracted with dK ---
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    const int nk = (nr + 3) >> 2;
    const T irange = T(th.inv_range);
#pragma unroll
    for (int s = 0; s < TPW; ++s) {
      if (tJ[s] < G && tI[s] < Gp) {
        acc_t c;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = T(0);
        const int iI = tI[s] * 16, jJ = tJ[s] * 16;
        for (int kq = 0; kq < nk; ++kq) {
          const int q = 4 * kq + lg;
          const T sg = q == 0 ? T(1) : T(-1);
          const T av = sg * X[(iI + lr) * ldx + q];
          const T bv = X[(jJ + lr) * ldx + q];
          c = Mma<T>::op(av, bv, c);
        }
        const double wgt = tI[s] == tJ[s] ? 1.0 : 2.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = iI + Mma<T>::row(lg, r), j = jJ + lr;
          if (i < p && j < p) {
            const T dx = su[i] - su[j];
            const T dy = su[P + i] - su[P + j];
            const T dz = su[2 * P + i] - su[2 * P + j];
            const T x = sqrt_fast<T>(dx * dx + dy * dy + dz * dz);
            T rho, drho;
            mc.rho_drange(x, irange, rho, drho);
            const double wv2 = wgt * (double)c[r];
            g0 += wv2 * (double)rho;
            g1 += wv2 * (double)drho;
            if (i == j) g2 += (double)c[r];
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // every thread has read the pivot sums from sred
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      g0 += __shfl_down(g0, off, 64);
      g1 += __shfl_down(g1, off, 64);
      g2 += __shfl_down(g2, off, 64);
    }
    if (ln == 0) {
      sred[0][wv] = g0;
      sred[1][wv] = g1;
      sred[2][wv] = g2;
    }
    __syncthreads();
    if (tid == 0) {
      const double s0 = ((sred[0][0] + sred[0][1]) + sred[0][2]) + sred[0][3];
      const double s1 = ((sred[1][0] + sred[1][1]) + sred[1][2]) + sred[1][3];
      const double s2 = ((sred[2][0] + sred[2][1]) + sred[2][2]) + sred[2][3];
      const size_t o = (size_t)tt * a.bc + b;
      const bool bad = (flag & 2) && !a.fp32_guard;
      a.partial[o] = bad ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
      a.gpart[3 * o + 0] = bad ? __builtin_nan("") : 0.5 * s0;
      a.gpart[3 * o + 1] = bad ? __builtin_nan("") : 0.5 * th.sigma2 * s1;
      a.gpart[3 * o + 2] = bad ? __builtin_nan("") : 0.5 * s2;
      a.flag[o] = flag | a.flag_or;
    }
  }
}

// dynamic LDS bytes of one launch
template <typename T, int G, int MODE>
static size_t mfma_lds_bytes(int ldx) {
  constexpr int P = 16 * G;
  const size_t head = sizeof(T) * 4 * P;
  size_t work = sizeof(T) * (size_t)mfma_pan_elems(G);
  if (MODE != 0) {
    const size_t adj = sizeof(T) * ((size_t)P * ldx + 16 * (size_t)P);
    work = adj > work ? adj : work;
  }
  return head + work;
}

template <typename T, int G, int MODE>
static hipError_t launch_mfma_g(const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  const size_t lds = mfma_lds_bytes<T, G, MODE>(a.ldx);
  hipLaunchKernelGGL((bv_mfma_kernel<T, G, MODE>), dim3(grid), dim3(256), lds, s, a, thp);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_mfma_t(int g, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  switch (g) {
    case 1: return launch_mfma_g<T, 1, MODE>(a, thp, grid, s);
    case 2: return launch_mfma_g<T, 2, MODE>(a, thp, grid, s);
    case 3: return launch_mfma_g<T, 3, MODE>(a, thp, grid, s);
    case 4: return launch_mfma_g<T, 4, MODE>(a, thp, grid, s);
    case 5: return launch_mfma_g<T, 5, MODE>(a, thp, grid, s);
    case 6: return launch_mfma_g<T, 6, MODE>(a, thp, grid, s);
    case 7: return launch_mfma_g<T, 7, MODE>(a, thp, grid, s);
    case 8: return launch_mfma_g<T, 8, MODE>(a, thp, grid, s);
    case 9: return launch_mfma_g<T, 9, MODE>(a, thp, grid, s);
    case 10: return launch_mfma_g<T, 10, MODE>(a, thp, grid, s);
    case 11: return launch_mfma_g<T, 11, MODE>(a, thp, grid, s);
    default: return hipErrorInvalidValue;
  }
}

size_t mfma_lds_need(int g, bool fp32, int mode, int ldx) {
  const size_t P = 16 * (size_t)g, e = fp32 ? 4 : 8;
  size_t work = e * 2 * 4 * P;
  if (mode != 0) {
    const size_t adj = e * (P * (size_t)ldx + 16 * P);
    work = adj > work ? adj : work;
  }
  // static arrays: sred, dcopy, sdk, swk
  return e * 4 * P + work + 12 * 8 + e * (32 + 2 * P);
}

hipError_t launch_mfma(int g, bool fp32, int mode, const AdjArgs& a, const ThetaPack& thp, int grid,
                       hipStream_t s) {
  if (mode == 0) return fp32 ? launch_mfma_t<float, 0>(g, a, thp, grid, s) : launch_mfma_t<double, 0>(g, a, thp, grid, s);
  if (mode == 1) return fp32 ? launch_mfma_t<float, 1>(g, a, thp, grid, s) : launch_mfma_t<double, 1>(g, a, thp, grid, s);
  return launch_mfma_t<double, 2>(g, a, thp, grid, s);
}

}  // namespace bv
