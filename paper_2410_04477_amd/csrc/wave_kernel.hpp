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
// update).  Lanes exchange panel data through LDS with wavefront-scope
// fences, so a panel costs no cross-wave synchronisation.  Pivots d_k and
// border entries w_k (k >= m) give log det and the quadratic form, summed in
// FP64.
//
// Adjoint: X = L^-T [ w | [z; 0] | [0; I_l] ] is pure MFMA work tile row by
// tile row, X_K <- inv(L_KK)^T X_K, then X_J -= L_KJ^T X_K for the rows above;
// W = alpha alpha^T - b b^T - X_R X_R^T is formed tile by tile with MFMA and
// contracted against dK regenerated entry by entry (FP64 across tiles):
// d l_i = 1/2 <W, dK>.  MODE 5 keeps the factor in the registers (the
// diagonal inverses formed during the factorisation from 16 rows appended to
// each panel) and takes its A operands from the accumulator registers;
// MODE 1 stores the factor tiles to the item's slot of a global tile buffer,
// inverts the diagonal blocks there (16 lanes per block, all blocks in one
// pass) and reads its A operands from the buffer; MODES 2 + 3 split the two
// halves over two launches, and MODES 6 + 3 likewise with a left-looking
// factorisation (FP64 above G = 9).
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
  // position, inside a tile stored in accumulator order (lane * 4 + register),
  // of element (4 s + l / 16, l % 16): the A operand of lane l for k-step s
  // when the stored tile is used transposed
  static __device__ __forceinline__ constexpr int aop(int l, int s) { return ((l & 15) + 16 * s) * 4 + (l >> 4); }
  // position of element (i, j) of a tile stored in accumulator order
  static __device__ __forceinline__ constexpr int at(int i, int j) { return (j + 16 * (i >> 2)) * 4 + (i & 3); }
};
template <> struct WMma<double> {
  typedef w64x4_t acc;
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int g, int r) { return g + 4 * r; }
  static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / sqrt(x); }
  static __device__ __forceinline__ constexpr int aop(int l, int s) { return l * 4 + s; }
  static __device__ __forceinline__ constexpr int at(int i, int j) { return (j + 16 * (i & 3)) * 4 + (i >> 2); }
};

// lower-triangular tile (I, J), J <= I, in row-major packed order
__host__ __device__ constexpr int tix(int I, int J) { return I * (I + 1) / 2 + J; }

constexpr int kStageStride = 260;   // staged 16 x 16 tiles, padded so tiles four apart fall in different banks

__host__ __device__ constexpr int wave_max(int x, int y) { return x > y ? x : y; }

// The kernels below run one wave per workgroup, and a wave's LDS operations
// are performed in issue order, so lanes exchange data through LDS with a
// wavefront-scope fence (it keeps the compiler from moving LDS accesses across
// it) and no wait for the LDS traffic.  Exchanges through global memory (the
// tile buffer of mode 1, the stored tile columns of mode 6) keep the workgroup
// barrier.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ constexpr int wave_lds_elems(int G, int mode) {
  // su (3 P) for the whole kernel, then a work region: the panel (4 columns of
  // P rows, plus 16 appended rows in the modes that form the diagonal inverses
  // during the factorisation) and sy, sdk, swk (P each) during the
  // factorisation; for the adjoint, one chunk of right-hand sides
  // (P x (wave_chunk(G) + 1), plus 32 elements that reads of the last row's
  // unused columns may touch), which also holds the G staged diagonal tiles
  // before the first chunk
  // (mode 5 keeps the border row w of the factor after that, 16 G elements)
  return 3 * 16 * G + wave_max(4 * (16 * G + (mode == 2 || mode == 5 || mode == 6 ? 16 : 0)) + 3 * 16 * G,
                               mode == 0 || mode == 2 || mode == 4 || mode == 6 ? 0
                               : (16 * (wave_chunk(G) + 1) > kStageStride
                                      ? 16 * G * (wave_chunk(G) + 1) + 32
                                      : G * kStageStride)) +
         (mode == 5 ? 16 * G : 0);
}

template <typename T, int G, int MODE>
constexpr int wave_min_waves() { return (sizeof(T) == 4 && (G <= 9 || MODE == 3)) || MODE == 6 ? 2 : 1; }

// Modes: 0 value; 1 value and gradient in one launch; 2 value and the factor
// tiles to the tile buffer; 3 gradient from those tiles (a second launch that
// holds no tiles in registers, so it runs more waves per SIMD than mode 1);
// 4 prediction (Alg. 2): the block rows are new locations, the border row
// carries y_N and zeros, and only the neighbour columns are eliminated, which
// leaves the Schur complement -- the conditional covariance of the block and,
// in the border row, minus its conditional mean -- in the trailing tiles.
// 5 value and gradient in one launch with the factor kept in the registers
// through the back-substitution (no tile buffer; right-hand sides in passes
// of wave_chunk(G), at G = 9 one pass only: l + 2 <= wave_chunk(G)).
// 6 value and the factor tiles to the tile buffer, as mode 2, but left-looking
// by tile columns: a tile column is generated when its turn comes, updated
// with the stored columns to its left (MFMA, operands read back from the
// buffer), factored in its four panels and stored, so that only one tile
// column is in the registers at a time (FP64 classes above G = 9, whose tiles
// exceed the register file); mode 3 takes the adjoint from its tiles.
// GEN: covariances by the Bessel form for any nu instead of the closed forms.
template <typename T, int G, int MODE, bool GEN>
__global__ void __launch_bounds__(64, (wave_min_waves<T, G, MODE>())) bv_wave_kernel(AdjArgs a, ThetaPack thp) {
  constexpr int P = 16 * G;
  constexpr int NT = G * (G + 1) / 2;
  typedef WMma<T> M;
  typedef typename M::acc acc_t;
  extern __shared__ __align__(16) unsigned char smem[];
  T* su = reinterpret_cast<T*>(smem);  // scaled coordinates relative to the block's first point, su[k * P + i]
  // FP32 closed forms: the coordinates carry a factor log2(e), so e^-x is one
  // exp2 of the distance and the polynomial coefficients carry powers of ln 2
  constexpr bool LOG2U = !GEN && sizeof(T) == 4;
  T* work = su + 3 * P;
  // MODE 5 appends 16 rows to the panel (the identity rows whose elimination
  // gives the inverse of each diagonal tile of the factor)
  constexpr bool LEFT = MODE == 6;                // left-looking by tile columns
  constexpr bool EINV = MODE == 5 || MODE == 2 || LEFT;   // diagonal inverses formed during the factorisation
  constexpr int PS = EINV ? P + 16 : P;            // panel column stride
  static_assert(3 * P + 4 * PS + 3 * P <= wave_lds_elems(G, MODE), "factorisation LDS");
  T* sy = work + 4 * PS;               // border row y_J
  T* sdk = sy + P;                     // pivots d_k
  T* swk = sdk + P;                    // border entries w_k

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
  const int l = b1 - b0, m = n1 - n0;
  // prediction pads the neighbour rows with identity up to a panel boundary
  const int mq = MODE == 4 ? pred_rows(m) : m;
  const int p = mq + l;
  // rows that hold a point (the rest of the P rows are identity padding)
  auto real_row = [&](int i) __attribute__((always_inline)) { return i < p && (MODE != 4 || i < m || i >= mq); };
  if (MODE == 4 && l == 0) return;
  const double* org = (MODE == 4 ? a.locs2 : a.locs) + (size_t)b0 * a.d;   // coordinate origin: the block's first point

  for (int i = ln; i < P; i += 64) {
    if (real_row(i)) {
      const double* src;
      if (MODE == 4) {
        const bool nb = i < m;
        src = nb ? a.locs + (size_t)a.nbr_idx[n0 + i] * a.d : a.locs2 + (size_t)(b0 + i - mq) * a.d;
        sy[i] = nb ? T(a.y[a.nbr_idx[n0 + i]]) : T(0);   // the border row is [y_N, 0]
      } else {
        const int g = (i < m) ? a.nbr_idx[n0 + i] : (b0 + i - m);
        src = a.locs + (size_t)g * a.d;
        if (MODE != 3) sy[i] = T(a.y[g]);
      }
      for (int k = 0; k < 3; ++k)
        su[k * P + i] = k < a.d ? T((src[k] - org[k]) * (th.inv_scale[k] * (LOG2U ? kLog2E : 1.0))) : T(0);
    } else {
      if (MODE != 3) sy[i] = T(0);
      for (int k = 0; k < 3; ++k) su[k * P + i] = T(0);
    }
  }
  wave_lds_sync();
  const size_t o = (size_t)tt * a.bc + b;
  // tile slot (MODE 1-3, 6): the NT factor tiles (MODES 2, 6: the diagonal
  // ones replaced by their inverses), then the border row w (16 G elements)
  constexpr int SLOT = NT * 256 + 16 * G;
  T* Lg = reinterpret_cast<T*>(a.tiles) + (size_t)(wi - a.item_base) * SLOT;
  double acc_ll = 0.0;
  int flag = 0;
  const MaternF<T, GEN> mc(th);
  acc_t acc[NT];   // the bordered matrix, then its factor (unused by MODE 3)
  if constexpr (MODE != 3) {   // MODE 3 starts from the factor tiles of a MODE 2 or 6 launch

  // ---- generate the bordered joint matrix in the accumulator tiles ----------
  const T sig2 = T(th.sigma2), nug = T(th.nugget);
  // closed forms: -sigma2 (1 + c1 x + c2 x^2) e^-x with the scale and sign in
  // the coefficients
  T ns0 = T(0), ns1 = T(0), ns2 = T(0);
  if constexpr (!GEN) {
    const double u1 = LOG2U ? kLn2 : 1.0;
    ns0 = -sig2;
    ns1 = T(-th.sigma2 * (double)mc.c1 * u1);
    ns2 = T(-th.sigma2 * (double)mc.c2 * u1 * u1);
  }
  // mode 6: tile row I's coordinates (row M::row(lg, r) of the tile in ri[r])
  // and the generation of one tile, as in the loop below
  auto row_coords = [&](int I, T (&ri)[4][3]) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I * 16 + M::row(lg, r);
      ri[r][0] = su[i];
      ri[r][1] = su[P + i];
      ri[r][2] = su[2 * P + i];
    }
  };
  auto gen_tile = [&](auto I_c, auto J_c, const T (&ri)[4][3]) __attribute__((always_inline)) {
    constexpr int I = decltype(I_c)::value, J = decltype(J_c)::value;
    const int j = J * 16 + lr;
    const T sj0 = su[j], sj1 = su[P + j], sj2 = su[2 * P + j];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I * 16 + M::row(lg, r);
      const T dx = ri[r][0] - sj0, dy = ri[r][1] - sj1, dz = ri[r][2] - sj2;
      const T x = sqrt_fast<T>(dx * dx + dy * dy + dz * dz);
      // the tiles hold the negated matrix (updates add L L^T)
      T v;
      if constexpr (GEN) v = -(sig2 * mc.rho(x));
      else if constexpr (LOG2U) v = mc.neg_cov_log2(x, ns0, ns1, ns2);
      else v = mc.neg_cov(x, ns0, ns1, ns2);
      if constexpr (I == J) v -= (i == j) ? nug : T(0);   // the nugget: same-index pairs only
      if (!(real_row(i) && real_row(j))) v = (i == j) ? T(-1) : T(0);
      acc[tix(I, J)][r] = v;
    }
    if (I == (p >> 4)) {  // border row p: y_J
      const T yb = sy[j];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (I * 16 + M::row(lg, r) == p && j < p) acc[tix(I, J)][r] = -yb;
    }
    // D = 0 * 0 + C: hands the finished tile to the accumulator registers now,
    // so the generated values do not pile up in VGPRs until the first update
    // (the FP32 gradient kernels up to G = 9 keep the tiles in VGPRs and skip it)
    if constexpr (!(sizeof(T) == 4 && G <= 9 && (MODE == 5 || MODE == 2)))
      acc[tix(I, J)] = M::op(T(0), T(0), acc[tix(I, J)]);
  };
  if constexpr (!LEFT) {   // the whole matrix now (mode 6: a tile column at a time, through gen_tile)
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
        // the tiles hold the negated matrix (updates add L L^T)
        T v;
        if constexpr (GEN) v = -(sig2 * mc.rho(x));
        else if constexpr (LOG2U) v = mc.neg_cov_log2(x, ns0, ns1, ns2);
        else v = mc.neg_cov(x, ns0, ns1, ns2);
        if constexpr (I == J) v -= (i == j) ? nug : T(0);   // the nugget: same-index pairs only
        if (!(real_row(i) && real_row(j))) v = (i == j) ? T(-1) : T(0);
        acc[tix(I, J)][r] = v;
      }
      if (I == (p >> 4)) {  // border row p: y_J
        const T yb = sy[j];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (I * 16 + M::row(lg, r) == p && j < p) acc[tix(I, J)][r] = -yb;
      }
      // D = 0 * 0 + C: hands the finished tile to the accumulator registers now,
      // so the generated values do not pile up in VGPRs until the first update
      // (the FP32 gradient kernels up to G = 9 keep the tiles in VGPRs and skip it)
      if constexpr (!(sizeof(T) == 4 && G <= 9 && (MODE == 5 || MODE == 2)))
        acc[tix(I, J)] = M::op(T(0), T(0), acc[tix(I, J)]);
    });
  });
  }

  // ---- factorisation, four columns per step -----------------------------------
  T* pan = work;  // pan[c * PS + row], c < 4
  // MODES 5, 2 and 6: the 16 rows appended below the matrix while tile column K is
  // eliminated, R = e_j^T at column 16 K + j (zero left of the tile column,
  // so earlier columns leave them untouched).  After the tile column they hold
  // R L_KK^-T = L_KK^-T, and the transpose of that, inv(L_KK), replaces L_KK
  // in the tiles (nothing in the factorisation reads L_KK afterwards).  Held
  // negated like the matrix tiles.
  acc_t einv;
  // columns c0 .. c0 + 3 of tile column Kc to the panel
  auto publish = [&](auto Kc_c, int c0) __attribute__((always_inline)) {
    constexpr int Kc = decltype(Kc_c)::value;
    if (lr >= c0 && lr < c0 + 4) {
      static_for<Kc, G>(BV_CI(I) {
        BV_CV(I);
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[(lr - c0) * PS + I * 16 + M::row(lg, r)] = acc[tix(I, Kc)][r];
      });
      if (EINV) {
#pragma unroll
        for (int r = 0; r < 4; ++r) pan[(lr - c0) * PS + P + M::row(lg, r)] = einv[r];
      }
    }
  };
  // the panel at column k0: 4 x 4 diagonal block (same values in every lane),
  // then its rows from the diagonal tile down (zero above the block, L_dd in
  // it, TRSM below); pivots and border entries to LDS
  auto factor_panel = [&](int k0) __attribute__((always_inline)) {
    T Ld[4][4], rinv[4], piv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) Ld[r][c] = r >= c ? -pan[c * PS + k0 + r] : T(0);   // panel holds -A
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
    const int i0 = k0 & ~15;
    constexpr int NCH = (PS + 63) / 64;   // 64-row chunks of the panel
    // every chunk's entries are read before any is used (the row index is
    // clamped into the panel; the clamped lanes store nothing)
    T pv[NCH][4];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int i = i0 + ln + 64 * q;
      const int ic = i < PS ? i : PS - 1;
#pragma unroll
      for (int c = 0; c < 4; ++c) pv[q][c] = pan[c * PS + ic];
    }
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int i = i0 + ln + 64 * q;
      if (i < PS) {
        // every lane runs the substitution, which also yields the rows of the
        // diagonal block up to their diagonal (the operations that formed Ld);
        // right of the diagonal there, and above the block, is zero.  Only the
        // first chunk holds such rows (i0 + 64 > k0 + 3).  An appended row j
        // stands for column i0 + j.
        T x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          T v = -pv[q][c];
#pragma unroll
          for (int j = 0; j < c; ++j) v -= x[j] * Ld[c][j];
          x[c] = v * rinv[c];
          if (q == 0) x[c] = (i < P ? i : i0 + (i - P)) - k0 < c && i < P ? T(0) : x[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) pan[c * PS + i] = x[c];
        if (i == p) {
#pragma unroll
          for (int c = 0; c < 4; ++c) swk[k0 + c] = x[c];
        }
      }
    }
    if (k0 + 4 > p) {
      // the panel holds padding columns (at and beyond p, the last ones): they
      // become identity columns.  What the substitution wrote there fed only
      // later columns of the panel, which are padding too.
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        const int i = i0 + ln + 64 * q;
        if (i < PS) {
          const int di = (i < P ? i : i0 + (i - P)) - k0;
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (k0 + c >= p) pan[c * PS + i] = di == c ? T(1) : T(0);
        }
      }
    }
    if (ln == 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sdk[k0 + c] = piv[c];
      }
    }
  };

  const int kend = MODE == 4 ? mq : p;   // columns to eliminate
  static_for<0, G>(BV_CI(K) {
    BV_CV(K);
    if (K * 16 >= kend) return;
    if constexpr (LEFT) {
      // tile column K: generated now, then updated with the stored columns to
      // its left, C_IK += L_IJ L_KJ^T (J < K, 16-wide contractions as four
      // k-steps; both operands take element (lane % 16, 4 s + lane / 16) of
      // their stored tile)
      static_for<K, G>(BV_CI(I) {
        BV_CV(I);
        T ri[4][3];
        row_coords(I, ri);
        gen_tile(std::integral_constant<int, I>{}, std::integral_constant<int, K>{}, ri);
      });
      for (int Jp = 0; Jp < K; ++Jp) {
        const T* LK = Lg + (size_t)(K * (K + 1) / 2 + Jp) * 256;
        T bq[4];
#pragma unroll
        for (int sq = 0; sq < 4; ++sq) bq[sq] = LK[M::at(lr, 4 * sq + lg)];
        static_for<K, G>(BV_CI(I) {
          BV_CV(I);
          const T* LI = Lg + (size_t)(I * (I + 1) / 2 + Jp) * 256;
          T aq[4];
#pragma unroll
          for (int sq = 0; sq < 4; ++sq) aq[sq] = LI[M::at(lr, 4 * sq + lg)];
#pragma unroll
          for (int sq = 0; sq < 4; ++sq) acc[tix(I, K)] = M::op(aq[sq], bq[sq], acc[tix(I, K)]);
        });
      }
    }
    if constexpr (EINV) {
      // -e_j for the columns the loop below eliminates; columns it skips (at
      // and beyond kend: the border column and the padding) keep +e_j, the
      // identity of the inverse there
#pragma unroll
      for (int r = 0; r < 4; ++r)
        einv[r] = M::row(lg, r) == lr ? (K * 16 + lr < kend ? T(-1) : T(1)) : T(0);
    }
    if constexpr (sizeof(T) == 4 && (MODE == 5 || MODE == 2)) {
      // FP32 gradient, one step per panel of four columns: the rank-4 update of tile
      // column K first (the next panel's columns are in it) and the finished
      // columns kept, then the next panel is published before the update of
      // the tiles right of column K is issued, and its factorisation follows
      // while the matrix core still works on that update.  (FP64 keeps the
      // plain order: its tiles leave no registers for the longer-lived panel;
      // the value and prediction kernels measured faster in it as well.)
      publish(std::integral_constant<int, K>{}, 0);
      wave_lds_sync();
      factor_panel(K * 16);
      wave_lds_sync();
#pragma nounroll
      for (int c0 = 0;; c0 += 4) {
        T v[G];
        static_for<K, G>(BV_CI(I) {
          BV_CV(I);
          v[I] = pan[lg * PS + I * 16 + lr];
        });
        static_for<K, G>(BV_CI(I) {
          BV_CV(I);
          acc[tix(I, K)] = M::op(v[I], v[K], acc[tix(I, K)]);
        });
        if (EINV) einv = M::op(pan[lg * PS + P + lr], v[K], einv);
        if (MODE != 0 && MODE != 4 && lr >= c0 && lr < c0 + 4) {
          // keep the finished factor columns in the tiles
          static_for<K, G>(BV_CI(I) {
            BV_CV(I);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[tix(I, K)][r] = pan[(lr - c0) * PS + I * 16 + M::row(lg, r)];
          });
          if (EINV) {
#pragma unroll
            for (int r = 0; r < 4; ++r) einv[r] = pan[(lr - c0) * PS + P + M::row(lg, r)];
          }
        }
        // the rank-4 update of the tiles right of tile column K
        auto trailing = [&]() __attribute__((always_inline)) {
          static_for<K + 1, G>(BV_CI(I) {
            BV_CV(I);
            static_for<K + 1, I + 1>(BV_CI(J) {
              BV_CV(J);
              acc[tix(I, J)] = M::op(v[I], v[J], acc[tix(I, J)]);
            });
          });
        };
        const bool next = c0 + 4 < 16 && K * 16 + c0 + 4 < kend;
        wave_lds_sync();
        if (next) publish(std::integral_constant<int, K>{}, c0 + 4);
        wave_lds_sync();
        trailing();
        if (!next) break;
        factor_panel(K * 16 + c0 + 4);
        wave_lds_sync();
      }
    } else {
#pragma nounroll
      for (int c0 = 0; c0 < 16; c0 += 4) {
        const int k0 = K * 16 + c0;
        if (k0 >= kend) break;
        publish(std::integral_constant<int, K>{}, c0);
        wave_lds_sync();
        factor_panel(k0);
        wave_lds_sync();
        T v[G];
        static_for<K, G>(BV_CI(I) {
          BV_CV(I);
          v[I] = pan[lg * PS + I * 16 + lr];
        });
        static_for<K, G>(BV_CI(I) {
          BV_CV(I);
          static_for<K, (LEFT ? K + 1 : I + 1)>(BV_CI(J) {   // mode 6: its own tile column only
            BV_CV(J);
            acc[tix(I, J)] = M::op(v[I], v[J], acc[tix(I, J)]);
          });
        });
        if (EINV) einv = M::op(pan[lg * PS + P + lr], v[K], einv);
        if (MODE != 0 && MODE != 4 && lr >= c0 && lr < c0 + 4) {
          // keep the finished factor columns in the tiles
          static_for<K, G>(BV_CI(I) {
            BV_CV(I);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[tix(I, K)][r] = pan[(lr - c0) * PS + I * 16 + M::row(lg, r)];
          });
          if (EINV) {
#pragma unroll
            for (int r = 0; r < 4; ++r) einv[r] = pan[(lr - c0) * PS + P + M::row(lg, r)];
          }
        }
        wave_lds_sync();
      }
    }
    if constexpr (EINV) {
      // inv(L_KK) = (L_KK^-T)^T into the diagonal tile, transposed through LDS
#pragma unroll
      for (int r = 0; r < 4; ++r) pan[lr * 16 + M::row(lg, r)] = einv[r];
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[tix(K, K)][r] = pan[M::row(lg, r) * 16 + lr];
      wave_lds_sync();
    }
    if constexpr (LEFT) {
      // the finished tile column to the item's slot; the later columns read it
      // back through global memory (hence the workgroup barrier)
      static_for<K, G>(BV_CI(I) {
        BV_CV(I);
#pragma unroll
        for (int r = 0; r < 4; ++r) Lg[(I * (I + 1) / 2 + K) * 256 + ln * 4 + r] = acc[tix(I, K)][r];
      });
      __syncthreads();
    }
  });

  if constexpr (MODE == 4) {
    // ---- prediction outputs from the trailing tiles (they hold -A) ------------
    int bad = 0;
    for (int k = ln; k < m; k += 64) bad |= !((double)sdk[k] > 0.0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bad |= __shfl_xor(bad, off, 64);
    const double nanv = __builtin_nan("");
    double* pm = a.out_mean + b0;
    double* pv = a.out_var + b0;
    double* pc = a.out_cov ? a.out_cov + (size_t)b * a.ldc * a.ldc : nullptr;
    static_for<0, G>(BV_CI(I) {
      BV_CV(I);
      if (I * 16 > p) return;
      static_for<0, I + 1>(BV_CI(J) {
        BV_CV(J);
        if (J * 16 + 15 < mq) return;
        const int j = J * 16 + lr;
        if (j < mq || j >= p) return;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = I * 16 + M::row(lg, r);
          const double v = (double)acc[tix(I, J)][r];
          if (i == p) {
            pm[j - mq] = bad ? nanv : v;            // border row: -(-mu)
          } else if (i >= j && i < p) {
            const double c = bad ? nanv : -v;       // Schur complement: Sigma_B
            if (i == j) pv[j - mq] = c;
            if (pc) {
              pc[(size_t)(i - mq) * a.ldc + (j - mq)] = c;
              pc[(size_t)(j - mq) * a.ldc + (i - mq)] = c;
            }
          }
        }
      });
    });
    return;
  }

  // ---- log-determinant, quadratic form and pivot guard (FP64) -----------------
  const double guard = a.fp32_guard == 2 ? INFINITY
      : a.fp32_guard ? fmax(0.5 * th.nugget, (double)p * 1.1920928955078125e-07 * (th.sigma2 + th.nugget))
      : 0.0;
  for (int k = ln; k < p; k += 64) {
    const double dd = (double)sdk[k];
    if (!(dd > guard)) flag |= a.fp32_guard ? 1 : 2;
    if (!(dd > 0.0)) flag |= 2;
    if (k >= m) {
      const double wk = (double)swk[k];
      // FP32 pivots: log2 by the hardware (about 1 ulp of the FP32 value)
      const double lgd = sizeof(T) == 4 ? (double)__builtin_amdgcn_logf((float)sdk[k]) * kLn2 : log(dd);
      acc_ll += lgd + wk * wk;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc_ll += __shfl_down(acc_ll, off, 64);
    flag |= __shfl_down(flag, off, 64);
  }
  if (MODE == 0 || MODE == 2 || MODE == 6) {
    if (ln == 0) {
      a.partial[o] = (flag & 2) && !a.fp32_guard ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
      a.flag[o] = flag | a.flag_or;
    }
  }
  if (MODE == 0) return;
  if constexpr (MODE != 5) {
    // the factor leaves the registers for this item's slot of the tile buffer
    // (accumulator order, 256 elements per tile), so the adjoint's phases do not
    // hold the tiles in registers
    if constexpr (!LEFT) {   // (mode 6 stored its tiles column by column)
      static_for<0, NT>(BV_CI(t) {
        BV_CV(t);
#pragma unroll
        for (int r = 0; r < 4; ++r) Lg[t * 256 + ln * 4 + r] = acc[t][r];
      });
    }
    // the border row w = L^-1 y_J (the diagonal tiles no longer hold it in MODES 2, 6)
    for (int j = ln; j < P; j += 64) Lg[NT * 256 + j] = j < p ? swk[j] : T(0);
    __syncthreads();
  }
  if (MODE == 2 || MODE == 6) return;
  } else {
    flag = a.flag[o];   // written by the factorisation launch
  }

  constexpr int CH = wave_chunk(G);   // right-hand sides per pass
  constexpr int NQ = (CH + 15) / 16;             // 16-column tiles of one pass
  constexpr int LDX = CH + 1;
  // with CH < 32 the second 16-column tile is partly outside a row: its reads
  // there are harmless (other columns of the MFMA results), its writes masked
  auto colok = [&](int q) __attribute__((always_inline)) { return (q + 1) * 16 <= CH || q * 16 + lr < CH; };
  constexpr int GM = G > 1 ? G - 1 : 1;   // tile rows above a diagonal step, at most
  const int nr = l + 2;
  const int Gp = (p + 15) >> 4;
  T* X = work;   // X[row * LDX + col], one chunk of right-hand sides
  // clears X (and the 32 elements after it) with 16-byte stores
  auto zero_x = [&]() __attribute__((always_inline)) {
    constexpr int V = 16 / (int)sizeof(T);
    static_assert((P * LDX + 32) % V == 0 && (3 * P * sizeof(T)) % 16 == 0, "16-byte stores into X");
    typedef T vec_t __attribute__((ext_vector_type(V)));
    vec_t* xv = reinterpret_cast<vec_t*>(X);
    for (int e = ln; e < (P * LDX + 32) / V; e += 64) xv[e] = vec_t(0);
  };

  const T irange = T(th.inv_range);
  T dh0 = T(0), dh1 = T(0), dh2 = T(0);   // closed forms: d rho / d range coefficients over the range
  if constexpr (!GEN) {
    const double u1 = LOG2U ? kLn2 : 1.0;
    dh0 = T((double)mc.g0 * th.inv_range * u1);
    dh1 = T((double)mc.g1 * th.inv_range * u1 * u1);
    dh2 = T((double)mc.g2 * th.inv_range * u1 * u1 * u1);
  }
  // d/d sigma2 needs no entry of dK: with d K_J / d sigma2 = (K_J - nugget I) / sigma2,
  // <W, K_J> = ||w||^2 - ||w_N||^2 - l (the quadratic forms of y_J and y_N, and
  // tr(X_R^T K_J X_R) = l) and tr W = 2 d l / d nugget, so that
  // d l / d sigma2 = (sum_{k >= m} w_k^2 - l - nugget tr W) / (2 sigma2)
  double g1 = 0.0, g2 = 0.0, qb = 0.0, g3 = 0.0;   // g3: <W, d rho / d nu> (Bessel form, on request)
  const bool want_nu = GEN && a.gnu != nullptr;
  // W = alpha alpha^T - b b^T - X_R X_R^T over the right-hand sides [cb, cb + nc)
  // held in X, contracted with dK regenerated entry by entry
  auto contract = [&](int cb, int nc) __attribute__((always_inline)) {
    // the next tile's MFMA chain is issued before this tile's contraction
    const int nk = (nc + 3) >> 2;
    for (int I = 0; I < Gp; ++I) {
      T av[CH / 4];
#pragma unroll
      for (int kq = 0; kq < CH / 4; ++kq) {
        const int q = 4 * kq + lg;
        av[kq] = (cb + q == 0 ? T(1) : T(-1)) * X[(I * 16 + lr) * LDX + q];
      }
      T ri[4][3];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * 16 + M::row(lg, r);
        ri[r][0] = su[i];
        ri[r][1] = su[P + i];
        ri[r][2] = su[2 * P + i];
      }
      auto wtile = [&](int J) __attribute__((always_inline)) {
        // all B operands are read before the first product (the reads stay in
        // the row: 4 kq + lg < CH), so the chain waits for LDS once
        T xb[CH / 4];
#pragma unroll
        for (int kq = 0; kq < CH / 4; ++kq) xb[kq] = X[(J * 16 + lr) * LDX + 4 * kq + lg];
        acc_t c;
#pragma unroll
        for (int r = 0; r < 4; ++r) c[r] = T(0);
#pragma unroll
        for (int kq = 0; kq < CH / 4; ++kq)
          if (kq < nk) c = M::op(av[kq], xb[kq], c);
        return c;
      };
      acc_t cn = wtile(0);
      for (int J = 0; J <= I; ++J) {
        const acc_t c = cn;
        if (J < I) cn = wtile(J + 1);
        const int j = J * 16 + lr;
        const T sj0 = su[j], sj1 = su[P + j], sj2 = su[2 * P + j];
        T s1 = T(0), s2 = T(0), s3 = T(0);
        auto entry = [&](int r) __attribute__((always_inline)) {
          const T dx = ri[r][0] - sj0, dy = ri[r][1] - sj1, dz = ri[r][2] - sj2;
          const T x = sqrt_fast<T>(dx * dx + dy * dy + dz * dz);
          if constexpr (GEN) {
            if (want_nu) {
              T dr, dn;
              mc.drange_dnu(x, irange, dr, dn);
              s1 += c[r] * dr;
              s3 += c[r] * dn;
            } else {
              s1 += c[r] * mc.drange(x, irange);
            }
          } else {
            if constexpr (LOG2U) s1 += c[r] * mc.drange_scaled_log2(x, dh0, dh1, dh2);
            else s1 += c[r] * mc.drange_scaled(x, dh0, dh1, dh2);
          }
        };
        if ((I + 1) * 16 <= p) {   // a tile inside the point rows (wave-uniform)
#pragma unroll
          for (int r = 0; r < 4; ++r) entry(r);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (I * 16 + M::row(lg, r) < p && j < p) entry(r);
        }
        if (I == J) {   // d K / d nugget is the identity
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (M::row(lg, r) == lr && j < p) s2 += c[r];
        }
        const double wgt = I == J ? 1.0 : 2.0;
        g1 += wgt * (double)s1;
        g2 += (double)s2;
        if (GEN) g3 += wgt * (double)s3;
      }
    }
  };

  if constexpr (MODE == 5) {
    // ---- factor kept in the registers (its diagonal tiles already replaced by
    // their inverses), CH right-hand sides per pass ---------------------------
    // border row of the bordered factor, w = L^-1 y_J, from the factorisation's
    // LDS record to LDS past the right-hand sides (which overwrite the record)
    T* sw = work + wave_max(4 * PS + 3 * P, P * LDX + 32);
    static_assert(3 * P + wave_max(4 * PS + 3 * P, P * LDX + 32) + P <= wave_lds_elems(G, MODE), "LDS of w");
    for (int j = ln; j < P; j += 64) {
      const T w = j < p ? swk[j] : T(0);
      sw[j] = w;
      if (j >= m && j < p) qb += (double)w * (double)w;
    }
    for (int cb = 0; cb < nr; cb += CH) {
    const int nc = nr - cb < CH ? nr - cb : CH;
    wave_lds_sync();
    // columns cb .. cb + nc - 1 of the right-hand sides [ w | [z; 0] | [0; I_l] ]
    zero_x();
    wave_lds_sync();
    for (int c = ln; c < nc; c += 64)
      if (cb + c >= 2) X[(m + cb + c - 2) * LDX + c] = T(1);
    if (cb == 0) {
      for (int j = ln; j < p; j += 64) {
        X[j * LDX] = sw[j];
        if (j < m) X[j * LDX + 1] = sw[j];
      }
    }
    wave_lds_sync();
    // X <- L^-T X, tile row by tile row from the bottom.  Every product
    // contracts over the rows of a factor tile, so the accumulator registers
    // serve as the A operand as they are: k-step s of lane (i, k) takes
    // register s, i.e. row M::row(k, s) of the tile, and the B operand takes
    // the same row of X.  The diagonal step's result, in accumulator layout,
    // is then directly the B operand of the updates of the rows above.
    // (all NQ column tiles every step: the columns at and beyond nc are zero
    // and stay zero, so no step branches on the chunk width)
    static_for_down<0, G>(BV_CI(K) {
      BV_CV(K);
      if (K >= Gp) return;
      acc_t dq[NQ];
      T xb[NQ][4];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) xb[q][sb] = X[(K * 16 + M::row(lg, sb)) * LDX + q * 16 + lr];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dq[q][r] = T(0);
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) dq[q] = M::op(acc[tix(K, K)][sb], xb[q][sb], dq[q]);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (colok(q)) {
#pragma unroll
          for (int r = 0; r < 4; ++r) X[(K * 16 + M::row(lg, r)) * LDX + q * 16 + lr] = dq[q][r];
        }
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) dq[q][r] = -dq[q][r];
      // rows above: X_J -= L_KJ^T X_K
      static_for<0, K>(BV_CI(J) {
        BV_CV(J);
        acc_t cj[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) cj[q][r] = X[(J * 16 + M::row(lg, r)) * LDX + q * 16 + lr];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
#pragma unroll
          for (int q = 0; q < NQ; ++q) cj[q] = M::op(acc[tix(K, J)][sb], dq[q][sb], cj[q]);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (colok(q)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) X[(J * 16 + M::row(lg, r)) * LDX + q * 16 + lr] = cj[q][r];
          }
      });
      wave_lds_sync();
    });
    contract(cb, nc);
    if constexpr (!wave_regadj_passes(G, sizeof(T) == 4)) break;   // one pass: nr <= CH
    }
  } else {
  // border row p of the bordered factor: w = L^-1 y_J, stored after the tiles
  constexpr int NW = (P + 63) / 64;
  T wreg[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int j = ln + 64 * k;
    wreg[k] = j < p ? Lg[NT * 256 + j] : T(0);
    if (j >= m && j < p) qb += (double)wreg[k] * (double)wreg[k];
  }

  // ---- inverses of the diagonal 16 x 16 blocks of L (MODE 1; MODE 3 reads the
  // ones its factorisation launch formed) ---------------------------------------
  if constexpr (MODE == 1) {
  // all Gp blocks staged at once (the border row and the padding become
  // identity rows); lane (c = l % 16, g = l / 16) forms column c of inv(L_KK)
  // for K = g, g + 4, g + 8 by forward substitution, three independent chains
  {
    constexpr int NB = (G + 3) / 4;   // blocks per lane group
    for (int K = 0; K < Gp; ++K) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rw = M::row(lg, r);
        const int i = K * 16 + rw, j = K * 16 + lr;
        T v = Lg[(K * (K + 1) / 2 + K) * 256 + ln * 4 + r];
        if (i >= p || j >= p) v = (i == j) ? T(1) : T(0);
        X[K * kStageStride + rw * 16 + lr] = v;
      }
    }
    wave_lds_sync();
    const int c = lr;
    T x[NB][16];
    const T* Lk[NB];
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      const int K = lg + 4 * jb;
      Lk[jb] = X + (K < Gp ? K : 0) * kStageStride;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        T sum = T(0);
#pragma unroll
        for (int k = 0; k < i; ++k) sum += Lk[jb][i * 16 + k] * x[jb][k];
        const T rd = T(1) / Lk[jb][i * 16 + i];
        x[jb][i] = i < c ? T(0) : (i == c ? rd : -sum * rd);
      }
    }
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      const int K = lg + 4 * jb;
      if (K < Gp) {
        T* dst = Lg + (K * (K + 1) / 2 + K) * 256;
#pragma unroll
        for (int i = 0; i < 16; ++i) dst[M::at(i, c)] = x[jb][i];
      }
    }
  }
  }   // MODE 1
  __syncthreads();

  // ---- X <- L^-T X and the contraction, CH right-hand sides per pass ---------
  for (int cb = 0; cb < nr; cb += CH) {
    const int nc = nr - cb < CH ? nr - cb : CH;
    const int nq = (nc + 15) >> 4;
    wave_lds_sync();
    zero_x();
    wave_lds_sync();
    // column cb + c of [ w | [z; 0] | [0; I_l] ]
    for (int c = ln; c < nc; c += 64)
      if (cb + c >= 2) X[(m + cb + c - 2) * LDX + c] = T(1);
    if (cb == 0) {
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int j = ln + 64 * k;
        if (j < p) {
          X[j * LDX] = wreg[k];
          if (j < m) X[j * LDX + 1] = wreg[k];
        }
      }
    }
    wave_lds_sync();
    for (int K = Gp - 1; K >= 0; --K) {
      const T* Lrow = Lg + (K * (K + 1) / 2) * 256;   // tile row K: tiles (K, 0..K)
      // A operands from the tile buffer: inv(L_KK)^T and -L_KJ^T, J < K
      T ad[4];
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) ad[sb] = Lrow[K * 256 + M::aop(ln, sb)];
      T aj[GM][4];
#pragma unroll
      for (int J = 0; J < GM; ++J)
        if (J < K) {
#pragma unroll
          for (int sb = 0; sb < 4; ++sb) aj[J][sb] = -Lrow[J * 256 + M::aop(ln, sb)];
        }
      // diagonal step: X_K <- inv(L_KK)^T X_K
      acc_t dq[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dq[q][r] = T(0);
        if (q < nq) {
#pragma unroll
          for (int sb = 0; sb < 4; ++sb) dq[q] = M::op(ad[sb], X[(K * 16 + 4 * sb + lg) * LDX + q * 16 + lr], dq[q]);
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (q < nq && colok(q)) {
#pragma unroll
          for (int r = 0; r < 4; ++r) X[(K * 16 + M::row(lg, r)) * LDX + q * 16 + lr] = dq[q][r];
        }
      wave_lds_sync();
      // rows above: X_J -= L_KJ^T X_K (all tiles loaded first, then the MFMA chains)
      if (K > 0) {
        T bq[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int sb = 0; sb < 4; ++sb) bq[q][sb] = X[(K * 16 + 4 * sb + lg) * LDX + q * 16 + lr];
        acc_t cj[GM][2];
#pragma unroll
        for (int J = 0; J < GM; ++J)
          if (J < K) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
              if (q < nq) {
#pragma unroll
                for (int r = 0; r < 4; ++r) cj[J][q][r] = X[(J * 16 + M::row(lg, r)) * LDX + q * 16 + lr];
              }
          }
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
#pragma unroll
          for (int J = 0; J < GM; ++J)
#pragma unroll
            for (int q = 0; q < 2; ++q)
              if (J < K && q < nq) cj[J][q] = M::op(aj[J][sb], bq[q][sb], cj[J][q]);
#pragma unroll
        for (int J = 0; J < GM; ++J)
          if (J < K) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
              if (q < nq && colok(q)) {
#pragma unroll
                for (int r = 0; r < 4; ++r) X[(J * 16 + M::row(lg, r)) * LDX + q * 16 + lr] = cj[J][q][r];
              }
          }
        wave_lds_sync();
      }
    }

    contract(cb, nc);
  }
  }   // MODE != 5
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    qb += __shfl_down(qb, off, 64);
    if (GEN) g3 += __shfl_down(g3, off, 64);
    g1 += __shfl_down(g1, off, 64);
    g2 += __shfl_down(g2, off, 64);
  }
  if (ln == 0) {
    const bool bad = (flag & 2) && !a.fp32_guard;
    if (MODE == 1 || MODE == 5) {
      a.partial[o] = bad ? __builtin_nan("") : -0.5 * (acc_ll + (double)l * kLog2Pi);
      a.flag[o] = flag | a.flag_or;
    }
    a.gpart[3 * o + 0] = bad ? __builtin_nan("") : 0.5 * (qb - (double)l - th.nugget * g2) / th.sigma2;
    a.gpart[3 * o + 1] = bad ? __builtin_nan("") : 0.5 * th.sigma2 * g1;
    a.gpart[3 * o + 2] = bad ? __builtin_nan("") : 0.5 * g2;
    if (want_nu) a.gnu[o] = bad ? __builtin_nan("") : 0.5 * th.sigma2 * g3;
  }
}

template <typename T, int G, int MODE, bool GEN>
static hipError_t launch_wave_g(const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  const size_t lds = sizeof(T) * (size_t)wave_lds_elems(G, MODE);
  hipLaunchKernelGGL((bv_wave_kernel<T, G, MODE, GEN>), dim3(grid), dim3(64), lds, s, a, thp);
  return hipGetLastError();
}

template <typename T, int MODE, bool GEN = false>
static hipError_t launch_wave_t(int g, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  if constexpr (MODE == 5) {   // factor kept in the registers: up to G = 9 (FP32: 10)
    switch (g) {
      case 1: return launch_wave_g<T, 1, MODE, GEN>(a, thp, grid, s);
      case 2: return launch_wave_g<T, 2, MODE, GEN>(a, thp, grid, s);
      case 3: return launch_wave_g<T, 3, MODE, GEN>(a, thp, grid, s);
      case 4: return launch_wave_g<T, 4, MODE, GEN>(a, thp, grid, s);
      case 5: return launch_wave_g<T, 5, MODE, GEN>(a, thp, grid, s);
      case 6: return launch_wave_g<T, 6, MODE, GEN>(a, thp, grid, s);
      case 7: return launch_wave_g<T, 7, MODE, GEN>(a, thp, grid, s);
      case 8: return launch_wave_g<T, 8, MODE, GEN>(a, thp, grid, s);
      case 9: return launch_wave_g<T, 9, MODE, GEN>(a, thp, grid, s);
#if BV_REGADJ_MAX_G32 >= 10
      case 10:   // FP32 only (one wave per SIMD)
        if constexpr (sizeof(T) == 4) return launch_wave_g<T, 10, MODE, GEN>(a, thp, grid, s);
        return hipErrorInvalidValue;
#endif
      default: return hipErrorInvalidValue;
    }
  } else if constexpr (MODE == 6) {   // left-looking factorisation: FP64 above G = 9
    if constexpr (sizeof(T) == 8) {
      if (g == 10) return launch_wave_g<T, 10, MODE, GEN>(a, thp, grid, s);
      if (g == 11) return launch_wave_g<T, 11, MODE, GEN>(a, thp, grid, s);
    }
    return hipErrorInvalidValue;
  } else if constexpr (MODE == 2 || MODE == 3) {   // split gradient: only the classes that use it
    // (FP32: factorisation by mode 2; FP64: by mode 6, adjoint by mode 3 in both)
    if constexpr (sizeof(T) == 4 || MODE == 3) {
      if constexpr (sizeof(T) == 8 || BV_REGADJ_MAX_G32 < 10) {
        if (g == 10) return launch_wave_g<T, 10, MODE, GEN>(a, thp, grid, s);
      }
      if (g == 11) return launch_wave_g<T, 11, MODE, GEN>(a, thp, grid, s);
    }
    return hipErrorInvalidValue;
  } else if constexpr (MODE == 1 && sizeof(T) == 4) {   // FP32 G >= 10 use the split gradient
    switch (g) {
      case 1: return launch_wave_g<T, 1, MODE, GEN>(a, thp, grid, s);
      case 2: return launch_wave_g<T, 2, MODE, GEN>(a, thp, grid, s);
      case 3: return launch_wave_g<T, 3, MODE, GEN>(a, thp, grid, s);
      case 4: return launch_wave_g<T, 4, MODE, GEN>(a, thp, grid, s);
      case 5: return launch_wave_g<T, 5, MODE, GEN>(a, thp, grid, s);
      case 6: return launch_wave_g<T, 6, MODE, GEN>(a, thp, grid, s);
      case 7: return launch_wave_g<T, 7, MODE, GEN>(a, thp, grid, s);
      case 8: return launch_wave_g<T, 8, MODE, GEN>(a, thp, grid, s);
      case 9: return launch_wave_g<T, 9, MODE, GEN>(a, thp, grid, s);
      default: return hipErrorInvalidValue;
    }
  } else {
  switch (g) {
    case 1: return launch_wave_g<T, 1, MODE, GEN>(a, thp, grid, s);
    case 2: return launch_wave_g<T, 2, MODE, GEN>(a, thp, grid, s);
    case 3: return launch_wave_g<T, 3, MODE, GEN>(a, thp, grid, s);
    case 4: return launch_wave_g<T, 4, MODE, GEN>(a, thp, grid, s);
    case 5: return launch_wave_g<T, 5, MODE, GEN>(a, thp, grid, s);
    case 6: return launch_wave_g<T, 6, MODE, GEN>(a, thp, grid, s);
    case 7: return launch_wave_g<T, 7, MODE, GEN>(a, thp, grid, s);
    case 8: return launch_wave_g<T, 8, MODE, GEN>(a, thp, grid, s);
    case 9: return launch_wave_g<T, 9, MODE, GEN>(a, thp, grid, s);
    case 10: return launch_wave_g<T, 10, MODE, GEN>(a, thp, grid, s);
    case 11: return launch_wave_g<T, 11, MODE, GEN>(a, thp, grid, s);
    default: return hipErrorInvalidValue;
  }
  }
}

}  // namespace bv
