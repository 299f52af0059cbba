// Shared device-side definitions of the block Vecchia HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vecchia.h"

namespace bv {

constexpr int kMaxThetaPerLaunch = 24;   // theta values passed by value in kernel arguments
constexpr double kLog2Pi = 1.83787706640934548356065947281123527;

// One parameter vector as the kernels need it.  inv_scale[k] = 1 / (range * aniso[k]),
// so the Matern argument is x = || (s_i - s_j) * inv_scale ||.
struct ThetaDev {
  double sigma2;
  double nugget;
  double inv_scale[3];
  double inv_range;   // 1 / range (gradient w.r.t. range)
  int nu_code;        // 0: nu = 1/2, 1: nu = 3/2, 2: nu = 5/2
  int pad_;
};

struct ThetaPack {
  ThetaDev t[kMaxThetaPerLaunch];
};

template <typename T> __device__ __forceinline__ T expneg(T x);
template <> __device__ __forceinline__ double expneg<double>(double x) { return exp(-x); }
template <> __device__ __forceinline__ float expneg<float>(float x) { return __expf(-x); }

template <typename T> __device__ __forceinline__ T sqrt_(T x);
template <> __device__ __forceinline__ double sqrt_<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float sqrt_<float>(float x) { return sqrtf(x); }

// Matern correlation rho_nu(x) for half-integer nu, eq. (maternkernel) in closed form.
template <typename T>
__device__ __forceinline__ T matern_rho(T x, int nu_code) {
  const T e = expneg<T>(x);
  if (nu_code == 0) return e;
  if (nu_code == 1) return (T(1) + x) * e;
  return (T(1) + x + x * x * T(1.0 / 3.0)) * e;
}

// Branch-free closed forms: rho = e^-x (1 + c1 x + c2 x^2) with (c1, c2) =
// (0, 0), (1, 0), (1, 1/3) for nu = 1/2, 3/2, 5/2, and
// d rho / d range = (x / range) e^-x (g0 + g1 x + g2 x^2) with (g0, g1, g2) =
// (1, 0, 0), (0, 1, 0), (0, 1/3, 1/3).
template <typename T>
struct MaternCoef {
  T c1, c2, g0, g1, g2;
  __device__ __forceinline__ explicit MaternCoef(int nu_code)
      : c1(nu_code == 0 ? T(0) : T(1)),
        c2(nu_code == 2 ? T(1.0 / 3.0) : T(0)),
        g0(nu_code == 0 ? T(1) : T(0)),
        g1(nu_code == 0 ? T(0) : (nu_code == 1 ? T(1) : T(1.0 / 3.0))),
        g2(nu_code == 2 ? T(1.0 / 3.0) : T(0)) {}
  __device__ __forceinline__ T rho(T x) const { return expneg<T>(x) * (T(1) + x * (c1 + c2 * x)); }
  __device__ __forceinline__ void rho_drange(T x, T inv_range, T& r, T& dr) const {
    const T e = expneg<T>(x);
    r = e * (T(1) + x * (c1 + c2 * x));
    dr = x * inv_range * e * (g0 + x * (g1 + g2 * x));
  }
};

template <typename T> __device__ __forceinline__ T sqrt_fast(T x);
template <> __device__ __forceinline__ double sqrt_fast<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float sqrt_fast<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// rho and x * d rho / d x * (-1) / range, i.e. d rho(h/range) / d range.
template <typename T>
__device__ __forceinline__ void matern_rho_drange(T x, int nu_code, T inv_range, T& rho, T& drho) {
  const T e = expneg<T>(x);
  T g;
  if (nu_code == 0) {
    rho = e;
    g = e;
  } else if (nu_code == 1) {
    rho = (T(1) + x) * e;
    g = x * e;
  } else {
    rho = (T(1) + x + x * x * T(1.0 / 3.0)) * e;
    g = x * T(1.0 / 3.0) * (T(1) + x) * e;
  }
  drho = x * inv_range * g;
}

__host__ __device__ constexpr int threads_for_grid(int G) {
  return ((G * (G + 1) / 2 + 63) / 64) * 64;
}

// Register-tile configurations: tile size R, tile grid G (G x G lower triangle of
// tiles, one tile per thread), joint capacity P = R * G.
struct TileCfg {
  int R, G;
};
constexpr TileCfg kCfgs[] = {
    {1, 10}, {2, 10}, {3, 10}, {4, 10}, {3, 15}, {4, 15}, {4, 18},
    {4, 22}, {5, 22}, {6, 22}, {8, 18}, {7, 22}, {8, 22},
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);

__host__ __device__ inline int cfg_for_joint(int p) {
  for (int c = 0; c < kNumCfgs; ++c)
    if (kCfgs[c].R * kCfgs[c].G >= p) return c;
  return -1;
}

// Matrix-core engine: 16 x 16 tiles, G tile rows for the bordered (p + 1)-row
// matrix, G = 1..kMfmaMaxG; configuration id = G - 1.
constexpr int kMfmaMaxG = 11;
__host__ __device__ inline int cfg_mfma_for_joint(int p) {
  const int g = (p + 1 + 15) / 16;
  return (g >= 1 && g <= kMfmaMaxG) ? g - 1 : -1;
}

enum { kEngineMfma = 0, kEngineTiles = 1, kEngineMfmaWg = 2 };

}  // namespace bv
