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
  int nu_code;        // 0: nu = 1/2, 1: nu = 3/2, 2: nu = 5/2, 3: any other nu (Bessel form)
  int nu_n;           // nu_code 3: nu = nu_n + nu_mu, |nu_mu| <= 1/2
  // nu_code 3, order-only constants of the Bessel evaluation (host-computed):
  // Temme's Gamma1(mu), Gamma2(mu), 1/Gamma(1 + mu), 1/Gamma(1 - mu), and
  // log(2^(1 - nu) / Gamma(nu))
  double nu_mu, nu_gam1, nu_gam2, nu_gampl, nu_gammi, nu_lognorm;
};

struct ThetaPack {
  ThetaDev t[kMaxThetaPerLaunch];
};

// Matern correlation for any nu > 0, eq. (maternkernel) with the modified
// Bessel function of the second kind: rho(x) = 2^(1-nu)/Gamma(nu) x^nu K_nu(x),
// in FP64.  K is evaluated at order mu = nu - n (|mu| <= 1/2) by Temme's series
// (Temme 1975) for x <= 2 or Steed's continued fraction CF2 (Thompson and
// Barnett 1987) for x > 2, each giving K_mu and K_(mu+1), then raised to order
// nu by the forward recurrence K_(k+1) = 2k/x K_k + K_(k-1), which is stable for
// K.  Also returns g = 2^(1-nu)/Gamma(nu) x^(nu+1) K_(nu-1)(x), from
// d/dx [x^nu K_nu(x)] = -x^nu K_(nu-1)(x): d rho(h/range) / d range = g / range.
// Not inlined: its loops would otherwise be copied into every generation site.
__device__ __noinline__ inline void matern_general(double x, double mu, double gam1, double gam2, double gampl,
                                                   double gammi, double lognorm, int n, double* rho, double* g) {
  if (!(x > 0.0)) {
    *rho = 1.0;
    *g = 0.0;
    return;
  }
  const double kEps = 1e-16, kPi = 3.14159265358979323846;
  double km, kp;   // K_mu(x), K_(mu+1)(x)
  if (x <= 2.0) {
    // Temme: K_mu = sum c_k f_k, K_(mu+1) = (2/x) sum c_k (p_k - k f_k), c_k = (x^2/4)^k / k!
    const double lx = -log(0.5 * x);   // ln(2/x)
    const double sg = mu * lx;
    const double fact = fabs(mu) < 1e-14 ? 1.0 : kPi * mu / sin(kPi * mu);
    const double fact2 = fabs(sg) < 1e-14 ? 1.0 : sinh(sg) / sg;
    double f = fact * (gam1 * cosh(sg) + gam2 * fact2 * lx);
    const double es = exp(sg);
    double p = 0.5 * es / gampl;    // (x/2)^-mu Gamma(1 + mu) / 2
    double q = 0.5 / (es * gammi);  // (x/2)^mu Gamma(1 - mu) / 2
    const double x24 = 0.25 * x * x;
    double c = 1.0, s0 = f, s1 = p;
    for (int k = 1; k < 200; ++k) {
      const double dk = (double)k;
      f = (dk * f + p + q) / (dk * dk - mu * mu);
      c *= x24 / dk;
      p /= dk - mu;
      q /= dk + mu;
      const double t0 = c * f;
      s0 += t0;
      s1 += c * (p - dk * f);
      if (fabs(t0) < kEps * fabs(s0)) break;
    }
    km = s0;
    kp = s1 * (2.0 / x);
  } else {
    // Steed's algorithm for CF2: K_mu = sqrt(pi / 2x) e^-x / s
    const double a1 = 0.25 - mu * mu;
    double b = 2.0 * (1.0 + x), d = 1.0 / b, h = d, dh = d;
    double q1 = 0.0, q2 = 1.0, q = a1, c = a1, a = -a1;
    double s = 1.0 + q * dh;
    for (int i = 2; i < 1000; ++i) {
      a -= 2.0 * (i - 1);
      c = -a * c / i;
      const double qn = (q1 - b * q2) / a;
      q1 = q2;
      q2 = qn;
      q += c * qn;
      b += 2.0;
      d = 1.0 / (b + a * d);
      dh = (b * d - 1.0) * dh;
      h += dh;
      const double ds = q * dh;
      s += ds;
      if (fabs(ds) < kEps * fabs(s)) break;
    }
    km = sqrt(kPi / (2.0 * x)) * exp(-x) / s;
    kp = km * (mu + x + 0.5 - a1 * h) / x;
  }
  double kn, kn1;   // K_nu, K_(nu-1)
  if (n == 0) {
    kn = km;
    kn1 = kp - (2.0 * mu / x) * km;   // K_(mu-1)
  } else {
    for (int k = 1; k < n; ++k) {
      const double t = (2.0 * (mu + k) / x) * kp + km;
      km = kp;
      kp = t;
    }
    kn = kp;
    kn1 = km;
  }
  const double nu = mu + n, lxn = log(x);
  *rho = exp(lognorm + nu * lxn) * kn;
  *g = exp(lognorm + (nu + 1.0) * lxn) * kn1;
}

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

// The correlation a kernel generates: closed forms (GEN = false), or the
// Bessel form for any nu (GEN = true; FP64 evaluation rounded to T).
template <typename T, bool GEN> struct MaternF;
template <typename T> struct MaternF<T, false> : MaternCoef<T> {
  __device__ __forceinline__ explicit MaternF(const ThetaDev& t) : MaternCoef<T>(t.nu_code) {}
};
template <typename T> struct MaternF<T, true> {
  const ThetaDev& t;
  __device__ __forceinline__ explicit MaternF(const ThetaDev& th) : t(th) {}
  __device__ __forceinline__ T rho(T x) const {
    double r, g;
    matern_general((double)x, t.nu_mu, t.nu_gam1, t.nu_gam2, t.nu_gampl, t.nu_gammi, t.nu_lognorm, t.nu_n, &r, &g);
    return T(r);
  }
  __device__ __forceinline__ void rho_drange(T x, T inv_range, T& r, T& dr) const {
    double rr, g;
    matern_general((double)x, t.nu_mu, t.nu_gam1, t.nu_gam2, t.nu_gampl, t.nu_gammi, t.nu_lognorm, t.nu_n, &rr, &g);
    r = T(rr);
    dr = T(g) * inv_range;
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
