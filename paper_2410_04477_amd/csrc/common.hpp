// Shared device-side definitions of the block Vecchia HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vecchia.h"

namespace bv {

constexpr int kMaxThetaPerLaunch = 24;   // theta values passed by value in kernel arguments
constexpr double kLog2Pi = 1.83787706640934548356065947281123527;
constexpr double kLn2 = 0.693147180559945309417232121458176568;
constexpr double kLog2E = 1.44269504088896340735992468100189214;

// Order-only constants of the Bessel form (host-computed per theta): the
// order nu = n + mu with |mu| <= 1/2; Gamma(1 + mu), Gamma(1 - mu); Temme's
// Gamma1(mu) = (1/Gamma(1 - mu) - 1/Gamma(1 + mu)) / (2 mu) and Gamma2(mu) =
// (1/Gamma(1 - mu) + 1/Gamma(1 + mu)) / 2; mu pi / sin(mu pi);
// log(2^(1 - nu) / Gamma(nu)) and its derivative in nu, -log 2 - psi(nu).
struct BesselOrder {
  double mu, gplus, gminus, gam1, gam2, mu_pi_csc, lognorm, dlognorm;
  int n;
};

// One parameter vector as the kernels need it.  inv_scale[k] = 1 / (range * aniso[k]),
// so the Matern argument is x = || (s_i - s_j) * inv_scale ||.
struct ThetaDev {
  double sigma2;
  double nugget;
  double inv_scale[3];
  double inv_range;   // 1 / range (gradient w.r.t. range)
  int nu_code;        // 0: nu = 1/2, 1: nu = 3/2, 2: nu = 5/2, 3: any other nu (Bessel form)
  BesselOrder bes;    // nu_code 3: order-only constants of the Bessel form
};

struct ThetaPack {
  ThetaDev t[kMaxThetaPerLaunch];
};

// K_mu(x) and K_(mu+1)(x), |mu| <= 1/2, 0 < x <= 2: Temme's series (N. M.
// Temme, J. Comput. Phys. 19 (1975) 324-337).  With c_k = (x^2/4)^k / k!,
//   K_mu = sum_k c_k f_k,   K_(mu+1) = (2/x) sum_k c_k (p_k - k f_k),
// where p_k, q_k are p_0 = Gamma(1 + mu) (x/2)^-mu / 2 and q_0 = Gamma(1 - mu)
// (x/2)^mu / 2 divided by (1 - mu)..(k - mu) and (1 + mu)..(k + mu), and
// f_k = (k f_(k-1) + p_(k-1) + q_(k-1)) / (k^2 - mu^2) starts from
// f_0 = mu pi / sin(mu pi) [Gamma1 cosh(s) + Gamma2 ln(2/x) sinh(s) / s],
// s = mu ln(2/x).  About 15 terms reach FP64 rounding on this range.
__device__ inline void bessel_k_pair_series(double x, const BesselOrder& o, double& k_mu, double& k_mu1) {
  const double log2x = log(2.0 / x);
  const double s = o.mu * log2x;
  const double sinhc = fabs(s) < 1e-14 ? 1.0 : sinh(s) / s;
  const double es = exp(s);   // (2/x)^mu
  double f = o.mu_pi_csc * (o.gam1 * cosh(s) + o.gam2 * log2x * sinhc);
  double pk = 0.5 * o.gplus * es;
  double qk = 0.5 * o.gminus / es;
  const double quarter_x2 = 0.25 * x * x;
  double ck = 1.0;
  double sum_mu = f, sum_mu1 = pk;
  for (int k = 1; k < 60; ++k) {
    const double dk = (double)k;
    const double dm = dk - o.mu, dp = dk + o.mu;
    f = (dk * f + pk + qk) / (dm * dp);
    pk /= dm;
    qk /= dp;
    ck *= quarter_x2 / dk;
    const double t_mu = ck * f, t_mu1 = ck * (pk - dk * f);
    sum_mu += t_mu;
    sum_mu1 += t_mu1;
    if (fabs(t_mu) <= 1e-17 * fabs(sum_mu) && fabs(t_mu1) <= 1e-17 * fabs(sum_mu1)) break;
  }
  k_mu = sum_mu;
  k_mu1 = sum_mu1 * (2.0 / x);
}

// K_mu(x) and K_(mu+1)(x), |mu| <= 1/2, x > 2: the trapezoidal rule on the
// integral representation K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt,
// whose integrand is analytic and decays doubly exponentially, so the rule
// converges geometrically in 1/h (L. N. Trefethen and J. A. C. Weideman,
// SIAM Review 56 (2014) 385-458).  Step h = min(1/8, 0.7/sqrt(x)) keeps the
// discretisation error below FP64 rounding for |v| <= 3/2 (the integrand's
// width shrinks like 1/sqrt(x)); nodes are added until the integrand falls
// below 1e-18 of the sum, at most 64 (13 to 31 on this range).  e^(+-v t) and
// e^(+-t) advance by multiplication, so each node costs one exponential.
__device__ inline void bessel_k_pair_quad(double x, double mu, double& k_mu, double& k_mu1) {
  const double h = fmin(0.125, 0.7 * rsqrt(x));
  const double a = exp(mu * h), ai = 1.0 / a, b = exp(h), bi = 1.0 / b;
  double emu = 1.0, emui = 1.0, et = 1.0, eti = 1.0;   // e^(mu t), e^(-mu t), e^t, e^-t
  double w = exp(-x);
  double s_mu = 0.5 * w, s_mu1 = 0.5 * w;              // the t = 0 node carries weight 1/2
  for (int k = 1; k < 64; ++k) {
    emu *= a;
    emui *= ai;
    et *= b;
    eti *= bi;
    w = exp(-0.5 * x * (et + eti));
    const double c1 = 0.5 * (emu * et + emui * eti);   // cosh((mu + 1) t)
    s_mu += w * 0.5 * (emu + emui);
    s_mu1 += w * c1;
    if (w * c1 < 1e-18 * s_mu1) break;
  }
  k_mu = h * s_mu;
  k_mu1 = h * s_mu1;
}

// Matern correlation for any nu > 0, eq. (maternkernel) with the modified
// Bessel function of the second kind: rho(x) = 2^(1-nu)/Gamma(nu) x^nu K_nu(x),
// in FP64.  K at the reduced order mu, then raised to nu = n + mu by the
// three-term recurrence K_(v+1) = K_(v-1) + (2 v / x) K_v, which is stable
// upwards for K.  Also returns g = 2^(1-nu)/Gamma(nu) x^(nu+1) K_(nu-1)(x),
// from d/dx [x^nu K_nu(x)] = -x^nu K_(nu-1)(x): d rho(h/range) / d range =
// g / range.  Not inlined: its loops would otherwise be copied into every
// generation site.
__device__ __noinline__ inline void matern_general(double x, const BesselOrder& o, double* rho, double* g) {
  if (!(x > 0.0)) {
    *rho = 1.0;
    *g = 0.0;
    return;
  }
  double k_lo, k_hi;   // K_(v-1), K_v as v climbs from mu
  {
    double k_mu, k_mu1;
    if (x <= 2.0)
      bessel_k_pair_series(x, o, k_mu, k_mu1);
    else
      bessel_k_pair_quad(x, o.mu, k_mu, k_mu1);
    // K_(mu-1) = K_(mu+1) - (2 mu / x) K_mu
    k_lo = o.n == 0 ? k_mu1 - (2.0 * o.mu / x) * k_mu : k_mu;
    k_hi = o.n == 0 ? k_mu : k_mu1;
    for (int v = 1; v < o.n; ++v) {
      const double next = k_lo + (2.0 * (o.mu + v) / x) * k_hi;
      k_lo = k_hi;
      k_hi = next;
    }
  }
  const double nu = o.mu + o.n, logx = log(x);
  *rho = exp(o.lognorm + nu * logx) * k_hi;
  *g = exp(o.lognorm + (nu + 1.0) * logx) * k_lo;
}

// rho and g as matern_general, and d rho / d nu.  K_mu, K_(mu+1) and their
// derivatives in the order come from the trapezoidal rule on
//   K_v(x) = int_0^inf exp(-x cosh t) cosh(v t) dt,
//   d K_v / d v = int_0^inf t exp(-x cosh t) sinh(v t) dt
// for every x > 0 (the same nodes serve all four; the step as in
// bessel_k_pair_quad, nodes until the integrands fall below 1e-18 of the sums
// and t > 1, at most 320: about 110 at x = 1e-4, fewer as x grows).  The
// order is raised by the recurrence K_(v+1) = K_(v-1) + (2 v / x) K_v and its
// derivative D_(v+1) = D_(v-1) + (2 v / x) D_v + (2 / x) K_v (mu moves with
// nu).  Then d rho / d nu = 2^(1-nu)/Gamma(nu) x^nu [K_nu (log x - log 2 -
// psi(nu)) + D_nu].
__device__ __noinline__ inline void matern_general_dnu(double x, const BesselOrder& o, double* rho, double* g,
                                                       double* drho_dnu) {
  if (!(x > 0.0)) {
    *rho = 1.0;
    *g = 0.0;
    *drho_dnu = 0.0;
    return;
  }
  const double h = fmin(0.125, 0.7 * rsqrt(x));
  const double a = exp(o.mu * h), ai = 1.0 / a, b = exp(h), bi = 1.0 / b;
  double emu = 1.0, emui = 1.0, et = 1.0, eti = 1.0;
  const double w0 = exp(-x);
  double k0 = 0.5 * w0, k1 = 0.5 * w0, d0 = 0.0, d1 = 0.0;   // t = 0: weight 1/2, sinh(0) = 0
  for (int k = 1; k < 320; ++k) {
    emu *= a;
    emui *= ai;
    et *= b;
    eti *= bi;
    const double t = k * h;
    const double w = exp(-0.5 * x * (et + eti));
    const double c1 = 0.5 * (emu * et + emui * eti), s1 = 0.5 * (emu * et - emui * eti);
    k0 += w * 0.5 * (emu + emui);
    k1 += w * c1;
    d0 += w * t * 0.5 * (emu - emui);
    d1 += w * t * s1;
    if (t > 1.0 && w * t * c1 < 1e-18 * k1) break;
  }
  k0 *= h;
  k1 *= h;
  d0 *= h;
  d1 *= h;
  double klo, khi, dhi;   // K_(nu-1), K_nu, d K_nu / d nu
  if (o.n == 0) {
    klo = k1 - (2.0 * o.mu / x) * k0;
    khi = k0;
    dhi = d0;
  } else {
    klo = k0;
    khi = k1;
    double dlo = d0;
    dhi = d1;
    for (int v = 1; v < o.n; ++v) {
      const double vv = o.mu + v;
      const double kn = klo + (2.0 * vv / x) * khi;
      const double dn = dlo + (2.0 * vv / x) * dhi + (2.0 / x) * khi;
      klo = khi;
      khi = kn;
      dlo = dhi;
      dhi = dn;
    }
  }
  const double nu = o.mu + o.n, logx = log(x);
  const double c = exp(o.lognorm + nu * logx);
  *rho = c * khi;
  *g = c * x * klo;
  *drho_dnu = c * (khi * (logx + o.dlognorm) + dhi);
}

template <typename T> __device__ __forceinline__ T expneg(T x);
template <> __device__ __forceinline__ double expneg<double>(double x) { return exp(-x); }
template <> __device__ __forceinline__ float expneg<float>(float x) { return __expf(-x); }

// 2^-x: one v_exp_f32 in FP32
template <typename T> __device__ __forceinline__ T exp2neg(T x);
template <> __device__ __forceinline__ double exp2neg<double>(double x) { return exp2(-x); }
template <> __device__ __forceinline__ float exp2neg<float>(float x) { return __builtin_amdgcn_exp2f(-x); }

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
  __device__ __forceinline__ T drange(T x, T inv_range) const {
    return x * inv_range * expneg<T>(x) * (g0 + x * (g1 + g2 * x));
  }
  // -(sigma2 rho(x)) with the scale and sign folded into the coefficients
  // (s0, s1, s2) = -sigma2 (1, c1, c2)
  __device__ __forceinline__ T neg_cov(T x, T s0, T s1, T s2) const { return expneg<T>(x) * (s0 + x * (s1 + s2 * x)); }
  // d rho / d range with 1 / range folded into (h0, h1, h2) = (g0, g1, g2) / range
  __device__ __forceinline__ T drange_scaled(T x, T h0, T h1, T h2) const {
    return x * expneg<T>(x) * (h0 + x * (h1 + h2 * x));
  }
  // the two above for a distance u = x log2(e) (e^-x = 2^-u), the coefficients
  // of u^k carrying the factor ln(2)^k (neg_cov) or ln(2)^(k+1) (drange)
  __device__ __forceinline__ T neg_cov_log2(T u, T s0, T s1, T s2) const {
    return exp2neg<T>(u) * (s0 + u * (s1 + s2 * u));
  }
  __device__ __forceinline__ T drange_scaled_log2(T u, T h0, T h1, T h2) const {
    return u * exp2neg<T>(u) * (h0 + u * (h1 + h2 * u));
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
    matern_general((double)x, t.bes, &r, &g);
    return T(r);
  }
  __device__ __forceinline__ void rho_drange(T x, T inv_range, T& r, T& dr) const {
    double rr, g;
    matern_general((double)x, t.bes, &rr, &g);
    r = T(rr);
    dr = T(g) * inv_range;
  }
  __device__ __forceinline__ T drange(T x, T inv_range) const {
    double rr, g;
    matern_general((double)x, t.bes, &rr, &g);
    return T(g) * inv_range;
  }
  // d rho / d range and d rho / d nu (the derivative in nu by quadrature)
  __device__ __forceinline__ void drange_dnu(T x, T inv_range, T& dr, T& dn) const {
    double rr, g, d;
    matern_general_dnu((double)x, t.bes, &rr, &g, &d);
    dr = T(g) * inv_range;
    dn = T(d);
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
