// Derivative of the block Vecchia log-likelihood w.r.t. the Matern
// smoothness nu (eq. (maternkernel); Section 3 estimates nu with the other
// parameters).  d K_nu / d nu has no closed form, so the derivative is the
// central difference of two FP64 log-likelihoods at nu (1 +- h), evaluated by
// the one-wave Bessel-form kernels through vecchia_loglik and combined on the
// device.
#include <cmath>

#include "internal.hpp"

namespace bv {

// Orders the Bessel form accepts (the same range vecchia_loglik checks).
constexpr double kDnuNuMin = 0.05, kDnuNuMax = 10.0;

__global__ void nu_diff_kernel(const double* __restrict__ llpm, double inv_step, double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = (llpm[0] - llpm[1]) * inv_step;
}

}  // namespace bv

using namespace bv;

extern "C" int vecchia_loglik_dnu(const vecchia_plan* plan, const double* locs_perm, const double* y_perm, int32_t d,
                                  const int32_t* block_ptr, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                                  const vecchia_theta* theta, int32_t ntheta, double rel_step, double* dnu,
                                  double* tmp, void* stream) {
  if (!plan || !theta || ntheta <= 0 || !dnu || !tmp || !(rel_step > 0.0 && rel_step <= 0.1))
    return VECCHIA_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  for (int t = 0; t < ntheta; ++t) {
    const double nu = theta[t].nu;
    if (!std::isfinite(nu) || !(nu > 0.0)) return VECCHIA_EINVAL;
    if (nu < kDnuNuMin || nu > kDnuNuMax) return VECCHIA_EUNSUPPORTED;
    // stencil nu (1 +- rel_step), clipped to the Bessel form's range
    vecchia_theta pm[2] = {theta[t], theta[t]};
    pm[0].nu = std::fmin(nu * (1.0 + rel_step), kDnuNuMax);
    pm[1].nu = std::fmax(nu * (1.0 - rel_step), kDnuNuMin);
    const double step = pm[0].nu - pm[1].nu;
    if (!(step > 0.0)) return VECCHIA_EINVAL;
    int r;
    if (plan->max_theta >= 2) {
      r = vecchia_loglik(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, pm, 2, VECCHIA_FP64, tmp + 2 * t,
                         nullptr, nullptr, stream);
    } else {
      r = vecchia_loglik(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, pm, 1, VECCHIA_FP64, tmp + 2 * t,
                         nullptr, nullptr, stream);
      if (r == VECCHIA_OK)
        r = vecchia_loglik(plan, locs_perm, y_perm, d, block_ptr, nbr_ptr, nbr_idx, pm + 1, 1, VECCHIA_FP64,
                           tmp + 2 * t + 1, nullptr, nullptr, stream);
    }
    if (r != VECCHIA_OK) return r;
    hipLaunchKernelGGL(nu_diff_kernel, dim3(1), dim3(64), 0, s, tmp + 2 * t, 1.0 / step, dnu + t);
    if (hipGetLastError() != hipSuccess) return VECCHIA_EHIP;
  }
  return VECCHIA_OK;
}
