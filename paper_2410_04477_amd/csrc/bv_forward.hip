// Fused per-block forward pass of the block Vecchia log-likelihood (Alg. 1).
//
// One workgroup evaluates one block i for one theta.  The joint index set is
// J = N_i followed by B_i (p = m_i + l_i points).  The workgroup
//   1. gathers the p locations (centred on the block's first point and scaled
//      by 1/(range*aniso)) into LDS -- covariance generation, Alg. 1;
//   2. builds K_J in registers: the p x p lower triangle is cut into R x R
//      tiles, one tile per thread, each thread generating its own Matern
//      entries (eq. (maternkernel)) plus the nugget on the diagonal;
//   3. runs right-looking symmetric elimination over the bordered matrix
//      [[K_J], [y_J^T]].  Eliminating the first m_i pivots is the Cholesky of
//      Sigma^con with the TRSM / TRSV of Alg. 1 folded in (the border row
//      becomes L^-1 y_NN); the trailing l_i x l_i block is then
//      Sigma^new = Sigma^lk - Sigma^cor and its border is y_B - mu; its
//      elimination gives L' and v = L'^-1 (y_B - mu).
//   4. accumulates in FP64, for the trailing pivots d_k (k >= m_i),
//      sum (log d_k + y'_k^2 / d_k): this is d_i + u_i of Alg. 1 since
//      L'_kk = sqrt(d_k) and v_k = y'_k / sqrt(d_k).
//
// Step k needs the updated column k; its owners publish it to LDS one step
// ahead (double buffer), so each elimination step costs one barrier.  Only
// the pivots and border values are needed for the log-likelihood, so the
// factor itself is never scaled or stored.
#include "internal.hpp"

namespace bv {

template <typename T, int R, int G>
__global__ void __launch_bounds__(threads_for_grid(G))
bv_fwd_kernel(FwdArgs a, ThetaPack thp) {
  constexpr int P = R * G;
  constexpr int NTILE = G * (G + 1) / 2;
  __shared__ int sidx[P];
  __shared__ T su[3][P];
  __shared__ T colbuf[2][P];
  __shared__ T pivbuf[2];
  __shared__ T ybuf[2];

  const int tid = threadIdx.x;
  // tile owned by this thread: column-major over the lower triangle of tiles
  int J = 0, rem = tid;
  while (J < G && rem >= G - J) {
    rem -= G - J;
    ++J;
  }
  const bool has = tid < NTILE;
  const int I = J + rem;

  const int total = a.list ? *a.list_count : a.nsched * a.ntheta;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    int b, tt;
    if (a.list) {
      const int e = a.list[w];
      tt = e / a.bc;
      b = e - tt * a.bc;
    } else {
      tt = w / a.nsched;
      b = a.sched[w - tt * a.nsched];
    }
    const ThetaDev& th = thp.t[tt];
    const int b0 = a.block_ptr[b], b1 = a.block_ptr[b + 1];
    const int n0 = a.nbr_ptr[b], n1 = a.nbr_ptr[b + 1];
    const int l = b1 - b0, m = n1 - n0, p = m + l;

    __syncthreads();  // previous work item fully done with LDS
    for (int i = tid; i < p; i += blockDim.x) {
      const int g = (i < m) ? a.nbr_idx[n0 + i] : (b0 + i - m);
      sidx[i] = g;
      for (int k = 0; k < 3; ++k) {
        T v = T(0);
        if (k < a.d) v = T((a.locs[(size_t)g * a.d + k] - a.locs[(size_t)b0 * a.d + k]) * th.inv_scale[k]);
        su[k][i] = v;
      }
    }
    __syncthreads();

    const T sig2 = T(th.sigma2), nug = T(th.nugget);
    T t[R][R];
    T yv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = I * R + r;
      yv[r] = T(0);
      if (has && I == J && i < p) yv[r] = T(a.y[sidx[i]]);
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const int j = J * R + c;
        T v;
        if (!has) {
          v = T(0);
        } else if (i < p && j < p) {
          const T dx = su[0][i] - su[0][j];
          const T dy = su[1][i] - su[1][j];
          const T dz = su[2][i] - su[2][j];
          const T x = sqrt_<T>(dx * dx + dy * dy + dz * dz);
          v = sig2 * matern_rho<T>(x, th.nu_code);
          if (i == j) v += nug;
        } else {
          v = (i == j) ? T(1) : T(0);  // padding: identity, contributes nothing
        }
        t[r][c] = v;
      }
    }
    // publish column 0
    if (has && J == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = I * R + r;
        colbuf[0][row] = (row > 0) ? t[r][0] : T(0);
      }
      if (I == 0) {
        pivbuf[0] = t[0][0];
        ybuf[0] = yv[0];
      }
    }

    // FP32 guard: in exact arithmetic every pivot is >= the smallest eigenvalue of K_J,
    // which is >= nugget; a pivot below half of it (or below p rounding units of the
    // diagonal) is a rounding artefact and the block is re-run in FP64.
    const double guard = a.fp32_guard == 2 ? INFINITY
        : a.fp32_guard ? fmax(0.5 * th.nugget, (double)p * 1.1920928955078125e-07 * (th.sigma2 + th.nugget))
        : 0.0;
    double acc = 0.0;
    int flag = 0;

    for (int K = 0; K < G; ++K) {
      if (K * R >= p) break;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        const int k = K * R + c;
        if (k >= p) break;
        __syncthreads();
        const int cur = k & 1, nxt = cur ^ 1;
        const T dk = pivbuf[cur];
        const T yk = ybuf[cur];
        if (tid == 0) {
          const double dd = (double)dk;
          if (!(dd > guard)) flag |= a.fp32_guard ? 1 : 2;
          if (!(dd > 0.0)) flag |= 2;
          if (k >= m) {
            const double yy = (double)yk;
            acc += log(dd) + yy * yy / dd;
          }
        }
        const T inv = T(1) / dk;
        const T tk = yk * inv;
        if (has && J >= K) {
          T si[R];
#pragma unroll
          for (int r = 0; r < R; ++r) si[r] = colbuf[cur][I * R + r];
          if (I == J) {
#pragma unroll
            for (int r = 0; r < R; ++r) yv[r] -= si[r] * tk;
          }
#pragma unroll
          for (int r = 0; r < R; ++r) si[r] *= inv;
#pragma unroll
          for (int cc = 0; cc < R; ++cc) {
            const T bj = colbuf[cur][J * R + cc];
#pragma unroll
            for (int r = 0; r < R; ++r) t[r][cc] -= si[r] * bj;
          }
        }
        // publish column k + 1 for the next step
        if (c + 1 < R) {
          if (has && J == K) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int row = I * R + r;
              colbuf[nxt][row] = (row > k + 1) ? t[r][(c + 1) % R] : T(0);
            }
            if (I == K) {
              pivbuf[nxt] = t[(c + 1) % R][(c + 1) % R];
              ybuf[nxt] = yv[(c + 1) % R];
            }
          }
        } else {
          if (has && J == K + 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int row = I * R + r;
              colbuf[nxt][row] = (row > k + 1) ? t[r][0] : T(0);
            }
            if (I == K + 1) {
              pivbuf[nxt] = t[0][0];
              ybuf[nxt] = yv[0];
            }
          }
        }
      }
    }
    if (tid == 0) {
      const size_t o = (size_t)tt * a.bc + b;
      a.partial[o] = (flag & 2) && !a.fp32_guard ? __builtin_nan("") : -0.5 * (acc + (double)l * kLog2Pi);
      a.flag[o] = flag | a.flag_or;
    }
  }
}

template <typename T, int C>
static hipError_t launch_cfg(const FwdArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  constexpr int R = kCfgs[C].R, G = kCfgs[C].G;
  hipLaunchKernelGGL((bv_fwd_kernel<T, R, G>), dim3(grid), dim3(threads_for_grid(G)), 0, s, a, thp);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(int cfg, const FwdArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_cfg<T, 0>(a, thp, grid, s);
    case 1: return launch_cfg<T, 1>(a, thp, grid, s);
    case 2: return launch_cfg<T, 2>(a, thp, grid, s);
    case 3: return launch_cfg<T, 3>(a, thp, grid, s);
    case 4: return launch_cfg<T, 4>(a, thp, grid, s);
    case 5: return launch_cfg<T, 5>(a, thp, grid, s);
    case 6: return launch_cfg<T, 6>(a, thp, grid, s);
    case 7: return launch_cfg<T, 7>(a, thp, grid, s);
    case 8: return launch_cfg<T, 8>(a, thp, grid, s);
    case 9: return launch_cfg<T, 9>(a, thp, grid, s);
    case 10: return launch_cfg<T, 10>(a, thp, grid, s);
    case 11: return launch_cfg<T, 11>(a, thp, grid, s);
    case 12: return launch_cfg<T, 12>(a, thp, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_forward(int cfg, bool fp32, const FwdArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  return fp32 ? launch_t<float>(cfg, a, thp, grid, s) : launch_t<double>(cfg, a, thp, grid, s);
}

}  // namespace bv
