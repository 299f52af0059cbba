// Adjoint of the per-block chain of Alg. 1: d l_i / d(sigma2, range, nugget).
//
// Block term: l_i = log N(y_J; 0, K_J) - log N(y_N; 0, K_N), J = N_i followed by
// B_i.  With alpha = K_J^-1 y_J, b = K_N^-1 y_N (padded with zeros to J) and
// G = K_J^-1 - pad(K_N^-1),
//   d l_i = 1/2 [ alpha^T dK_J alpha - b^T dK_N b - <G, dK_J> ].
// If K_J = L L^T (L lower, L = [[L_N, 0], [A^T, L']]), then G = R^T R where R is
// the last l_i rows of L^-1, so every quantity comes from one back-substitution
//   X = L^-T [ w | [z; 0] | [0; I_l] ],  w = L^-1 y_J,  z = w[0:m_i],
// giving X = [alpha | b | R^T].  Nothing is stored between the forward and
// the adjoint: the workgroup regenerates K_J, re-factorises it in registers
// (the same elimination as the forward kernel, now also scaling each finished
// column into L), solves with L^T tile row by tile row (the owners of a tile
// row publish it to LDS; all threads update the right-hand sides), and finally
// contracts W = alpha alpha^T - b b^T - X_R X_R^T against dK regenerated entry by
// entry, accumulating in FP64.
//
// Coefficient mode (simulator): with y_J = e_last, alpha = K_J^-1 e_last =
// [-c / s; 1 / s] where c = K_N^-1 k_N,last and s = k_last,last - k^T c, the
// conditional-mean weights and variance of the last point given the others.
#include "internal.hpp"

namespace bv {

template <typename T, int R, int G, int MODE>
__global__ void __launch_bounds__(threads_for_grid(G))
bv_adj_kernel(AdjArgs a, ThetaPack thp) {
  constexpr int P = R * G;
  constexpr int NTILE = G * (G + 1) / 2;
  constexpr int NT = threads_for_grid(G);
  extern __shared__ __align__(16) unsigned char dyn_smem[];
  T* X = reinterpret_cast<T*>(dyn_smem);  // P x ldx, row-major
  __shared__ int sidx[P];
  __shared__ T su[3][P];
  __shared__ T colbuf[2][P];
  __shared__ T pivbuf[2];
  __shared__ T ybuf[2];
  __shared__ T lrow[R][P];
  __shared__ double sred[3][NT / 64];

  const int tid = threadIdx.x;
  int J = 0, rem = tid;
  while (J < G && rem >= G - J) {
    rem -= G - J;
    ++J;
  }
  const bool has = tid < NTILE;
  const int I = J + rem;
  const int ldx = a.ldx;

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
    const int nr = MODE == 0 ? l + 2 : 1;  // right-hand sides of the back-substitution

    __syncthreads();
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

    // ---- forward: generate K_J and factor it, keeping L -------------------
    const T sig2 = T(th.sigma2), nug = T(th.nugget);
    T t[R][R];
    T yv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = I * R + r;
      yv[r] = T(0);
      if (has && I == J && i < p) {
        if (MODE == 0) yv[r] = T(a.y[sidx[i]]);
        else yv[r] = (i == p - 1) ? T(1) : T(0);
      }
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
          v = (i == j) ? T(1) : T(0);
        }
        t[r][c] = v;
      }
    }
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
          if (MODE == 0 && k >= m) {
            const double yy = (double)yk;
            acc += log(dd) + yy * yy / dd;
          }
        }
        const T inv = T(1) / dk;
        const T tk = yk * inv;
        const T sq = sqrt_<T>(dk);
        const T rs = T(1) / sq;
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
        // column k is final: scale it into L; border entry k becomes w_k
        if (has && J == K) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int row = I * R + r;
            t[r][c] = row > k ? t[r][c] * rs : (row == k ? sq : T(0));
          }
          if (I == K) yv[c] = yk * rs;
        }
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

    // ---- right-hand sides -------------------------------------------------
    __syncthreads();
    for (int e = tid; e < P * ldx; e += NT) X[e] = T(0);
    __syncthreads();
    if (has && I == J) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = I * R + r;
        if (i < p) {
          X[i * ldx] = yv[r];                          // w
          if (MODE == 0) {
            X[i * ldx + 1] = i < m ? yv[r] : T(0);     // [z; 0]
            if (i >= m) X[i * ldx + 2 + (i - m)] = T(1);  // [0; I_l]
          }
        }
      }
    }

    // ---- back-substitution X <- L^-T X, one tile row at a time ------------
    const int Gp = (p + R - 1) / R;
    for (int K = Gp - 1; K >= 0; --K) {
      __syncthreads();
      if (has && I == K) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < R; ++c) lrow[r][J * R + c] = t[r][c];
      }
      __syncthreads();
      // diagonal tile: X_K <- L_KK^-T X_K (one thread per right-hand side)
      for (int j = tid; j < nr; j += NT) {
        for (int rr = R - 1; rr >= 0; --rr) {
          const int row = K * R + rr;
          T x = X[row * ldx + j];
          for (int r2 = rr + 1; r2 < R; ++r2) x -= lrow[r2][row] * X[(K * R + r2) * ldx + j];
          X[row * ldx + j] = x / lrow[rr][row];
        }
      }
      __syncthreads();
      // rows above: X_i -= sum_r L[K*R + r][i] X[K*R + r]
      const int nup = K * R * nr;
      for (int e = tid; e < nup; e += NT) {
        const int i = e / nr, j = e - (e / nr) * nr;
        T x = X[i * ldx + j];
#pragma unroll
        for (int r = 0; r < R; ++r) x -= lrow[r][i] * X[(K * R + r) * ldx + j];
        X[i * ldx + j] = x;
      }
    }
    __syncthreads();

    if (MODE == 1) {
      // conditional-mean weights and variance of the last point given the others
      const double al = (double)X[(p - 1) * ldx];
      for (int j = tid; j < m; j += NT) a.coef[(size_t)tt * a.coef_stride + n0 + j] = -(double)X[j * ldx] / al;
      if (tid == 0) {
        a.cvar[(size_t)tt * a.bc + b] = 1.0 / al;
        a.flag[(size_t)tt * a.bc + b] = flag;
      }
      continue;
    }

    // ---- contraction with dK (W accumulated in the tile registers) ---------
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    if (has) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < R; ++c) t[r][c] = T(0);
      const int iI = I * R, jJ = J * R;
      for (int q = 0; q < nr; ++q) {
        const T sgn = q == 0 ? T(1) : T(-1);
        T xi[R], xj[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          xi[r] = sgn * X[(iI + r) * ldx + q];
          xj[r] = X[(jJ + r) * ldx + q];
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int c = 0; c < R; ++c) t[r][c] += xi[r] * xj[c];
      }
      const double wgt = I == J ? 1.0 : 2.0;
      const T irange = T(th.inv_range);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = iI + r;
#pragma unroll
        for (int c = 0; c < R; ++c) {
          const int j = jJ + c;
          if (i < p && j < p) {
            const T dx = su[0][i] - su[0][j];
            const T dy = su[1][i] - su[1][j];
            const T dz = su[2][i] - su[2][j];
            const T x = sqrt_<T>(dx * dx + dy * dy + dz * dz);
            T rho, drho;
            matern_rho_drange<T>(x, th.nu_code, irange, rho, drho);
            const double wv = wgt * (double)t[r][c];
            g0 += wv * (double)rho;
            g1 += wv * (double)drho;
            if (i == j) g2 += (double)t[r][c];
          }
        }
      }
    }
    // workgroup reduction of the three sums (fixed order)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      g0 += __shfl_down(g0, off, 64);
      g1 += __shfl_down(g1, off, 64);
      g2 += __shfl_down(g2, off, 64);
    }
    if ((tid & 63) == 0) {
      sred[0][tid >> 6] = g0;
      sred[1][tid >> 6] = g1;
      sred[2][tid >> 6] = g2;
    }
    __syncthreads();
    if (tid == 0) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int q = 0; q < NT / 64; ++q) {
        s0 += sred[0][q];
        s1 += sred[1][q];
        s2 += sred[2][q];
      }
      const size_t o = (size_t)tt * a.bc + b;
      const bool bad = (flag & 2) && !a.fp32_guard;
      a.partial[o] = bad ? __builtin_nan("") : -0.5 * (acc + (double)l * kLog2Pi);
      a.gpart[3 * o + 0] = bad ? __builtin_nan("") : 0.5 * s0;
      a.gpart[3 * o + 1] = bad ? __builtin_nan("") : 0.5 * th.sigma2 * s1;
      a.gpart[3 * o + 2] = bad ? __builtin_nan("") : 0.5 * s2;
      a.flag[o] = flag | a.flag_or;
    }
  }
}

size_t adjoint_lds_need(int cfg, bool fp32, int ldx) {
  const size_t R = kCfgs[cfg].R, G = kCfgs[cfg].G, P = R * G, e = fp32 ? 4 : 8;
  const size_t nt = threads_for_grid((int)G);
  // X (dynamic) + sidx, su, colbuf, pivbuf, ybuf, lrow, sred
  return e * P * (size_t)ldx + 4 * P + e * (5 * P + 4 + R * P) + 8 * 3 * (nt / 64);
}

template <typename T, int C, int MODE>
static hipError_t launch_adj_cfg(const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  constexpr int R = kCfgs[C].R, G = kCfgs[C].G;
  const size_t dyn = sizeof(T) * (size_t)R * G * a.ldx;
  hipLaunchKernelGGL((bv_adj_kernel<T, R, G, MODE>), dim3(grid), dim3(threads_for_grid(G)), dyn, s, a, thp);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_adj_t(int cfg, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_adj_cfg<T, 0, MODE>(a, thp, grid, s);
    case 1: return launch_adj_cfg<T, 1, MODE>(a, thp, grid, s);
    case 2: return launch_adj_cfg<T, 2, MODE>(a, thp, grid, s);
    case 3: return launch_adj_cfg<T, 3, MODE>(a, thp, grid, s);
    case 4: return launch_adj_cfg<T, 4, MODE>(a, thp, grid, s);
    case 5: return launch_adj_cfg<T, 5, MODE>(a, thp, grid, s);
    case 6: return launch_adj_cfg<T, 6, MODE>(a, thp, grid, s);
    case 7: return launch_adj_cfg<T, 7, MODE>(a, thp, grid, s);
    case 8: return launch_adj_cfg<T, 8, MODE>(a, thp, grid, s);
    case 9: return launch_adj_cfg<T, 9, MODE>(a, thp, grid, s);
    case 10: return launch_adj_cfg<T, 10, MODE>(a, thp, grid, s);
    case 11: return launch_adj_cfg<T, 11, MODE>(a, thp, grid, s);
    case 12: return launch_adj_cfg<T, 12, MODE>(a, thp, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint(int cfg, bool fp32, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  return fp32 ? launch_adj_t<float, 0>(cfg, a, thp, grid, s) : launch_adj_t<double, 0>(cfg, a, thp, grid, s);
}

hipError_t launch_coefficients(int cfg, const AdjArgs& a, const ThetaPack& thp, int grid, hipStream_t s) {
  return launch_adj_t<double, 1>(cfg, a, thp, grid, s);
}

}  // namespace bv
