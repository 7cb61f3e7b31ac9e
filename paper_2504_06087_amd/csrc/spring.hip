// The natural-gradient parameter update of the optimisation loop (Methods,
// variational Monte Carlo, eq. spring) and its variant for a gradient that is
// not of the form Obar^T (dL / d log psi) (SI, non-hermitian operator
// gradients in Spring, eq. aux_spring):
//
//   delta = Obar^T (Obar Obar^T + lambda I)^-1 (eps + eps~ - Obar eta delta_prev)
//           + eta delta_prev + delta~_out
//
// with Obar[w] = O[w] - mean_w O[w] the centred per-walker gradients of
// log|psi| (W x P, one row per walker), eps[w] = E_L,w - mean E_L, and for an
// extra gradient delta~ its projection onto the rows of Obar, Obar^T eps~ with
// eps~ = (Obar Obar^T + lambda0 I)^-1 Obar delta~ (a damped pseudo-inverse),
// and the rest delta~_out = delta~ - Obar^T eps~.
//
// The W x W Gram matrix is formed from the uncentred rows by one FP64 MFMA
// GEMM (contraction over the P parameters) and centred afterwards:
// Obar Obar^T = G - r 1^T - 1 r^T + s 1 1^T with G = O O^T, r = G 1 / W,
// s = 1^T G 1 / W^2.  The damped system is solved by a blocked FP64 Cholesky
// factorisation; products with Obar and Obar^T subtract the column mean on
// the fly, so the centred W x P matrix is never formed.
#include "gemm.hpp"
#include "handle.hpp"

namespace fire {

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

constexpr int CHB = 64;          // Cholesky block
constexpr int SPRING_WMAX = 8192;

// mu[p] = (1/W) sum_w O[w][p]
__global__ void k_col_mean(int64_t P, int W, const double* __restrict__ O, double* __restrict__ mu) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int w = 0; w < W; ++w) s += O[(int64_t)w * P + p];
  mu[p] = s / W;
}

FIRE_DEV double block_sum_d(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
  return t;
}

// out[b] = X[b] . v for the rows b of X (one workgroup per row; row b = W:
// the vector mu when given, so that mu . v comes out as out[W])
__global__ __launch_bounds__(256) void k_row_dots(int64_t P, int W, const double* __restrict__ X,
                                                  const double* __restrict__ mu, const double* __restrict__ v,
                                                  double* __restrict__ out) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const double* row = b < W ? X + (int64_t)b * P : mu;
  double s = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) s += row[p] * v[p];
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) out[b] = s;
}

// r[i] = (1/W) sum_j G[i][j]; r[W] = (1/W) sum_i r[i] after k_mean_tail
__global__ __launch_bounds__(256) void k_gram_rowmean(int W, const double* __restrict__ G, double* __restrict__ r) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < W; j += blockDim.x) s += G[(int64_t)i * W + j];
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) r[i] = s / W;
}
__global__ __launch_bounds__(256) void k_mean_tail(int W, double* __restrict__ r) {
  __shared__ double red[4];
  double s = 0.0;
  for (int j = threadIdx.x; j < W; j += blockDim.x) s += r[j];
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) r[W] = s / W;
}

// A = G - r 1^T - 1 r^T + s + lambda I
__global__ void k_gram_center(int W, const double* __restrict__ G, const double* __restrict__ r, double lambda,
                              double* __restrict__ A) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)W * W) return;
  const int i = (int)(q / W), j = (int)(q % W);
  A[q] = G[q] - r[i] - r[j] + r[W] + (i == j ? lambda : 0.0);
}

// ---------------------------------------------------------------------------
// blocked Cholesky A = L L^T (lower, row-major, in place), FP64
// ---------------------------------------------------------------------------
// the diagonal block [k0, k0 + nb)
__global__ __launch_bounds__(256) void k_potrf_diag(int W, int k0, double* __restrict__ A, int* __restrict__ fail) {
  __shared__ double S[CHB][CHB + 1];
  const int nb = W - k0 < CHB ? W - k0 : CHB;
  for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) {
    const int i = q / nb, j = q % nb;
    S[i][j] = A[(int64_t)(k0 + i) * W + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (threadIdx.x == 0) {
      const double d = S[j][j];
      if (!(d > 0.0)) *fail = 1;
      S[j][j] = sqrt(d > 0.0 ? d : 1.0);
    }
    __syncthreads();
    const double djj = S[j][j];
    for (int i = j + 1 + threadIdx.x; i < nb; i += blockDim.x) S[i][j] /= djj;
    __syncthreads();
    // trailing update of the lower triangle of the block
    const int m = nb - j - 1;
    for (int q = threadIdx.x; q < m * m; q += blockDim.x) {
      const int i = j + 1 + q / m, l = j + 1 + q % m;
      if (l <= i) S[i][l] -= S[i][j] * S[l][j];
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) {
    const int i = q / nb, j = q % nb;
    if (j <= i) A[(int64_t)(k0 + i) * W + k0 + j] = S[i][j];
  }
}

// panel rows below the diagonal block: A[i][k0..] <- A[i][k0..] L_kk^-T
__global__ __launch_bounds__(256) void k_trsm_panel(int W, int k0, double* __restrict__ A) {
  __shared__ double Lk[CHB][CHB + 1];
  __shared__ double B[CHB][CHB + 1];
  const int nb = W - k0 < CHB ? W - k0 : CHB;
  const int i0 = k0 + nb + blockIdx.x * CHB;
  const int rows = W - i0 < CHB ? W - i0 : CHB;
  for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) {
    const int i = q / nb, j = q % nb;
    Lk[i][j] = j <= i ? A[(int64_t)(k0 + i) * W + k0 + j] : 0.0;
  }
  for (int q = threadIdx.x; q < rows * nb; q += blockDim.x) {
    const int i = q / nb, j = q % nb;
    B[i][j] = A[(int64_t)(i0 + i) * W + k0 + j];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < rows) {
    for (int j = 0; j < nb; ++j) {
      double x = B[t][j];
      for (int l = 0; l < j; ++l) x -= B[t][l] * Lk[j][l];
      B[t][j] = x / Lk[j][j];
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < rows * nb; q += blockDim.x) {
    const int i = q / nb, j = q % nb;
    A[(int64_t)(i0 + i) * W + k0 + j] = B[i][j];
  }
}

// trailing update A[I][J] -= P_I P_J^T for the tiles I >= J below the panel
__global__ __launch_bounds__(256) void k_syrk_update(int W, int k0, double* __restrict__ A) {
  __shared__ double PI[CHB][33], PJ[CHB][33];
  const int nb = W - k0 < CHB ? W - k0 : CHB;
  const int t0 = k0 + nb;
  // triangular tile index -> (bi, bj), bi >= bj
  const int b = blockIdx.x;
  int bi = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
  while (bi * (bi + 1) / 2 > b) --bi;
  const int bj = b - bi * (bi + 1) / 2;
  const int i0 = t0 + bi * CHB, j0 = t0 + bj * CHB;
  if (i0 >= W || j0 >= W) return;
  const int ri = W - i0 < CHB ? W - i0 : CHB, rj = W - j0 < CHB ? W - j0 : CHB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;   // 16 x 16 threads, 4 x 4 outputs each
  double acc[4][4] = {};
  for (int kc = 0; kc < nb; kc += 32) {
    const int kl = nb - kc < 32 ? nb - kc : 32;
    for (int q = threadIdx.x; q < CHB * 32; q += blockDim.x) {
      const int i = q / 32, k = q % 32;
      PI[i][k] = (i < ri && k < kl) ? A[(int64_t)(i0 + i) * W + k0 + kc + k] : 0.0;
      PJ[i][k] = (i < rj && k < kl) ? A[(int64_t)(j0 + i) * W + k0 + kc + k] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k) {
      double a[4], c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { a[u] = PI[ty + 16 * u][k]; c[u] = PJ[tx + 16 * u][k]; }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * c[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ty + 16 * u, j = tx + 16 * v;
      if (i < ri && j < rj && (i0 + i) >= (j0 + j)) A[(int64_t)(i0 + i) * W + j0 + j] -= acc[u][v];
    }
}

// L y = b (row-oriented: row j of L is read contiguously), then L^T x = y
// (column-oriented on L^T, i.e. again rows of L); one workgroup, the vector
// in LDS.  b is overwritten by x.
__global__ __launch_bounds__(256) void k_chol_solve(int W, const double* __restrict__ L, double* __restrict__ b) {
  extern __shared__ double v[];
  __shared__ double red[4];
  for (int j = threadIdx.x; j < W; j += blockDim.x) v[j] = b[j];
  __syncthreads();
  for (int j = 0; j < W; ++j) {
    double s = 0.0;
    for (int l = threadIdx.x; l < j; l += blockDim.x) s += L[(int64_t)j * W + l] * v[l];
    s = block_sum_d(s, red);
    if (threadIdx.x == 0) v[j] = (v[j] - s) / L[(int64_t)j * W + j];
    __syncthreads();
  }
  for (int j = W - 1; j >= 0; --j) {
    if (threadIdx.x == 0) v[j] /= L[(int64_t)j * W + j];
    __syncthreads();
    const double xj = v[j];
    for (int l = threadIdx.x; l < j; l += blockDim.x) v[l] -= L[(int64_t)j * W + l] * xj;
    __syncthreads();
  }
  for (int j = threadIdx.x; j < W; j += blockDim.x) b[j] = v[j];
}

static hipError_t cholesky_solve(int W, double* A, double* rhs, int* fail, hipStream_t st) {
  for (int k0 = 0; k0 < W; k0 += CHB) {
    const int nb = W - k0 < CHB ? W - k0 : CHB;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, W, k0, A, fail);
    CHECK(hipGetLastError());
    const int rest = W - k0 - nb;
    if (rest > 0) {
      const int nbk = (rest + CHB - 1) / CHB;
      hipLaunchKernelGGL(k_trsm_panel, dim3(nbk), dim3(256), 0, st, W, k0, A);
      CHECK(hipGetLastError());
      hipLaunchKernelGGL(k_syrk_update, dim3(nbk * (nbk + 1) / 2), dim3(256), 0, st, W, k0, A);
      CHECK(hipGetLastError());
    }
  }
  CHECK(hipFuncSetAttribute((const void*)k_chol_solve, hipFuncAttributeMaxDynamicSharedMemorySize, W * 8));
  hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(256), (size_t)W * 8, st, W, (const double*)A, rhs);
  return hipGetLastError();
}

// rhs[w] = (e[w] - mean e) - eta (Odp[w] - mu.dp) + extra[w]
__global__ __launch_bounds__(256) void k_spring_rhs(int W, const double* __restrict__ e, const double* __restrict__ odp,
                                                    double eta, const double* __restrict__ extra,
                                                    double* __restrict__ rhs) {
  __shared__ double red[4];
  double s = 0.0;
  for (int w = threadIdx.x; w < W; w += blockDim.x) s += e[w];
  const double mean = block_sum_d(s, red) / W;
  for (int w = threadIdx.x; w < W; w += blockDim.x) {
    double v = e[w] - mean;
    if (odp) v -= eta * (odp[w] - odp[W]);
    if (extra) v += extra[w];
    rhs[w] = v;
  }
}

// (Obar v)[w] = O[w].v - mu.v  from the row dots (out[W] = mu . v)
__global__ void k_center_dots(int W, double* __restrict__ d) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < W) d[w] -= d[W];
}

// sum of a vector into out[0] (one workgroup)
__global__ __launch_bounds__(256) void k_vsum(int W, const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int w = threadIdx.x; w < W; w += blockDim.x) s += x[w];
  s = block_sum_d(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

// delta[p] = sum_w O[w][p] y[w] - mu[p] sum(y) + eta dprev[p] + dtilde[p]
__global__ void k_spring_combine(int64_t P, int W, const double* __restrict__ O, const double* __restrict__ y,
                                 const double* __restrict__ sumy, const double* __restrict__ mu, double eta,
                                 const double* __restrict__ dprev, const double* __restrict__ dtilde,
                                 double* __restrict__ delta) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int w = 0; w < W; ++w) s += O[(int64_t)w * P + p] * y[w];
  s -= mu[p] * sumy[0];
  if (dprev) s += eta * dprev[p];
  if (dtilde) s += dtilde[p];
  delta[p] = s;
}

// c = a - b (b may be null: a copy)
__global__ void k_vsub(int W, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < W) c[w] = a[w] - (b ? b[w] : 0.0);
}

__global__ void k_zero_flag(int32_t* f) { *f = 0; }

struct SpringLayout {
  size_t G, A, A2, r, mu, odp, otd, rhs, et, y, sumy, total;
};
static SpringLayout spring_layout(int64_t P, int W) {
  SpringLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  const size_t WW = (size_t)W * W * 8;
  L.G = take(WW);
  L.A = take(WW);
  L.A2 = take(WW);
  L.r = take((size_t)(W + 1) * 8);
  L.mu = take((size_t)P * 8);
  L.odp = take((size_t)(W + 1) * 8);
  L.otd = take((size_t)(W + 1) * 8);
  L.rhs = take((size_t)W * 8);
  L.et = take((size_t)W * 8);
  L.y = take((size_t)W * 8);
  L.sumy = take(8);
  L.total = o;
  return L;
}

size_t spring_ws_bytes(int64_t P, int W) { return W <= SPRING_WMAX ? spring_layout(P, W).total : 0; }

// info (device int32): 0, or 1 when a damped Gram matrix was not positive
// definite (a non-positive pivot; the solve then used a unit pivot there)
hipError_t spring_step(int64_t P, int W, const double* O, const double* e_loc, double lambda, double eta,
                       const double* dprev, const double* dtilde, double lambda0, double* delta, char* ws,
                       int32_t* info, hipStream_t st) {
  const SpringLayout L = spring_layout(P, W);
  double* G = (double*)(ws + L.G);
  double* A = (double*)(ws + L.A);
  double* A2 = (double*)(ws + L.A2);
  double* r = (double*)(ws + L.r);
  double* mu = (double*)(ws + L.mu);
  double* odp = (double*)(ws + L.odp);
  double* otd = (double*)(ws + L.otd);
  double* rhs = (double*)(ws + L.rhs);
  double* et = (double*)(ws + L.et);
  double* y = (double*)(ws + L.y);
  double* sumy = (double*)(ws + L.sumy);
  int* fail = info;
  hipLaunchKernelGGL(k_col_mean, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, W, O, mu);
  CHECK(hipGetLastError());
  // G = O O^T (FP64 MFMA, contraction over the parameters)
  {
    GemmArgs g{};
    g.A = O; g.amap = rows_dense(P); g.Bt = O; g.ldb = P; g.C = G; g.cmap = rows_dense(W); g.ccol = cols_dense();
    g.M = W; g.N = W; g.K = (int)(P < 0x7fffffff ? P : 0x7fffffff);
    if ((int64_t)g.K != P) return hipErrorInvalidValue;
    CHECK(gemm(MMA_F64, g, st));
  }
  hipLaunchKernelGGL(k_gram_rowmean, dim3(W), dim3(256), 0, st, W, (const double*)G, r);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_mean_tail, dim3(1), dim3(256), 0, st, W, r);
  CHECK(hipGetLastError());
  const int64_t WW = (int64_t)W * W;
  hipLaunchKernelGGL(k_gram_center, dim3((unsigned)((WW + 255) / 256)), dim3(256), 0, st, W, (const double*)G,
                     (const double*)r, lambda, A);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, st, fail);
  CHECK(hipGetLastError());
  if (dprev) {
    hipLaunchKernelGGL(k_row_dots, dim3(W + 1), dim3(256), 0, st, P, W, O, (const double*)mu, dprev, odp);
    CHECK(hipGetLastError());
  }
  const double* extra = nullptr;
  if (dtilde) {
    // eps~ = (Obar Obar^T + lambda0 I)^-1 Obar dtilde
    hipLaunchKernelGGL(k_gram_center, dim3((unsigned)((WW + 255) / 256)), dim3(256), 0, st, W, (const double*)G,
                       (const double*)r, lambda0, A2);
    CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_row_dots, dim3(W + 1), dim3(256), 0, st, P, W, O, (const double*)mu, dtilde, otd);
    CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_center_dots, dim3((W + 255) / 256), dim3(256), 0, st, W, otd);
    CHECK(hipGetLastError());
    CHECK(cholesky_solve(W, A2, otd, fail, st));
    hipLaunchKernelGGL(k_vsub, dim3((W + 255) / 256), dim3(256), 0, st, W, (const double*)otd, (const double*)nullptr,
                       et);
    CHECK(hipGetLastError());
    extra = et;
  }
  hipLaunchKernelGGL(k_spring_rhs, dim3(1), dim3(256), 0, st, W, e_loc, dprev ? (const double*)odp : nullptr, eta,
                     extra, rhs);
  CHECK(hipGetLastError());
  CHECK(cholesky_solve(W, A, rhs, fail, st));
  // y = x - eps~ (the in-span part of delta~ leaves through Obar^T eps~)
  hipLaunchKernelGGL(k_vsub, dim3((W + 255) / 256), dim3(256), 0, st, W, (const double*)rhs, extra, y);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_vsum, dim3(1), dim3(256), 0, st, W, (const double*)y, sumy);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_spring_combine, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, W, O,
                     (const double*)y, (const double*)sumy, (const double*)mu, eta, dprev, dtilde, delta);
  return hipGetLastError();
}

}  // namespace fire
