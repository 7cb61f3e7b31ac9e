// Kernels shared by the full evaluation and the single-electron update path.
#pragma once
#include "forward.hpp"

namespace fire {

// ---------------------------------------------------------------------------
// a1: neighbour lists.  One workgroup per walker; electron i lists every
// j != i with |r_i - r_j| <= c, same-spin first, then opposite spin.
// ---------------------------------------------------------------------------
static __global__ __launch_bounds__(256) void k_nbr(const double* __restrict__ R, int W, int n, int nu,
                                             double cut2, int cap, int16_t* __restrict__ idx,
                                             int32_t* __restrict__ cnt, int32_t* status) {
  __shared__ double pos[256 * 3];
  int w = blockIdx.x;
  const double* Rw = R + (int64_t)w * n * 3;
  for (int t = threadIdx.x; t < 3 * n; t += blockDim.x) pos[t] = Rw[t];
  __syncthreads();
  int i = threadIdx.x;
  if (i >= n) return;
  double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  if (!isfinite(xi) || !isfinite(yi) || !isfinite(zi)) atomicOr(status + w, FIRE_W_NONFINITE);
  int16_t* out = idx + ((int64_t)w * n + i) * cap;
  int si = i < nu ? 0 : 1;
  int c[2] = {0, 0};
  int k = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      int sj = j < nu ? 0 : 1;
      if ((sj == si) != (pass == 0)) continue;
      double dx = xi - pos[3 * j], dy = yi - pos[3 * j + 1], dz = zi - pos[3 * j + 2];
      if (dx * dx + dy * dy + dz * dz <= cut2) {
        if (k < cap) out[k] = (int16_t)j;
        ++k;
        ++c[pass];
      }
    }
  }
  if (k > cap) {
    atomicOr(status + w, FIRE_W_NBR_OVERFLOW);
    c[0] = c[0] < cap ? c[0] : cap;
    c[1] = cap - c[0] < c[1] ? cap - c[0] : c[1];
  }
  cnt[((int64_t)w * n + i) * 2 + 0] = c[0];
  cnt[((int64_t)w * n + i) * 2 + 1] = c[1];
}

// ---------------------------------------------------------------------------
// Pair features shared by the electron-nucleus and electron-electron filters:
//   out[0..3]  rescaled features log(1+r)/r * [r, dx, dy, dz]
//   out[4..4+h2) second hidden layer SiLU(SiLU(e W1 + b1) W2 + b2)
//   out[12..44) radial part f_cut(r/c) exp(-sigma_k^2 r^2)
//   out[44]    f_cut(r/c) (zero: the pair does not contribute)
// ---------------------------------------------------------------------------
template <typename T>
FIRE_DEV void pair_features(T dx, T dy, T dz, const T* W1, const T* b1, const T* W2, const T* b2,
                            const T* sig, T cut, const Dims& D, T* out) {
  // loops run to the compile-time maxima with guards, so that every weight
  // load of a layer is issued before the first product needs it
  T r = sqrt(dx * dx + dy * dy + dz * dz);
  T e4[4] = {r, dx, dy, dz};
  T lo = log1p_over(r);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = lo * e4[k];
  T w1[4][kMaxH1], bb1[kMaxH1];
#pragma unroll
  for (int k = 0; k < kMaxH1; ++k) {
    bb1[k] = k < D.h1 ? b1[k] : T(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) w1[j][k] = k < D.h1 ? W1[j * D.h1 + k] : T(0);
  }
  T z1[kMaxH1];
#pragma unroll
  for (int k = 0; k < kMaxH1; ++k) {
    T a = bb1[k];
#pragma unroll
    for (int j = 0; j < 4; ++j) a += e4[j] * w1[j][k];
    z1[k] = k < D.h1 ? silu_(a) : T(0);
  }
#pragma unroll
  for (int k = 0; k < kMaxH2; ++k) {
    if (k < D.h2) {
      T w2[kMaxH1];
#pragma unroll
      for (int j = 0; j < kMaxH1; ++j) w2[j] = j < D.h1 ? W2[j * D.h2 + k] : T(0);
      T a = b2[k];
#pragma unroll
      for (int j = 0; j < kMaxH1; ++j) a += z1[j] * w2[j];
      out[4 + k] = silu_(a);
    }
  }
  T fc = fcut_(r / cut);
  T sg[kMaxG];
#pragma unroll
  for (int k = 0; k < kMaxG; ++k) sg[k] = k < D.G ? sig[k] : T(0);
#pragma unroll
  for (int k = 0; k < kMaxG; ++k)
    if (k < D.G) out[12 + k] = fc * exp(-(sg[k] * sg[k]) * r * r);
  out[44] = fc;
}
constexpr int FEAT = 48;

// ---------------------------------------------------------------------------
// a2 + a3 (first half): s_i = sum_m Gamma_m(e_im) * (nuc_emb_m + ebar_im W_n),
// then y_i = LayerNorm(s_i).  Workgroup: one thread per channel, EPB electrons.
// ---------------------------------------------------------------------------
constexpr int EPB = 8;
constexpr int MCH = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_en_embed(Net<T> P, const double* __restrict__ R, int64_t nrows,
                                                  T* __restrict__ y_out, int epb) {
  const Dims& D = P.D;
  __shared__ T feat[MCH * FEAT];
  __shared__ int ntp[MCH];
  __shared__ T red[16];
  const int c = threadIdx.x;
  const bool act = c < D.d;
  T w3[kMaxH2], wenv[kMaxG], wn[4];
  if (act) {
    for (int k = 0; k < D.h2; ++k) w3[k] = P.en_W3[k * D.d + c];
    for (int k = 0; k < D.G; ++k) wenv[k] = P.en_Wenv[k * D.d + c];
    for (int k = 0; k < 4; ++k) wn[k] = P.en_Wn[k * D.d + c];
  }
  for (int el = 0; el < epb; ++el) {
    int64_t e = (int64_t)blockIdx.x * epb + el;
    if (e >= nrows) break;
    const double rx = R[3 * e], ry = R[3 * e + 1], rz = R[3 * e + 2];
    T s = 0;
    for (int m0 = 0; m0 < D.M; m0 += MCH) {
      int mc = D.M - m0 < MCH ? D.M - m0 : MCH;
      __syncthreads();
      if (threadIdx.x < mc) {
        int m = m0 + threadIdx.x, t = P.ntype[m];
        ntp[threadIdx.x] = t;
        pair_features<T>((T)(rx - P.Rn[3 * m]), (T)(ry - P.Rn[3 * m + 1]), (T)(rz - P.Rn[3 * m + 2]),
                         P.en_W1 + t * 4 * D.h1, P.en_b1 + t * D.h1, P.en_W2, P.en_b2, P.en_sig,
                         (T)D.cutn, D, feat + threadIdx.x * FEAT);
      }
      __syncthreads();
      if (act) {
        // nuclear embeddings of 16 nuclei are loaded together
        constexpr int NG = 16;
        for (int k0 = 0; k0 < mc; k0 += NG) {
          T ne[NG];
#pragma unroll
          for (int u = 0; u < NG; ++u) ne[u] = k0 + u < mc ? P.nuc_emb[ntp[k0 + u] * D.d + c] : T(0);
#pragma unroll
          for (int u = 0; u < NG; ++u) {
            const int k = k0 + u;
            if (k >= mc) break;
            const T* f = feat + k * FEAT;
            if (f[44] == T(0)) continue;
            T g1 = 0, g2 = 0;
#pragma unroll
            for (int j = 0; j < kMaxH2; ++j)
              if (j < D.h2) g1 += f[4 + j] * w3[j];
#pragma unroll
            for (int j = 0; j < kMaxG; ++j)
              if (j < D.G) g2 += f[12 + j] * wenv[j];
            T v = ne[u] + f[0] * wn[0] + f[1] * wn[1] + f[2] * wn[2] + f[3] * wn[3];
            s += g1 * g2 * v;
          }
        }
      }
    }
    T mu = block_sum<T>(act ? s : T(0), red) / T(D.d);
    T dv = act ? s - mu : T(0);
    T var = block_sum<T>(dv * dv, red) / T(D.d);
    if (act) y_out[e * D.d + c] = dv / sqrt(var + T(kLnEps)) * P.ln_g[c] + P.ln_b[c];
  }
}

// GLU gate: t = u * SiLU(g) with [u | g] the two halves of each row of ug.
template <typename T>
__global__ void k_glu(const T* __restrict__ ug, T* __restrict__ out, int64_t nrows, int d) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nrows * d) return;
  int64_t r = i / d;
  int c = (int)(i % d);
  T u = ug[r * 2 * d + c], g = ug[r * 2 * d + d + c];
  out[i] = u * silu_(g);
}

// Envelope basis exp(-sigma_me |r_i - R_m|), row e = (w, i), column m*E + k.
template <typename T>
__global__ void k_env_basis(Net<T> P, const double* __restrict__ R, int64_t nrows, T* __restrict__ out) {
  const Dims& D = P.D;
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nrows * D.B) return;
  int64_t e = q / D.B;
  int b = (int)(q % D.B), m = b / D.E;
  double dx = R[3 * e] - P.Rn[3 * m], dy = R[3 * e + 1] - P.Rn[3 * m + 1], dz = R[3 * e + 2] - P.Rn[3 * m + 2];
  T dist = (T)sqrt(dx * dx + dy * dy + dz * dz);
  out[q] = exp(-P.env_sigma[b] * dist);
}


}  // namespace fire
