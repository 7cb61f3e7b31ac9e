// Parameter gradient g = sum_w c_w d log|psi_w| / d theta by a hand-written
// adjoint (Methods, variational Monte Carlo: energy gradient with
// c_w = (E_L,w - mean E_L) / W).
//
// Per chunk of walkers the node-level forward activations are recomputed and
// kept (they fit in HBM); edge-level quantities (filters and messages of every
// electron pair and electron-nucleus pair) are recomputed inside the backward
// kernels and never stored.  The chain:
//   Phibar = c_w w_d Phi^-T              (d log|psi| / d Phi_d, w_d = s_d e^{l_d} / psi)
//   obar = Phibar * env,  envbar = Phibar * o          (orbital projections, envelopes)
//   MLP, messages (edge recompute), node projections, GLU, LayerNorm and
//   electron-nucleus filters (edge recompute) in reverse;
// weight gradients are split-K GEMMs over the (walker, electron) rows.
#include <vector>

#include "embed_kernels.hpp"
#include "jastrow.hpp"

namespace fire {

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

constexpr int GNS = 32;      // K-splits of the weight-gradient GEMMs
constexpr int CNS = 1024;    // row splits of the bias-gradient column sums
constexpr int GBLK = 1024;   // persistent workgroups of the edge kernels
constexpr int ECH = 32;      // pairs per LDS chunk in the edge kernels
constexpr int EFEAT = 96;    // per-pair stored values (see edge_forward)

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// out[c][r] = in[r][c] for r < R, c < C (in rows through a row map)
template <typename T>
__global__ void k_transpose(const T* __restrict__ in, RowMap m, int R, int C, T* __restrict__ out) {
  __shared__ T tile[32][33];
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: ty 0..7
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < R && c < C) {
      const uint32_t rr = (uint32_t)r, p = (uint32_t)m.rpg, q = rr / p;
      tile[k][tx] = in[(int64_t)q * m.gstride + (int64_t)(rr - q * p) * m.rstride + c];
    }
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < R && c < C) out[(int64_t)c * R + r] = tile[tx][k];
  }
}

// grad[base + a*sa + (b/cpg)*sbg + (b%cpg)*sb] += sum_z part[z][a][b]
template <typename T>
__global__ void k_reduce_splits(const T* __restrict__ part, int ns, int M, int N, double* __restrict__ grad,
                                int64_t base, int64_t sa, int64_t cpg, int64_t sbg, int64_t sb) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)M * N) return;
  const int a = (int)(q / N), b = (int)(q % N);
  double v = 0.0;
  for (int z = 0; z < ns; ++z) v += (double)part[(int64_t)z * M * N + q];
  grad[base + a * sa + (b / cpg) * sbg + (b % cpg) * sb] += v;
}

// part[z][c] = sum over rows r in chunk z of X[r][c]
template <typename T>
__global__ void k_colsum(const T* __restrict__ X, RowMap m, int R, int C, int ns, T* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (c >= C) return;
  const int per = (R + ns - 1) / ns;
  const int r0 = z * per, r1 = r0 + per < R ? r0 + per : R;
  T v = 0;
  if (r0 < r1) {
    // row r sits at (r / rpg) gstride + (r % rpg) rstride: quotient and
    // remainder are stepped along the chunk
    const uint32_t p = (uint32_t)m.rpg;
    uint32_t q = (uint32_t)r0 / p, rem = (uint32_t)r0 - q * p;
    const T* xc = X + c;
    for (int r = r0; r < r1; ++r) {
      v += xc[(int64_t)q * m.gstride + (int64_t)rem * m.rstride];
      if (++rem == p) { rem = 0; ++q; }
    }
  }
  part[(int64_t)z * C + c] = v;
}

// grad[base + j] += sum_b part[b][col0 + j], j < len: one workgroup of 256
// threads per column j, the partials strided over its threads, then summed
// in a fixed order (the same on every call)
__global__ __launch_bounds__(256) void k_reduce_cols(const void* __restrict__ part, int tsize, int nb, int64_t stride,
                                                     int64_t col0, int len, double* __restrict__ grad, int64_t base) {
  __shared__ double red[256];
  const int j = blockIdx.x, t = threadIdx.x;
  if (j >= len) return;
  double v = 0.0;
  for (int b = t; b < nb; b += 256) {
    const int64_t q = (int64_t)b * stride + col0 + j;
    v += tsize == 8 ? ((const double*)part)[q] : (double)((const float*)part)[q];
  }
  red[t] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) grad[base + j] += red[0];
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// h1 = h0 + m for the chunk rows, from the cached state
template <typename T>
__global__ void k_h1_from_state(const Dims D, int Wc, int w0, const char* __restrict__ state, StateRec S,
                                T* __restrict__ h1) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)Wc * D.n * D.d) return;
  const int64_t e = q / D.d;
  const int c = (int)(q % D.d);
  const int64_t w = w0 + e / D.n;
  const int i = (int)(e % D.n);
  const char* rec = state + w * S.stride;
  h1[q] = ((const T*)(rec + S.h0))[(int64_t)i * D.d + c] + ((const T*)(rec + S.m))[(int64_t)i * D.d + c];
}

template <typename T>
__global__ void k_silu_inplace(const T* __restrict__ z, T* __restrict__ h, int64_t n) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) h[q] = silu_(z[q]);
}

// zbar = hbar * SiLU'(z)
template <typename T>
__global__ void k_silu_bar(const T* __restrict__ z, const T* __restrict__ hbar, T* __restrict__ zbar, int64_t n) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  T f, f1, f2;
  silu3(z[q], f, f1, f2);
  zbar[q] = hbar[q] * f1;
}

// Phibar = c_w w_d G;  obar = Phibar * env;  envbar = Phibar * o  (envbar overwrites o)
template <typename T, typename TI>
__global__ void k_orb_bar(const Dims D, int s, int Wc, int w0, const char* __restrict__ state, StateRec S,
                          const double* __restrict__ coeff, T* __restrict__ o, T* __restrict__ obar) {
  const int N = D.nsig(s), KN = D.K * N;
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)Wc * N * KN) return;
  const int64_t r = q / KN;
  const int col = (int)(q % KN);
  const int64_t w = w0 + r / N;
  const int iloc = (int)(r % N);
  const int det = col / N, l = col % N;
  const char* rec = state + w * S.stride;
  const double* ds = (const double*)(rec + S.dsign);
  const double* dl = (const double*)(rec + S.dlog);
  const double lp = *(const double*)(rec + S.lpsi), sp = *(const double*)(rec + S.spsi);
  const double wd = ds[2 * det] * ds[2 * det + 1] * sp * exp(dl[2 * det] + dl[2 * det + 1] - lp);
  const int64_t idx = det * phi_per_det(D) + phi_block_off(D, s) + (int64_t)iloc * N + l;
  const double g = (double)((const TI*)(rec + S.inv))[idx];
  const T pb = (T)(coeff[w] * wd * g);
  const T env = ((const T*)(rec + S.env))[idx];
  obar[q] = pb * env;
  o[q] = pb * o[q];
}

// Jastrow readout k (0: log part, 1: node part) of row r of walker
// w = w0 + r / per: its adjoint g = c_w (k = 0) or c_w / node_w (k = 1, the
// node factor's value, FP64 at byte node_off of the record); then
// a2bar = g w3 SiLU'(a2), the readout-weight terms g z2 and g itself (bias)
template <typename T>
__global__ void k_jm_readout_bar(int64_t rows, int per, int w0, int Hj, int k, const char* __restrict__ state,
                                 size_t stride, size_t node_off, const double* __restrict__ coeff,
                                 const T* __restrict__ w3, const T* __restrict__ a2, const T* z2,
                                 T* __restrict__ a2bar, T* gz2, T* __restrict__ gcol) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= rows * Hj) return;
  const int64_t r = q / Hj;
  const int c = (int)(q % Hj);
  const int64_t w = w0 + r / per;
  double g = coeff[w];
  if (k == 1) {
    const double s2 = *(const double*)(state + w * stride + node_off);
    g = s2 != 0.0 && isfinite(s2) ? g / s2 : 0.0;
  }
  T f, f1, f2;
  silu3(a2[q], f, f1, f2);
  a2bar[q] = (T)(g * (double)w3[c] * (double)f1);
  gz2[q] = (T)(g * (double)z2[q]);
  if (c == 0) gcol[r] = (T)g;
}

// attention Jastrow: register embeddings V = N / Z of walkers w0 + [0, Wc)
template <typename T>
__global__ void k_ja_vrows(const Dims D, int Wc, int w0, const char* __restrict__ state, StateRec S,
                           T* __restrict__ V) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int NV = D.NV();
  if (q >= (int64_t)Wc * NV) return;
  const int64_t wl = q / NV;
  const int c = (int)(q % NV);
  const double* jt = (const double*)(state + (w0 + wl) * S.stride + S.jat);
  V[q] = (T)(jt[2 * D.Ra + c] / jt[D.Ra + c / D.dr]);
}

// attention Jastrow adjoint per row (w, i): with p_ri = e^{l_ri - m_r} / Z_r,
//   ubar_ric = Vbar_rc p_ri,  lbar_ri = p_ri sum_c Vbar_rc (u_ric - V_rc)
template <typename T>
__global__ __launch_bounds__(256) void k_ja_bar(const Dims D, int w0, const char* __restrict__ state, StateRec S,
                                                const T* __restrict__ Vbar, T* __restrict__ abar) {
  const int64_t row = blockIdx.x;
  const int n = D.n, NA = D.NA(), NV = D.NV(), Ra = D.Ra, dr = D.dr;
  const int64_t wl = row / n;
  const int i = (int)(row % n);
  const char* rec = state + (w0 + wl) * S.stride;
  const T* a = (const T*)(rec + S.jae) + (int64_t)i * NA;
  const double* jt = (const double*)(rec + S.jat);
  const T* vb = Vbar + wl * NV;
  for (int c = threadIdx.x; c < NA; c += blockDim.x) {
    const int r = c < Ra ? c : (c - Ra) / dr;
    const double Z = jt[Ra + r];
    const double p = exp((double)a[r] - jt[r]) / Z;
    double v;
    if (c < Ra) {
      double acc = 0.0;
      for (int e = 0; e < dr; ++e) {
        const int cc = r * dr + e;
        acc += (double)vb[cc] * ((double)a[Ra + cc] - jt[2 * Ra + cc] / Z);
      }
      v = p * acc;
    } else {
      v = (double)vb[c - Ra] * p;
    }
    abar[row * NA + c] = (T)v;
  }
}

// ubar = tbar * SiLU(g), gbar = tbar * u * SiLU'(g)
template <typename T>
__global__ void k_glu_bar(const T* __restrict__ ug, const T* __restrict__ tbar, T* __restrict__ ugbar, int64_t nrows,
                          int d) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nrows * d) return;
  const int64_t r = q / d;
  const int c = (int)(q % d);
  const T u = ug[r * 2 * d + c], g = ug[r * 2 * d + d + c];
  T f, f1, f2;
  silu3(g, f, f1, f2);
  const T tb = tbar[q];
  ugbar[r * 2 * d + c] = tb * f;
  ugbar[r * 2 * d + d + c] = tb * u * f1;
}

// envelope exponents: sigmabar[b] partial over rows = sum_r basisbar * (-rho) * basis
template <typename T>
__global__ void k_envsig_bar(Net<T> P, const double* __restrict__ R, int e0, int N, int Wc, const T* __restrict__ bb,
                             int ns, T* __restrict__ part) {
  const Dims& D = P.D;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (b >= D.B) return;
  const int m = b / D.E;
  const int rows = Wc * N, per = (rows + ns - 1) / ns;
  const int r0 = z * per, r1 = r0 + per < rows ? r0 + per : rows;
  T v = 0;
  for (int r = r0; r < r1; ++r) {
    const int64_t e = (int64_t)(r / N) * D.n + e0 + r % N;
    const double dx = R[3 * e] - P.Rn[3 * m], dy = R[3 * e + 1] - P.Rn[3 * m + 1], dz = R[3 * e + 2] - P.Rn[3 * m + 2];
    const T rho = (T)sqrt(dx * dx + dy * dy + dz * dz);
    v += bb[((int64_t)(r / N) * D.n + r % N) * D.B + b] * (-rho) * exp(-P.env_sigma[b] * rho);
  }
  part[(int64_t)z * D.B + b] = v;
}

// ---------------------------------------------------------------------------
// pair features with the intermediates the backward pass needs:
//   [0..4) e4 = [r, dx, dy, dz]      [4..8)  rescaled features
//   [8..24) z1 pre-activations       [24..40) z1
//   [40..48) z2 pre-activations      [48..56) z2
//   [56..88) exp(-sigma_k^2 r^2)     [88] f_cut(r/c)
// ---------------------------------------------------------------------------
template <typename T>
FIRE_DEV void edge_forward(T dx, T dy, T dz, const T* W1, const T* b1, const T* W2, const T* b2, const T* sig, T cut,
                           const Dims& D, T* f) {
  const T r = sqrt(dx * dx + dy * dy + dz * dz);
  f[0] = r; f[1] = dx; f[2] = dy; f[3] = dz;
  const T lo = log1p_over(r);
  for (int k = 0; k < 4; ++k) f[4 + k] = lo * f[k];
  for (int k = 0; k < D.h1; ++k) {
    T a = b1[k];
    for (int j = 0; j < 4; ++j) a += f[j] * W1[j * D.h1 + k];
    f[8 + k] = a;
    f[24 + k] = silu_(a);
  }
  for (int k = 0; k < D.h2; ++k) {
    T a = b2[k];
    for (int j = 0; j < D.h1; ++j) a += f[24 + j] * W2[j * D.h2 + k];
    f[40 + k] = a;
    f[48 + k] = silu_(a);
  }
  for (int k = 0; k < D.G; ++k) f[56 + k] = exp(-(sig[k] * sig[k]) * r * r);
  f[88] = fcut_(r / cut);
}

// Backward of the filters of a chunk of pairs in two steps, so that no two
// threads ever add into the same accumulator entry:
//  edge_backward_terms (one thread per pair, f = its edge_forward values,
//    zb2 = zbar2 (h2), chib = chibar (G)) writes the per-pair terms
//    t = [pre2bar (h2) | pre1bar (h1) | d/dsigma terms (G)], zeros for a
//    pair outside the cutoff;
//  edge_param_sums (all threads, one accumulator entry each) adds their sums
//    over the chunk into W2, b2, sigma and W1, b1 (shared, or per pair slot
//    when each slot has its own first layer).
constexpr int ET = kMaxH2 + kMaxH1 + kMaxG;   // per-pair terms
template <typename T>
FIRE_DEV void edge_backward_terms(const T* f, const T* zb2, const T* chib, const T* W2, const T* sig, T* t) {
  constexpr int h1 = kMaxH1, h2 = kMaxH2, G = kMaxG;
  const T r = f[0], fc = f[88];
  if (fc == T(0)) {
    for (int k = 0; k < ET; ++k) t[k] = T(0);
    return;
  }
  for (int k = 0; k < G; ++k) t[h2 + h1 + k] = chib[k] * fc * f[56 + k] * (T(-2) * sig[k] * r * r);
  T pre2b[h2];
  for (int k = 0; k < h2; ++k) {
    T sv, s1, s2;
    silu3(f[40 + k], sv, s1, s2);
    pre2b[k] = zb2[k] * s1;
    t[k] = pre2b[k];
  }
  for (int j = 0; j < h1; ++j) {
    T z1b = 0;
    for (int k = 0; k < h2; ++k) z1b += pre2b[k] * W2[j * h2 + k];
    T sv, s1, s2;
    silu3(f[8 + j], sv, s1, s2);
    t[h2 + j] = z1b * s1;
  }
}

template <typename T, bool W1SLOT>
FIRE_DEV void edge_param_sums(const T* feat, const T* et, int np, T* accW1, T* accb1, T* accW2, T* accb2,
                              T* accsig) {
  constexpr int h1 = kMaxH1, h2 = kMaxH2, G = kMaxG;
  constexpr int NW2 = h1 * h2, NSH = NW2 + h2 + G + (W1SLOT ? 0 : 5 * h1);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int q = tid; q < NSH; q += nt) {
    T sum = 0;
    if (q < NW2) {
      const int j = q / h2, kk = q % h2;
      for (int k = 0; k < np; ++k) sum += et[k * ET + kk] * feat[k * EFEAT + 24 + j];
      accW2[q] += sum;
    } else if (q < NW2 + h2) {
      const int kk = q - NW2;
      for (int k = 0; k < np; ++k) sum += et[k * ET + kk];
      accb2[kk] += sum;
    } else if (q < NW2 + h2 + G) {
      const int g = q - NW2 - h2;
      for (int k = 0; k < np; ++k) sum += et[k * ET + h2 + h1 + g];
      accsig[g] += sum;
    } else {
      const int q3 = q - NW2 - h2 - G;
      if (q3 < 4 * h1) {
        const int i = q3 / h1, j = q3 % h1;
        for (int k = 0; k < np; ++k) sum += et[k * ET + h2 + j] * feat[k * EFEAT + i];
        accW1[q3] += sum;
      } else {
        const int j = q3 - 4 * h1;
        for (int k = 0; k < np; ++k) sum += et[k * ET + h2 + j];
        accb1[j] += sum;
      }
    }
  }
  if constexpr (W1SLOT) {
    for (int q = tid; q < np * 5 * h1; q += nt) {
      const int k = q / (5 * h1), r5 = q % (5 * h1);
      if (r5 < 4 * h1) {
        const int i = r5 / h1, j = r5 % h1;
        accW1[k * 4 * h1 + r5] += et[k * ET + h2 + j] * feat[k * EFEAT + i];
      } else {
        const int j = r5 - 4 * h1;
        accb1[k * h1 + j] += et[k * ET + h2 + j];
      }
    }
  }
}

// partial layout of one filter (shared by both edge kernels)
struct FiltOff {
  int W1, b1, W2, b2, W3, Wenv, sig, size;
};
FIRE_HOST_DEVICE FiltOff filt_off(const Dims& D) {
  FiltOff o;
  o.W1 = 0; o.b1 = 4 * D.h1; o.W2 = o.b1 + D.h1; o.b2 = o.W2 + D.h1 * D.h2; o.W3 = o.b2 + D.h2;
  o.Wenv = o.W3 + D.h2 * D.d; o.sig = o.Wenv + D.G * D.d; o.size = o.sig + D.G;
  return o;
}
// message partials per block: per alpha [filter | We (4d) | b (d)]
FIRE_HOST_DEVICE int msg_part_size(const Dims& D) { return 2 * (filt_off(D).size + 5 * D.d); }

// ---------------------------------------------------------------------------
// message backward.  For edge (i, j) of class alpha and channel c:
//   Gamma = g1 g2, g1 = z2 . W3[:,c], g2 = chi . Wenv[:,c], pre = a_i + b_j + ebar . We + b
//   m_i += Gamma SiLU(pre)
// mbar gives Gammabar = mbar SiLU(pre), prebar = mbar Gamma SiLU'(pre);
// abar_i += prebar, bbar_j += prebar (atomic), and the weight partials.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Reductions over channels for one chunk of up to 16 pairs (FP32):
//   red[k][q]     = sum_c u1[k][c] W3[q][c]      (q < h2)
//   red[k][8 + q] = sum_c u2[k][c] Wenv[q][c]    (q < G)
// Each thread holds u1[k], u2[k] of its channel c; each wave multiplies its
// 64 channels out on f32 16x16x4 MFMA (the u values are transposed through
// LDS), the four wave partials are summed in LDS.  wb: this lane's B
// operands, wb[s][t] = W_(16 t + l16)[64 wave + 4 s + l/16] (t = 0: W3 rows,
// zero past h2; t = 1, 2: Wenv rows).
// ---------------------------------------------------------------------------
typedef float f4v_ __attribute__((ext_vector_type(4)));
constexpr int RCH = 16;   // pairs per channel reduction

// One pair's channel sums on the FP64 path: out[q] = sum_c u1_c W3[q][c]
// (q < h2) and out[8 + q] = sum_c u2_c Wenv[q][c] (q < G).  Each wave's sums
// go to its row of w4 ([waves][40]); then one thread per output adds the
// waves in order, so the sums do not depend on scheduling.  Every thread of
// the block calls it.
template <typename T>
FIRE_DEV void pair_sums_waves(T u1, T u2, const T* w3, const T* wenv, bool act, int h2, int G, T* w4, T* out) {
  const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int q = 0; q < h2; ++q) {
    const T v = wave_sum(act ? u1 * w3[q] : T(0));
    if ((tid & 63) == 0) w4[wave * 40 + q] = v;
  }
  for (int q = 0; q < G; ++q) {
    const T v = wave_sum(act ? u2 * wenv[q] : T(0));
    if ((tid & 63) == 0) w4[wave * 40 + 8 + q] = v;
  }
  __syncthreads();
  if (tid < 40 && (tid < h2 || (tid >= 8 && tid < 8 + G))) {
    T v = 0;
    for (int x = 0; x < nw; ++x) v += w4[x * 40 + tid];
    out[tid] = v;
  }
  __syncthreads();
}

// us: LDS [waves][2][RCH][64] floats, filled by the caller (chan_slot: this
// thread's slots for u1 and u2 of pair k, zero past kc); wp: LDS
// [waves][RCH][40] floats; red: LDS [RCH][40] (overwritten for k < kc).
// Called by the whole block.
FIRE_DEV float* chan_slot(float* us, int k, int which) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return us + wave * 2 * RCH * 64 + (which * RCH + k) * 64 + lane;
}
FIRE_DEV void chan_reduce(int kc, const float* W3, const float* Wenv, int d, float* us, float* wp, float* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  float* mine = us + wave * 2 * RCH * 64;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  f4v_ r1 = {0.f, 0.f, 0.f, 0.f}, r2 = {0.f, 0.f, 0.f, 0.f}, r3 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int st = 0; st < 16; ++st) {
    // A[row = pair l16][k = channel 4 st + lg], B[k = channel][col = output l16]
    const int c = 64 * wave + 4 * st + lg;
    const bool cin = c < d;
    const float a1 = mine[l16 * 64 + 4 * st + lg];
    const float a2 = mine[(RCH + l16) * 64 + 4 * st + lg];
    const float b1 = (cin && l16 < kMaxH2) ? W3[l16 * d + c] : 0.f;
    const float b2 = cin ? Wenv[l16 * d + c] : 0.f;
    const float b3 = cin ? Wenv[(16 + l16) * d + c] : 0.f;
    r1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, r1, 0, 0, 0);
    r2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b2, r2, 0, 0, 0);
    r3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b3, r3, 0, 0, 0);
  }
  // output register e of lane (l16, lg): row 4 lg + e, column l16
  float* pw = wp + wave * RCH * 40;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = 4 * lg + e;
    if (l16 < 8) pw[k * 40 + l16] = r1[e];
    pw[k * 40 + 8 + l16] = r2[e];
    pw[k * 40 + 24 + l16] = r3[e];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kc * 40; q += blockDim.x) {
    float v = 0.f;
    for (int w = 0; w < nw; ++w) v += wp[w * RCH * 40 + q];
    red[q] = v;
  }
  __syncthreads();
}

// The sender side of the message backward: for row j and pair class a,
// the gradient of its projection b_j (slot 2 + a) collects, over the
// receivers i with j in N(i), pb_ij = mbar_i gamma_ij silu'(a_i + b_j +
// f_ij We + b), with gamma_ij and f_ij the filter and edge features of
// r_i - r_j.  The neighbour relation is symmetric, so the receivers are the
// class-a entries of j's own list, summed in list order: the result does not
// depend on scheduling (the receiver side, k_msg_bwd, writes slot a only).
template <typename T>
__global__ __launch_bounds__(256) void k_projbar_gather(Net<T> P, const double* __restrict__ R, int64_t nrows, int w0,
                                                        const int16_t* __restrict__ nidx,
                                                        const int32_t* __restrict__ ncnt,
                                                        const char* __restrict__ state, StateRec S,
                                                        const T* __restrict__ mbar, T* __restrict__ projbar) {
  const Dims& D = P.D;
  __shared__ T feat[ECH * EFEAT];
  __shared__ int jn[ECH];
  const int c = threadIdx.x, tid = threadIdx.x;
  const bool act = c < D.d;
  const int n = D.n, d = D.d;
  const int a = blockIdx.y;
  T w3[kMaxH2], wenv[kMaxG], we[4], bb = 0;
  if (act) {
    for (int k = 0; k < D.h2; ++k) w3[k] = P.ee_W3[(a * D.h2 + k) * d + c];
    for (int k = 0; k < D.G; ++k) wenv[k] = P.ee_Wenv[(a * D.G + k) * d + c];
    for (int k = 0; k < 4; ++k) we[k] = P.msg_We[(a * 4 + k) * d + c];
    bb = P.msg_b[a * d + c];
  }
  for (int64_t e = blockIdx.x; e < nrows; e += gridDim.x) {
    const int64_t wl = e / n;
    const int jrow = (int)(e % n);
    const char* rec = state + (w0 + wl) * S.stride;
    const T* proj = (const T*)(rec + S.proj);
    const double* Rw = R + wl * n * 3;
    const double rx = Rw[3 * jrow], ry = Rw[3 * jrow + 1], rz = Rw[3 * jrow + 2];
    const T bj = act ? proj[((int64_t)jrow * 4 + 2 + a) * d + c] : T(0);
    const int c0 = ncnt[2 * e], c1 = ncnt[2 * e + 1];
    const int na = a == 0 ? c0 : c1, sbase = a == 0 ? 0 : c0;
    T sum = 0;
    for (int i0 = 0; i0 < na; i0 += ECH) {
      const int ic = na - i0 < ECH ? na - i0 : ECH;
      __syncthreads();
      if (tid < ic) {
        const int i = nidx[e * D.cap_nbr + sbase + i0 + tid];
        jn[tid] = i;
        edge_forward<T>((T)(Rw[3 * i] - rx), (T)(Rw[3 * i + 1] - ry), (T)(Rw[3 * i + 2] - rz),
                        P.ee_W1 + a * 4 * D.h1, P.ee_b1 + a * D.h1, P.ee_W2 + a * D.h1 * D.h2, P.ee_b2 + a * D.h2,
                        P.ee_sig + a * D.G, (T)D.cut, D, feat + tid * EFEAT);
      }
      __syncthreads();
      if (act) {
        for (int k = 0; k < ic; ++k) {
          const T* f = feat + k * EFEAT;
          if (f[88] == T(0)) continue;
          const int i = jn[k];
          T g1 = 0, g2 = 0;
          for (int q = 0; q < D.h2; ++q) g1 += f[48 + q] * w3[q];
          for (int q = 0; q < D.G; ++q) g2 += f[88] * f[56 + q] * wenv[q];
          const T ai = proj[((int64_t)i * 4 + a) * d + c];
          const T pre = ai + bj + f[4] * we[0] + f[5] * we[1] + f[6] * we[2] + f[7] * we[3] + bb;
          T sf, s1, s2;
          silu3(pre, sf, s1, s2);
          sum += mbar[(wl * n + i) * d + c] * (g1 * g2) * s1;
        }
      }
    }
    if (act) projbar[(e * 4 + 2 + a) * d + c] += sum;
  }
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_msg_bwd(Net<T> P, const double* __restrict__ R, int64_t nrows, int w0,
                                                 const int16_t* __restrict__ nidx, const int32_t* __restrict__ ncnt,
                                                 const char* __restrict__ state, StateRec S,
                                                 const T* __restrict__ mbar, T* __restrict__ projbar,
                                                 T* __restrict__ part) {
  const Dims& D = P.D;
  const FiltOff fo = filt_off(D);
  __shared__ T feat[ECH * EFEAT];
  __shared__ T red[ECH * 40];
  __shared__ T eterm[ECH * ET];
  __shared__ int jn[ECH];
  extern __shared__ char dyn[];
  // LDS accumulators of the scalar filter parameters, per alpha:
  // [W1 | b1 | W2 | b2] (offsets as in the partials) then sigma at fo.W3
  const int astr = fo.W3 + D.G;
  T* acc = (T*)dyn;
  const int c = threadIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const bool act = c < D.d;
  const int n = D.n, d = D.d;
  for (int q = tid; q < astr; q += nt) acc[q] = T(0);
  __shared__ float red_us[sizeof(T) == 4 ? 4 * 2 * RCH * 64 : 1];
  __shared__ float red_wp[sizeof(T) == 4 ? 4 * RCH * 40 : 1];
  __shared__ T red4[sizeof(T) == 8 ? 4 * 40 : 1];
  // one pair class per launch row of blocks: a = blockIdx.y (par, anti), which
  // halves the live accumulators and so doubles the resident waves
  const int a = blockIdx.y;
  T aW3[kMaxH2], aWenv[kMaxG], aWe[4], ab = 0;
  for (int k = 0; k < kMaxH2; ++k) aW3[k] = 0;
  for (int k = 0; k < kMaxG; ++k) aWenv[k] = 0;
  for (int k = 0; k < 4; ++k) aWe[k] = 0;
  __syncthreads();
  for (int64_t e = blockIdx.x; e < nrows; e += gridDim.x) {
    const int64_t wl = e / n;
    const int i = (int)(e % n);
    const char* rec = state + (w0 + wl) * S.stride;
    const T* proj = (const T*)(rec + S.proj);
    const double* Rw = R + wl * n * 3;
    const double rx = Rw[3 * i], ry = Rw[3 * i + 1], rz = Rw[3 * i + 2];
    const T mb = act ? mbar[e * d + c] : T(0);
    const int c0 = ncnt[2 * e], c1 = ncnt[2 * e + 1];
    T abar = 0;
    {
      const int na = a == 0 ? c0 : c1, sbase = a == 0 ? 0 : c0;
      T w3[kMaxH2], wenv[kMaxG], we[4], bb = 0, ai = 0;
      if (act) {
        for (int k = 0; k < D.h2; ++k) w3[k] = P.ee_W3[(a * D.h2 + k) * d + c];
        for (int k = 0; k < D.G; ++k) wenv[k] = P.ee_Wenv[(a * D.G + k) * d + c];
        for (int k = 0; k < 4; ++k) we[k] = P.msg_We[(a * 4 + k) * d + c];
        bb = P.msg_b[a * d + c];
        ai = proj[((int64_t)i * 4 + a) * d + c];
      }
      for (int j0 = 0; j0 < na; j0 += ECH) {
        const int jc = na - j0 < ECH ? na - j0 : ECH;
        __syncthreads();
        if (tid < jc) {
          const int j = nidx[e * D.cap_nbr + sbase + j0 + tid];
          jn[tid] = j;
          edge_forward<T>((T)(rx - Rw[3 * j]), (T)(ry - Rw[3 * j + 1]), (T)(rz - Rw[3 * j + 2]),
                          P.ee_W1 + a * 4 * D.h1, P.ee_b1 + a * D.h1, P.ee_W2 + a * D.h1 * D.h2, P.ee_b2 + a * D.h2,
                          P.ee_sig + a * D.G, (T)D.cut, D, feat + tid * EFEAT);
        }
        for (int q = tid; q < jc * 40; q += nt) red[q] = T(0);
        __syncthreads();
        // pj: the neighbour's projection b_j of this channel (read ahead)
        auto proj_j = [&](int k) { return ((const T*)(rec + S.proj))[((int64_t)jn[k] * 4 + 2 + a) * d + c]; };
        auto pair_grads = [&](int k, T pj, T& u1, T& u2) {
          const T* f = feat + k * EFEAT;
          u1 = 0;
          u2 = 0;
          if (act && f[88] != T(0)) {
            T g1 = 0, g2 = 0;
            for (int q = 0; q < D.h2; ++q) g1 += f[48 + q] * w3[q];
            for (int q = 0; q < D.G; ++q) g2 += f[88] * f[56 + q] * wenv[q];
            const T gam = g1 * g2;
            const int j = jn[k];
            const T pre = ai + pj + f[4] * we[0] + f[5] * we[1] + f[6] * we[2] + f[7] * we[3] + bb;
            T sf, s1, s2;
            silu3(pre, sf, s1, s2);
            const T gb = mb * sf, pb = mb * gam * s1;
            abar += pb;
            for (int q = 0; q < 4; ++q) aWe[q] += pb * f[4 + q];
            ab += pb;
            u1 = gb * g2;
            u2 = gb * g1;
            for (int q = 0; q < D.h2; ++q) aW3[q] += u1 * f[48 + q];
            for (int q = 0; q < D.G; ++q) aWenv[q] += u2 * f[88] * f[56 + q];
          }
        };
        // per-pair reductions over channels: zbar2_q = sum_c u1 W3[q][c], chibar_q = sum_c u2 Wenv[q][c]
        if constexpr (sizeof(T) == 4) {
          for (int k0 = 0; k0 < jc; k0 += RCH) {
            const int kc = jc - k0 < RCH ? jc - k0 : RCH;
            T pjv[RCH];
            for (int kk = 0; kk < RCH; ++kk) pjv[kk] = act ? proj_j(kk < kc ? k0 + kk : k0) : T(0);
            for (int kk = 0; kk < RCH; ++kk) {
              T u1 = 0, u2 = 0;
              if (kk < kc) pair_grads(k0 + kk, pjv[kk], u1, u2);
              *chan_slot(red_us, kk, 0) = (float)u1;
              *chan_slot(red_us, kk, 1) = (float)u2;
            }
            chan_reduce(kc, (const float*)(P.ee_W3 + a * D.h2 * d), (const float*)(P.ee_Wenv + a * D.G * d), d,
                        red_us, red_wp, (float*)red + k0 * 40);
          }
        } else {
          for (int k = 0; k < jc; ++k) {
            T u1, u2;
            pair_grads(k, act ? proj_j(k) : T(0), u1, u2);
            pair_sums_waves(u1, u2, w3, wenv, act, D.h2, D.G, red4, red + k * 40);
          }
        }
        __syncthreads();
        // chi = f_cut * exp(-sigma^2 r^2): only the exponents are parameters
        if (tid < jc)
          edge_backward_terms<T>(feat + tid * EFEAT, red + tid * 40, red + tid * 40 + 8, P.ee_W2 + a * D.h1 * D.h2,
                                 P.ee_sig + a * D.G, eterm + tid * ET);
        __syncthreads();
        {
          T* A = acc;
          edge_param_sums<T, false>(feat, eterm, jc, A + fo.W1, A + fo.b1, A + fo.W2, A + fo.b2, A + fo.W3);
        }
      }
    }
    if (act) projbar[(e * 4 + a) * d + c] += abar;
  }
  __syncthreads();
  T* out = part + (int64_t)blockIdx.x * msg_part_size(D);
  {
    T* o = out + a * (fo.size + 5 * D.d);
    if (act) {
      for (int q = 0; q < D.h2; ++q) o[fo.W3 + q * d + c] = aW3[q];
      for (int q = 0; q < D.G; ++q) o[fo.Wenv + q * d + c] = aWenv[q];
      for (int q = 0; q < 4; ++q) o[fo.size + q * d + c] = aWe[q];
      o[fo.size + 4 * d + c] = ab;
    }
    for (int q = tid; q < fo.W3; q += nt) o[q] = acc[q];
    for (int q = tid; q < D.G; q += nt) o[fo.sig + q] = acc[fo.W3 + q];
  }
}

// ---------------------------------------------------------------------------
// LayerNorm backward: sbar from ybar, and the LayerNorm parameter partials.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ln_bwd(Net<T> P, const double* __restrict__ R, int64_t nrows,
                                                const T* __restrict__ ybar, T* __restrict__ sbar,
                                                T* __restrict__ part) {
  const Dims& D = P.D;
  __shared__ T feat[MCH * FEAT];
  __shared__ T red[16];
  const int c = threadIdx.x;
  const bool act = c < D.d;
  T w3[kMaxH2], wenv[kMaxG], wn[4];
  if (act) {
    for (int k = 0; k < D.h2; ++k) w3[k] = P.en_W3[k * D.d + c];
    for (int k = 0; k < D.G; ++k) wenv[k] = P.en_Wenv[k * D.d + c];
    for (int k = 0; k < 4; ++k) wn[k] = P.en_Wn[k * D.d + c];
  }
  T ag = 0, abeta = 0;
  for (int64_t e = blockIdx.x; e < nrows; e += gridDim.x) {
    const double rx = R[3 * e], ry = R[3 * e + 1], rz = R[3 * e + 2];
    T s = 0;
    for (int m0 = 0; m0 < D.M; m0 += MCH) {
      const int mc = D.M - m0 < MCH ? D.M - m0 : MCH;
      __syncthreads();
      if (threadIdx.x < mc) {
        const int m = m0 + threadIdx.x, t = P.ntype[m];
        pair_features<T>((T)(rx - P.Rn[3 * m]), (T)(ry - P.Rn[3 * m + 1]), (T)(rz - P.Rn[3 * m + 2]),
                         P.en_W1 + t * 4 * D.h1, P.en_b1 + t * D.h1, P.en_W2, P.en_b2, P.en_sig, (T)D.cutn, D,
                         feat + threadIdx.x * FEAT);
      }
      __syncthreads();
      if (act)
        for (int k = 0; k < mc; ++k) {
          const T* f = feat + k * FEAT;
          if (f[44] == T(0)) continue;
          T g1 = 0, g2 = 0;
          for (int j = 0; j < D.h2; ++j) g1 += f[4 + j] * w3[j];
          for (int j = 0; j < D.G; ++j) g2 += f[12 + j] * wenv[j];
          const T v = P.nuc_emb[P.ntype[m0 + k] * D.d + c] + f[0] * wn[0] + f[1] * wn[1] + f[2] * wn[2] + f[3] * wn[3];
          s += g1 * g2 * v;
        }
    }
    const T inv_d = T(1) / T(D.d);
    const T mu = block_sum<T>(act ? s : T(0), red) * inv_d;
    const T dv = act ? s - mu : T(0);
    const T var = block_sum<T>(dv * dv, red) * inv_d;
    const T rs = T(1) / sqrt(var + T(kLnEps));
    const T xh = dv * rs;
    const T yb = act ? ybar[e * D.d + c] : T(0);
    ag += yb * xh;
    abeta += yb;
    const T xb = act ? yb * P.ln_g[c] : T(0);
    const T m1 = block_sum<T>(xb, red) * inv_d;
    const T m2 = block_sum<T>(xb * xh, red) * inv_d;
    if (act) sbar[e * D.d + c] = rs * (xb - m1 - xh * m2);
  }
  if (act) {
    part[(int64_t)blockIdx.x * 2 * D.d + c] = ag;
    part[(int64_t)blockIdx.x * 2 * D.d + D.d + c] = abeta;
  }
}

// electron-nucleus partials per block: [nuc_emb NT d | W1 NT 4h1 | b1 NT h1 | W2 | b2 | W3 | Wenv | sig | Wn 4d]
struct EnOff {
  int nuc, W1, b1, W2, b2, W3, Wenv, sig, Wn, size;
};
FIRE_HOST_DEVICE EnOff en_off(const Dims& D) {
  EnOff o;
  o.nuc = 0; o.W1 = D.NT * D.d; o.b1 = o.W1 + D.NT * 4 * D.h1; o.W2 = o.b1 + D.NT * D.h1; o.b2 = o.W2 + D.h1 * D.h2;
  o.W3 = o.b2 + D.h2; o.Wenv = o.W3 + D.h2 * D.d; o.sig = o.Wenv + D.G * D.d; o.Wn = o.sig + D.G;
  o.size = o.Wn + 4 * D.d;
  return o;
}
constexpr int ENCH = 32;   // nuclei per block column of the electron-nucleus backward

// ---------------------------------------------------------------------------
// electron-nucleus backward for nuclei [m0, m0 + ENCH) (blockIdx.y):
// s_i = sum_m Gamma_m * v_m, v_m = nuc_emb_m + ebar_im W_n.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_en_bwd(Net<T> P, const double* __restrict__ R, int64_t nrows,
                                                const T* __restrict__ sbar, T* __restrict__ part) {
  const Dims& D = P.D;
  const EnOff eo = en_off(D);
  const int m0 = blockIdx.y * ENCH;
  const int mc = D.M - m0 < ENCH ? D.M - m0 : ENCH;
  __shared__ T feat[ENCH * EFEAT];
  __shared__ T red[ENCH * 40];
  __shared__ T eterm[ENCH * ET];
  __shared__ int ntk[ENCH];
  extern __shared__ char dyn[];
  T* nucb = (T*)dyn;                       // [ENCH][d]
  T* sW1 = nucb + ENCH * D.d;              // [ENCH][4 h1]
  T* sb1 = sW1 + ENCH * 4 * D.h1;          // [ENCH][h1]
  T* sW2 = sb1 + ENCH * D.h1;              // [h1 h2]
  T* sb2 = sW2 + D.h1 * D.h2;              // [h2]
  T* ssig = sb2 + D.h2;                    // [G]
  const int nsc = ENCH * D.d + ENCH * 5 * D.h1 + D.h1 * D.h2 + D.h2 + D.G;
  const int c = threadIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const bool act = c < D.d;
  for (int q = tid; q < nsc; q += nt) nucb[q] = T(0);
  T w3[kMaxH2], wenv[kMaxG], wn[4];
  T aW3[kMaxH2], aWenv[kMaxG], aWn[4];
  for (int k = 0; k < kMaxH2; ++k) aW3[k] = 0;
  for (int k = 0; k < kMaxG; ++k) aWenv[k] = 0;
  for (int k = 0; k < 4; ++k) aWn[k] = 0;
  if (act) {
    for (int k = 0; k < D.h2; ++k) w3[k] = P.en_W3[k * D.d + c];
    for (int k = 0; k < D.G; ++k) wenv[k] = P.en_Wenv[k * D.d + c];
    for (int k = 0; k < 4; ++k) wn[k] = P.en_Wn[k * D.d + c];
  }
  // nucleus types of this block column, and the embeddings of the first
  // four types of this channel in registers
  if (tid < mc) ntk[tid] = P.ntype[m0 + tid];
  T nemb[4];
  for (int t = 0; t < 4; ++t) nemb[t] = (act && t < D.NT) ? P.nuc_emb[t * D.d + c] : T(0);
  // FP32: B operands and LDS of the MFMA channel reductions
  __shared__ float red_us[sizeof(T) == 4 ? 4 * 2 * RCH * 64 : 1];
  __shared__ float red_wp[sizeof(T) == 4 ? 4 * RCH * 40 : 1];
  __shared__ T red4[sizeof(T) == 8 ? 4 * 40 : 1];
  for (int64_t e = blockIdx.x; e < nrows; e += gridDim.x) {
    const double rx = R[3 * e], ry = R[3 * e + 1], rz = R[3 * e + 2];
    const T sb = act ? sbar[e * D.d + c] : T(0);
    __syncthreads();
    if (tid < mc) {
      const int m = m0 + tid, t = P.ntype[m];
      edge_forward<T>((T)(rx - P.Rn[3 * m]), (T)(ry - P.Rn[3 * m + 1]), (T)(rz - P.Rn[3 * m + 2]),
                      P.en_W1 + t * 4 * D.h1, P.en_b1 + t * D.h1, P.en_W2, P.en_b2, P.en_sig, (T)D.cutn, D,
                      feat + tid * EFEAT);
    }
    for (int q = tid; q < mc * 40; q += nt) red[q] = T(0);
    __syncthreads();
    // per pair: u1 = dL/dg1, u2 = dL/dg2 of this channel, and the weight
    // gradients that stay per channel
    auto pair_grads = [&](int k, T& u1, T& u2) {
      const T* f = feat + k * EFEAT;
      u1 = 0;
      u2 = 0;
      if (act && f[88] != T(0)) {
        T g1 = 0, g2 = 0;
        for (int q = 0; q < D.h2; ++q) g1 += f[48 + q] * w3[q];
        for (int q = 0; q < D.G; ++q) g2 += f[88] * f[56 + q] * wenv[q];
        const T gam = g1 * g2;
        const int tk = ntk[k];
        const T ne = tk == 0 ? nemb[0] : tk == 1 ? nemb[1] : tk == 2 ? nemb[2] : tk == 3 ? nemb[3]
                                                                               : P.nuc_emb[tk * D.d + c];
        const T v = ne + f[4] * wn[0] + f[5] * wn[1] + f[6] * wn[2] + f[7] * wn[3];
        const T gb = sb * v, vb = sb * gam;
        nucb[k * D.d + c] += vb;
        for (int q = 0; q < 4; ++q) aWn[q] += vb * f[4 + q];
        u1 = gb * g2;
        u2 = gb * g1;
        for (int q = 0; q < D.h2; ++q) aW3[q] += u1 * f[48 + q];
        for (int q = 0; q < D.G; ++q) aWenv[q] += u2 * f[88] * f[56 + q];
      }
    };
    if constexpr (sizeof(T) == 4) {
      // reductions over channels of 16 pairs at a time on MFMA
      for (int k0 = 0; k0 < mc; k0 += RCH) {
        const int kc = mc - k0 < RCH ? mc - k0 : RCH;
        for (int kk = 0; kk < RCH; ++kk) {
          T u1 = 0, u2 = 0;
          if (kk < kc) pair_grads(k0 + kk, u1, u2);
          *chan_slot(red_us, kk, 0) = (float)u1;
          *chan_slot(red_us, kk, 1) = (float)u2;
        }
        chan_reduce(kc, (const float*)P.en_W3, (const float*)P.en_Wenv, D.d, red_us, red_wp, (float*)red + k0 * 40);
      }
    } else {
      for (int k = 0; k < mc; ++k) {
        T u1, u2;
        pair_grads(k, u1, u2);
        pair_sums_waves(u1, u2, w3, wenv, act, D.h2, D.G, red4, red + k * 40);
      }
    }
    __syncthreads();
    if (tid < mc)
      edge_backward_terms<T>(feat + tid * EFEAT, red + tid * 40, red + tid * 40 + 8, P.en_W2, P.en_sig,
                             eterm + tid * ET);
    __syncthreads();
    edge_param_sums<T, true>(feat, eterm, mc, sW1, sb1, sW2, sb2, ssig);
  }
  __syncthreads();
  T* out = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * eo.size;
  for (int q = tid; q < eo.size; q += nt) out[q] = T(0);
  __syncthreads();
  // per-nucleus accumulators into their type rows (one thread per column)
  for (int k = 0; k < mc; ++k) {
    const int t = P.ntype[m0 + k];
    if (act) out[eo.nuc + t * D.d + c] += nucb[k * D.d + c];
    for (int q = tid; q < 5 * D.h1; q += nt) {
      if (q < 4 * D.h1) out[eo.W1 + t * 4 * D.h1 + q] += sW1[k * 4 * D.h1 + q];
      else out[eo.b1 + t * D.h1 + q - 4 * D.h1] += sb1[k * D.h1 + q - 4 * D.h1];
    }
    __syncthreads();
  }
  for (int q = tid; q < D.h1 * D.h2; q += nt) out[eo.W2 + q] = sW2[q];
  for (int q = tid; q < D.h2; q += nt) out[eo.b2 + q] = sb2[q];
  for (int q = tid; q < D.G; q += nt) out[eo.sig + q] = ssig[q];
  if (act) {
    for (int q = 0; q < D.h2; ++q) out[eo.W3 + q * D.d + c] = aW3[q];
    for (int q = 0; q < D.G; ++q) out[eo.Wenv + q * D.d + c] = aWenv[q];
    for (int q = 0; q < 4; ++q) out[eo.Wn + q * D.d + c] = aWn[q];
  }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct GradLayout {
  int Wc;
  size_t nidx, ncnt, y, ug, t, hk, zk, basis, o[2], obar[2], hbar, hbar2, zbar, h0bar, projbar, tbar, ugbar;
  size_t ybar, sbar, bbar, trA, trB, split, epart;
  size_t jm[7];   // MLP Jastrow: a1, z1, a2, z2, a2bar, z1bar/a1bar [rows][Hj]; readout bars [rows]
  size_t ja[10];  // attention Jastrow: V, Vbar [Wc][NV], abar [rows][NA], readout scratch as jm over Wc rows
  size_t total;
};

static GradLayout grad_layout(const fire_handle* h, int W) {
  const Dims& D = h->D;
  GradLayout L{};
  const size_t ts = h->tsize;
  const int nmax = D.nu > D.nd ? D.nu : D.nd;
  const int KNmax = D.K * nmax;
  int widest = 4 * D.d;
  if (KNmax > widest) widest = KNmax;
  if (D.B > widest) widest = D.B;
  if (D.NA() > widest) widest = D.NA();
  if (D.Ha > widest) widest = D.Ha;
  const size_t per_walker = (size_t)D.n * ts *
                            ((size_t)20 * D.d + 2 * (size_t)D.L * D.d + 2 * (size_t)D.B + 3 * (size_t)KNmax + 2 * widest +
                             (D.Hj > 0 ? (size_t)6 * D.Hj + 1 : 0) + (D.Ra > 0 ? (size_t)D.NA() + 8 * D.Ha : 0));
  const size_t budget = (size_t)24 << 30;
  int wc = (int)(budget / per_walker);
  if (wc < 1) wc = 1;
  if (wc > W) wc = W;
  L.Wc = wc;
  const int64_t R = (int64_t)wc * D.n;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  L.nidx = take(R * D.cap_nbr * 2);
  L.ncnt = take(R * 2 * 4);
  L.y = take(R * D.d * ts);
  L.ug = take(R * 2 * D.d * ts);
  L.t = take(R * D.d * ts);
  L.hk = take((size_t)(D.L + 1) * R * D.d * ts);
  L.zk = take((size_t)(D.L > 0 ? D.L : 1) * R * D.d * ts);
  L.basis = take(R * D.B * ts);
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s) > 0 ? D.nsig(s) : 1;
    L.o[s] = take((int64_t)wc * N * D.K * N * ts);
    L.obar[s] = take((int64_t)wc * N * D.K * N * ts);
  }
  L.hbar = take(R * D.d * ts);
  L.hbar2 = take(R * D.d * ts);
  L.zbar = take(R * D.d * ts);
  L.h0bar = take(R * D.d * ts);
  L.projbar = take(R * 4 * D.d * ts);
  L.tbar = take(R * D.d * ts);
  L.ugbar = take(R * 2 * D.d * ts);
  L.ybar = take(R * D.d * ts);
  L.sbar = take(R * D.d * ts);
  L.bbar = take(R * D.B * ts);
  L.trA = take(R * widest * ts);
  L.trB = take(R * widest * ts);
  L.split = take(((size_t)GNS * widest * widest > (size_t)CNS * widest ? (size_t)GNS * widest * widest
                                                                     : (size_t)CNS * widest) * ts);
  const size_t ep = (size_t)GBLK * ((size_t)msg_part_size(D) > (size_t)2 * D.d ? (size_t)msg_part_size(D) : 2 * D.d);
  const size_t enp = (size_t)GBLK * ((D.M + ENCH - 1) / ENCH) * en_off(D).size;
  L.epart = take((ep > enp ? ep : enp) * ts);
  for (int k = 0; k < 7; ++k) L.jm[k] = D.Hj > 0 ? take(R * (k < 6 ? D.Hj : 1) * ts) : 0;
  if (D.Ra > 0) {
    L.ja[0] = take((size_t)wc * D.NV() * ts);
    L.ja[1] = take((size_t)wc * D.NV() * ts);
    L.ja[2] = take(R * D.NA() * ts);
    for (int k = 0; k < 7; ++k) L.ja[3 + k] = take((size_t)wc * (k < 6 ? D.Ha : 1) * ts);
  }
  L.total = o;
  return L;
}

// the per-walker mode keeps a vector of ones (coefficients) after the layout
// after the adjoint's layout: W doubles (unit coefficients of the per-walker
// mode), then the cusp Jastrow's per-walker sums [W][4]
size_t grad_ws_bytes(const fire_handle* h, int W) {
  return grad_layout(h, W).total + align_up((size_t)W * 8) + align_up((size_t)W * 4 * 8);
}

// weight gradient C[a][b] = sum_r X[r][a] Y[r][b] (rows through maps), into grad
template <typename T>
static hipError_t wgrad(const fire_handle* h, const GradLayout& L, char* ws, const T* X, RowMap xm, int R, int A,
                        const T* Y, RowMap ym, int B, double* grad, int64_t base, int64_t sa, int64_t cpg, int64_t sbg,
                        int64_t sb, hipStream_t st) {
  T* xt = (T*)(ws + L.trA);
  T* yt = (T*)(ws + L.trB);
  T* part = (T*)(ws + L.split);
  hipLaunchKernelGGL(k_transpose<T>, dim3((R + 31) / 32, (A + 31) / 32), dim3(256), 0, st, X, xm, R, A, xt);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_transpose<T>, dim3((R + 31) / 32, (B + 31) / 32), dim3(256), 0, st, Y, ym, R, B, yt);
  CHECK(hipGetLastError());
  GemmArgs g{};
  g.A = xt; g.amap = rows_dense(R); g.Bt = yt; g.ldb = R; g.C = part; g.cmap = rows_dense(B); g.ccol = cols_dense();
  g.M = A; g.N = B; g.K = R; g.ksplit = GNS; g.c_split_stride = (int64_t)A * B;
  CHECK(gemm(sizeof(T) == 8 ? MMA_F64 : MMA_F32, g, st));
  hipLaunchKernelGGL(k_reduce_splits<T>, dim3((unsigned)(((int64_t)A * B + 255) / 256)), dim3(256), 0, st,
                     (const T*)part, GNS, A, B, grad, base, sa, cpg, sbg, sb);
  return hipGetLastError();
}

// bias gradient grad[base + c] += sum_r X[r][c]
template <typename T>
static hipError_t bgrad(const GradLayout& L, char* ws, const T* X, RowMap xm, int R, int C, double* grad, int64_t base,
                        hipStream_t st) {
  T* part = (T*)(ws + L.split);
  hipLaunchKernelGGL(k_colsum<T>, dim3((C + 255) / 256, CNS), dim3(256), 0, st, X, xm, R, C, CNS, part);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_splits<T>, dim3((C + 255) / 256), dim3(256), 0, st, (const T*)part, CNS, 1, C, grad,
                     base, (int64_t)0, (int64_t)1 << 40, (int64_t)0, (int64_t)1);
  return hipGetLastError();
}

// Backward of a pair of Jastrow readout MLPs over rows X [M][Q.in] (per rows
// per walker, walkers from w0): weight gradients into grad under the theta
// names prefix + W1, b1, W2, b2, w3, b3, and Xbar = sum_k a1bar_k W1_k^T
// (added to Xbar when accumulate).  buf: seven scratch arrays, six of [M][H]
// and one of [M] (T).
template <typename T>
static hipError_t readout_backward(const fire_handle* h, const GradLayout& L, char* ws, const Readout<T>& Q,
                                   const T* X, int M, int per, int w0, const char* state, size_t node_off,
                                   const double* coeff, const char* prefix, T* const* buf, T* Xbar, bool accumulate,
                                   double* grad, hipStream_t st) {
  const int H = Q.H, in = Q.in;
  T *a1 = buf[0], *z1 = buf[1], *a2 = buf[2], *z2 = buf[3], *a2b = buf[4], *z1b = buf[5], *gcol = buf[6];
  auto th = [&](const char* nm) { return theta_offset(h, (std::string(prefix) + nm).c_str()); };
  const int64_t nq = (int64_t)M * H;
  const unsigned gq = (unsigned)((nq + 255) / 256);
  for (int k = 0; k < 2; ++k) {
    const char* W1k = (const char*)Q.W1t + (size_t)k * H * in * h->gsize;
    const char* W2k = (const char*)Q.W2t + (size_t)k * H * H * h->gsize;
    GemmArgs g1{};
    g1.A = X; g1.amap = rows_dense(in); g1.Bt = W1k; g1.ldb = in; g1.bias = Q.b1 + (int64_t)k * H;
    g1.C = a1; g1.cmap = rows_dense(H); g1.ccol = cols_dense(); g1.M = M; g1.N = H; g1.K = in;
    CHECK(gemm_site(h, SITE_EMB, g1, st));
    hipLaunchKernelGGL(k_silu_inplace<T>, dim3(gq), dim3(256), 0, st, (const T*)a1, z1, nq);
    CHECK(hipGetLastError());
    GemmArgs g2{};
    g2.A = z1; g2.amap = rows_dense(H); g2.Bt = W2k; g2.ldb = H; g2.bias = Q.b2 + (int64_t)k * H;
    g2.C = a2; g2.cmap = rows_dense(H); g2.ccol = cols_dense(); g2.M = M; g2.N = H; g2.K = H;
    CHECK(gemm_site(h, SITE_EMB, g2, st));
    hipLaunchKernelGGL(k_silu_inplace<T>, dim3(gq), dim3(256), 0, st, (const T*)a2, z2, nq);
    CHECK(hipGetLastError());
    // z2 is not needed after this: it takes the readout-weight terms g z2
    hipLaunchKernelGGL(k_jm_readout_bar<T>, dim3(gq), dim3(256), 0, st, (int64_t)M, per, w0, H, k, state,
                       h->st.stride, node_off, coeff, Q.w3 + (int64_t)k * H, (const T*)a2, (const T*)z2, a2b, z2,
                       gcol);
    CHECK(hipGetLastError());
    CHECK(bgrad<T>(L, ws, z2, rows_dense(H), M, H, grad, th("w3") + (int64_t)k * H, st));
    CHECK(bgrad<T>(L, ws, gcol, rows_dense(1), M, 1, grad, th("b3") + k, st));
    CHECK(wgrad<T>(h, L, ws, z1, rows_dense(H), M, H, a2b, rows_dense(H), H, grad, th("W2") + (int64_t)k * H * H, H,
                   (int64_t)1 << 40, 0, 1, st));
    CHECK(bgrad<T>(L, ws, a2b, rows_dense(H), M, H, grad, th("b2") + (int64_t)k * H, st));
    // z1bar = a2bar W2_k^T, then a1bar = z1bar SiLU'(a1) (into a2, free now)
    GemmArgs b2{};
    b2.A = a2b; b2.amap = rows_dense(H); b2.Bt = (const char*)Q.W2n + (size_t)k * H * H * h->gsize;
    b2.ldb = H; b2.C = z1b; b2.cmap = rows_dense(H); b2.ccol = cols_dense(); b2.M = M; b2.N = H; b2.K = H;
    CHECK(gemm_site(h, SITE_GRAD, b2, st));
    hipLaunchKernelGGL(k_silu_bar<T>, dim3(gq), dim3(256), 0, st, (const T*)a1, (const T*)z1b, a2, nq);
    CHECK(hipGetLastError());
    CHECK(wgrad<T>(h, L, ws, X, rows_dense(in), M, in, a2, rows_dense(H), H, grad, th("W1") + (int64_t)k * in * H, H,
                   (int64_t)1 << 40, 0, 1, st));
    CHECK(bgrad<T>(L, ws, a2, rows_dense(H), M, H, grad, th("b1") + (int64_t)k * H, st));
    GemmArgs b1{};
    b1.A = a2; b1.amap = rows_dense(H); b1.Bt = (const char*)Q.W1n + (size_t)k * in * H * h->gsize;
    b1.ldb = H; b1.C = Xbar; b1.cmap = rows_dense(in); b1.ccol = cols_dense(); b1.M = M; b1.N = in;
    b1.K = H; b1.accumulate = accumulate || k == 1;
    CHECK(gemm_site(h, SITE_GRAD, b1, st));
  }
  return hipSuccess;
}

template <typename T>
static hipError_t grad_chunk(const fire_handle* h, const Net<T>& P, int w0, int Wc, const double* R, char* state,
                             char* ws, const double* coeff, double* grad, int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  const GradLayout L = grad_layout(h, Wc);
  const int n = D.n, d = D.d;
  const int64_t rows = (int64_t)Wc * n;
  const double* Rc = R + (int64_t)w0 * n * 3;
  const int blk = d <= 64 ? 64 : (d + 63) / 64 * 64;
  const int64_t srecT = S.stride / sizeof(T);
  auto th = [&](const char* nm) { return theta_offset(h, nm); };
  int16_t* nidx = (int16_t*)(ws + L.nidx);
  int32_t* ncnt = (int32_t*)(ws + L.ncnt);
  T* y = (T*)(ws + L.y);
  T* ug = (T*)(ws + L.ug);
  T* tt = (T*)(ws + L.t);
  T* hk = (T*)(ws + L.hk);
  T* zk = (T*)(ws + L.zk);
  T* basis = (T*)(ws + L.basis);
  T* hbar = (T*)(ws + L.hbar);
  T* hbar2 = (T*)(ws + L.hbar2);
  T* zbar = (T*)(ws + L.zbar);
  T* h0bar = (T*)(ws + L.h0bar);
  T* projbar = (T*)(ws + L.projbar);
  T* tbar = (T*)(ws + L.tbar);
  T* ugbar = (T*)(ws + L.ugbar);
  T* ybar = (T*)(ws + L.ybar);
  T* sbar = (T*)(ws + L.sbar);
  T* bbar = (T*)(ws + L.bbar);
  T* epart = (T*)(ws + L.epart);
  const char* st_base = state + (int64_t)w0 * S.stride;
  const RowMap h0map{n, srecT, d}, projmap{n, srecT, 4 * d};

  // ---- forward recompute of node activations
  launch_nbr(dim3(Wc), st, Rc, Wc, n, D.nu, D.cut * D.cut, D.cap_nbr, nidx, ncnt,
             status + w0);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_en_embed<T>, dim3((unsigned)((rows + EPB - 1) / EPB)), dim3(blk), 0, st, P, Rc, rows, y, EPB, (const int*)nullptr);
  CHECK(hipGetLastError());
  {
    GemmArgs g{};
    g.A = y; g.amap = rows_dense(d); g.Bt = P.Wvg_t; g.ldb = d; g.bias = P.b_vg;
    g.C = ug; g.cmap = rows_dense(2 * d); g.ccol = cols_dense(); g.M = (int)rows; g.N = 2 * d; g.K = d;
    CHECK(gemm_site(h, SITE_EMB, g, st));
  }
  hipLaunchKernelGGL(k_glu<T>, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, st, (const T*)ug, tt, rows, d, (const int*)nullptr);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_h1_from_state<T>, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, st, D, Wc, w0,
                     (const char*)state, S, hk);
  CHECK(hipGetLastError());
  for (int k = 0; k < D.L; ++k) {
    GemmArgs g{};
    g.A = hk + (int64_t)k * rows * d; g.amap = rows_dense(d);
    g.Bt = (const char*)P.mlp_t + (size_t)k * d * d * h->gsize; g.ldb = d; g.bias = P.mlp_b + (int64_t)k * d;
    g.C = zk + (int64_t)k * rows * d; g.cmap = rows_dense(d); g.ccol = cols_dense(); g.M = (int)rows; g.N = d; g.K = d;
    CHECK(gemm_site(h, SITE_EMB, g, st));
    hipLaunchKernelGGL(k_silu_inplace<T>, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, st,
                       (const T*)(zk + (int64_t)k * rows * d), hk + (int64_t)(k + 1) * rows * d, rows * d);
    CHECK(hipGetLastError());
  }
  const T* hL = hk + (int64_t)D.L * rows * d;
  hipLaunchKernelGGL(k_env_basis<T>, dim3((unsigned)((rows * D.B + 255) / 256)), dim3(256), 0, st, P, Rc, rows, basis, (const int*)nullptr);
  CHECK(hipGetLastError());

  // ---- orbitals and envelopes backward
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, st, hbar, rows * d, T(0));
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((rows * D.B + 255) / 256)), dim3(256), 0, st, bbar, rows * D.B, T(0));
  CHECK(hipGetLastError());
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s), e0 = s == 0 ? 0 : D.nu, KN = D.K * N;
    if (N == 0) continue;
    T* o = (T*)(ws + L.o[s]);
    T* ob = (T*)(ws + L.obar[s]);
    const RowMap sm{N, (int64_t)n * d, d};
    GemmArgs g{};
    g.A = hL + (int64_t)e0 * d; g.amap = sm; g.Bt = s == 0 ? P.orb_t0 : P.orb_t1; g.ldb = d;
    g.C = o; g.cmap = rows_dense(KN); g.ccol = cols_dense(); g.M = Wc * N; g.N = KN; g.K = d;
    CHECK(gemm_site(h, SITE_ORB, g, st));
    const int64_t tot = (int64_t)Wc * N * KN;
    if (h->isize == 8)
      hipLaunchKernelGGL((k_orb_bar<T, double>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, D, s, Wc, w0,
                         (const char*)state, S, coeff, o, ob);
    else
      hipLaunchKernelGGL((k_orb_bar<T, float>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, D, s, Wc, w0,
                         (const char*)state, S, coeff, o, ob);
    CHECK(hipGetLastError());
    // W_orb grad: [d][K N] -> orb_W[det][k][l]
    CHECK(wgrad<T>(h, L, ws, hL + (int64_t)e0 * d, sm, Wc * N, d, ob, rows_dense(KN), KN, grad,
                   th(s == 0 ? "orb_W_up" : "orb_W_dn"), N, N, (int64_t)d * N, 1, st));
    // pi grad: [B][K N] -> env_pi[(det,l)][b]
    const RowMap bm{N, (int64_t)n * D.B, D.B};
    CHECK(wgrad<T>(h, L, ws, basis + (int64_t)e0 * D.B, bm, Wc * N, D.B, o, rows_dense(KN), KN, grad,
                   th(s == 0 ? "env_pi_up" : "env_pi_dn"), 1, (int64_t)1 << 40, 0, D.B, st));
    // hbar = obar W^T,  basisbar = envbar pi
    GemmArgs hb{};
    hb.A = ob; hb.amap = rows_dense(KN); hb.Bt = s == 0 ? P.orb_n0 : P.orb_n1; hb.ldb = KN;
    hb.C = hbar + (int64_t)e0 * d; hb.cmap = sm; hb.ccol = cols_dense(); hb.M = Wc * N; hb.N = d; hb.K = KN;
    CHECK(gemm_site(h, SITE_GRAD, hb, st));
    GemmArgs bb{};
    bb.A = o; bb.amap = rows_dense(KN); bb.Bt = s == 0 ? P.pi_n0 : P.pi_n1; bb.ldb = KN;
    bb.C = bbar + (int64_t)e0 * D.B; bb.cmap = bm; bb.ccol = cols_dense(); bb.M = Wc * N; bb.N = D.B; bb.K = KN;
    CHECK(gemm_site(h, SITE_GRAD, bb, st));
    // envelope exponents
    T* part = (T*)(ws + L.split);
    hipLaunchKernelGGL(k_envsig_bar<T>, dim3((D.B + 255) / 256, GNS), dim3(256), 0, st, P, Rc, e0, N, Wc,
                       (const T*)(bbar + (int64_t)e0 * D.B), GNS, part);
    CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_splits<T>, dim3((D.B + 255) / 256), dim3(256), 0, st, (const T*)part, GNS, 1, D.B,
                       grad, th("env_sigma"), (int64_t)0, (int64_t)1 << 40, (int64_t)0, (int64_t)1);
    CHECK(hipGetLastError());
  }
  // ---- Jastrow readouts backward: the MLP Jastrow over the final
  // embeddings (hbar += its input adjoint), then the attention Jastrow over
  // the register embeddings and its softmax (hbar += abar Pn)
  T* jb[7];
  for (int k = 0; k < 7; ++k) jb[k] = (T*)(ws + L.jm[k]);
  if (D.Hj > 0)
    CHECK(readout_backward<T>(h, L, ws, jm_readout<T>(h, P), hL, (int)rows, n, w0, state, S.jms + 8, coeff, "jmlp_",
                              jb, hbar, true, grad, st));
  if (D.Ra > 0) {
    const int NV = D.NV(), NA = D.NA();
    T* V = (T*)(ws + L.ja[0]);
    T* Vbar = (T*)(ws + L.ja[1]);
    T* abar = (T*)(ws + L.ja[2]);
    T* rb[7];
    for (int k = 0; k < 7; ++k) rb[k] = (T*)(ws + L.ja[3 + k]);
    hipLaunchKernelGGL(k_ja_vrows<T>, dim3((unsigned)(((int64_t)Wc * NV + 255) / 256)), dim3(256), 0, st, D, Wc, w0,
                       (const char*)state, S, V);
    CHECK(hipGetLastError());
    CHECK(readout_backward<T>(h, L, ws, ja_readout<T>(h, P), V, Wc, 1, w0, state,
                              S.jat + (size_t)(2 * D.Ra + NV + 1) * 8, coeff, "jatt_", rb, Vbar, false, grad, st));
    hipLaunchKernelGGL(k_ja_bar<T>, dim3((unsigned)rows), dim3(256), 0, st, D, w0, (const char*)state, S,
                       (const T*)Vbar, abar);
    CHECK(hipGetLastError());
    // q[r][c] += sum_rows h[c] lbar[r];  Wv[r][c][e] += sum_rows h[c] ubar[r dr + e]
    CHECK(wgrad<T>(h, L, ws, hL, rows_dense(d), (int)rows, d, abar, rows_dense(NA), D.Ra, grad, th("jatt_q"), 1,
                   (int64_t)1 << 40, 0, d, st));
    CHECK(wgrad<T>(h, L, ws, hL, rows_dense(d), (int)rows, d, abar + D.Ra, rows_dense(NA), NV, grad, th("jatt_Wv"),
                   D.dr, D.dr, (int64_t)d * D.dr, 1, st));
    GemmArgs b1{};
    b1.A = abar; b1.amap = rows_dense(NA); b1.Bt = P.ja_Pn; b1.ldb = NA;
    b1.C = hbar; b1.cmap = rows_dense(d); b1.ccol = cols_dense(); b1.M = (int)rows; b1.N = d; b1.K = NA;
    b1.accumulate = 1;
    CHECK(gemm_site(h, SITE_GRAD, b1, st));
  }
  // ---- MLP backward
  T* hb_cur = hbar;
  T* hb_nxt = hbar2;
  for (int k = D.L - 1; k >= 0; --k) {
    const T* z = zk + (int64_t)k * rows * d;
    const T* hin = hk + (int64_t)k * rows * d;
    hipLaunchKernelGGL(k_silu_bar<T>, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, st, z,
                       (const T*)hb_cur, zbar, rows * d);
    CHECK(hipGetLastError());
    CHECK(wgrad<T>(h, L, ws, hin, rows_dense(d), (int)rows, d, zbar, rows_dense(d), d, grad,
                   th("mlp_W") + (int64_t)k * d * d, d, (int64_t)1 << 40, 0, 1, st));
    CHECK(bgrad<T>(L, ws, zbar, rows_dense(d), (int)rows, d, grad, th("mlp_b") + (int64_t)k * d, st));
    GemmArgs g{};
    g.A = zbar; g.amap = rows_dense(d); g.Bt = (const char*)P.mlp_n + (size_t)k * d * d * h->gsize; g.ldb = d;
    g.C = hb_nxt; g.cmap = rows_dense(d); g.ccol = cols_dense(); g.M = (int)rows; g.N = d; g.K = d;
    CHECK(gemm_site(h, SITE_GRAD, g, st));
    T* t = hb_cur; hb_cur = hb_nxt; hb_nxt = t;
  }
  // hb_cur = d/d h1 = mbar;  h0bar starts as h1bar
  CHECK(hipMemcpyAsync(h0bar, hb_cur, (size_t)rows * d * sizeof(T), hipMemcpyDeviceToDevice, st));
  // ---- messages backward
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((rows * 4 * d + 255) / 256)), dim3(256), 0, st, projbar, rows * 4 * d,
                     T(0));
  CHECK(hipGetLastError());
  const FiltOff fo = filt_off(D);
  const size_t msg_lds = (size_t)(fo.W3 + D.G) * sizeof(T);
  CHECK(hipFuncSetAttribute((const void*)k_msg_bwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)msg_lds));
  const int nb_msg = rows < GBLK ? (int)rows : GBLK;
  hipLaunchKernelGGL(k_msg_bwd<T>, dim3(nb_msg, 2), dim3(blk), msg_lds, st, P, Rc, rows, w0, (const int16_t*)nidx,
                     (const int32_t*)ncnt, (const char*)state, S, (const T*)hb_cur, projbar, epart);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_projbar_gather<T>, dim3(nb_msg, 2), dim3(blk), 0, st, P, Rc, rows, w0, (const int16_t*)nidx,
                     (const int32_t*)ncnt, (const char*)state, S, (const T*)hb_cur, projbar);
  CHECK(hipGetLastError());
  {
    const int ps = msg_part_size(D);
    for (int a = 0; a < 2; ++a) {
      const int64_t o = (int64_t)a * (fo.size + 5 * d);
      auto red = [&](int64_t col, int len, int64_t base) {
        hipLaunchKernelGGL(k_reduce_cols, dim3(len), dim3(256), 0, st, (const void*)epart, (int)sizeof(T),
                           nb_msg, (int64_t)ps, o + col, len, grad, base);
        return hipGetLastError();
      };
      CHECK(red(fo.W1, 4 * D.h1, th("ee_W1") + a * 4 * D.h1));
      CHECK(red(fo.b1, D.h1, th("ee_b1") + a * D.h1));
      CHECK(red(fo.W2, D.h1 * D.h2, th("ee_W2") + a * D.h1 * D.h2));
      CHECK(red(fo.b2, D.h2, th("ee_b2") + a * D.h2));
      CHECK(red(fo.W3, D.h2 * d, th("ee_W3") + (int64_t)a * D.h2 * d));
      CHECK(red(fo.Wenv, D.G * d, th("ee_Wenv") + (int64_t)a * D.G * d));
      CHECK(red(fo.sig, D.G, th("ee_sig") + a * D.G));
      CHECK(red(fo.size, 4 * d, th("msg_We") + (int64_t)a * 4 * d));
      CHECK(red(fo.size + 4 * d, d, th("msg_b") + (int64_t)a * d));
    }
  }
  // ---- node projections: W_proj grad and h0bar += projbar W_proj^T
  CHECK(wgrad<T>(h, L, ws, (const T*)(st_base + S.h0), h0map, (int)rows, d, projbar, rows_dense(4 * d), 4 * d, grad,
                 th("msg_Wa"), d, d, (int64_t)d * d, 1, st));
  {
    GemmArgs g{};
    g.A = projbar; g.amap = rows_dense(4 * d); g.Bt = P.Wproj_n; g.ldb = 4 * d;
    g.C = h0bar; g.cmap = rows_dense(d); g.ccol = cols_dense(); g.M = (int)rows; g.N = d; g.K = 4 * d;
    g.accumulate = 1;
    CHECK(gemm_site(h, SITE_GRAD, g, st));
  }
  // ---- GLU backward
  CHECK(wgrad<T>(h, L, ws, tt, rows_dense(d), (int)rows, d, h0bar, rows_dense(d), d, grad, th("glu_Wo"), d,
                 (int64_t)1 << 40, 0, 1, st));
  CHECK(bgrad<T>(L, ws, h0bar, rows_dense(d), (int)rows, d, grad, th("glu_bo"), st));
  {
    GemmArgs g{};
    g.A = h0bar; g.amap = rows_dense(d); g.Bt = P.Wo_n; g.ldb = d;
    g.C = tbar; g.cmap = rows_dense(d); g.ccol = cols_dense(); g.M = (int)rows; g.N = d; g.K = d;
    CHECK(gemm_site(h, SITE_GRAD, g, st));
  }
  hipLaunchKernelGGL(k_glu_bar<T>, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, st, (const T*)ug,
                     (const T*)tbar, ugbar, rows, d);
  CHECK(hipGetLastError());
  CHECK(wgrad<T>(h, L, ws, y, rows_dense(d), (int)rows, d, ugbar, rows_dense(2 * d), d, grad, th("glu_Wv"), d,
                 (int64_t)1 << 40, 0, 1, st));
  CHECK(wgrad<T>(h, L, ws, y, rows_dense(d), (int)rows, d, ugbar + d, rows_dense(2 * d), d, grad, th("glu_Wg"), d,
                 (int64_t)1 << 40, 0, 1, st));
  CHECK(bgrad<T>(L, ws, ugbar, rows_dense(2 * d), (int)rows, d, grad, th("glu_bv"), st));
  CHECK(bgrad<T>(L, ws, ugbar + d, rows_dense(2 * d), (int)rows, d, grad, th("glu_bg"), st));
  {
    GemmArgs g{};
    g.A = ugbar; g.amap = rows_dense(2 * d); g.Bt = P.Wvg_n; g.ldb = 2 * d;
    g.C = ybar; g.cmap = rows_dense(d); g.ccol = cols_dense(); g.M = (int)rows; g.N = d; g.K = 2 * d;
    CHECK(gemm_site(h, SITE_GRAD, g, st));
  }
  // ---- LayerNorm and electron-nucleus backward
  const int nb_ln = rows < GBLK ? (int)rows : GBLK;
  hipLaunchKernelGGL(k_ln_bwd<T>, dim3(nb_ln), dim3(blk), 0, st, P, Rc, rows, (const T*)ybar, sbar, epart);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_cols, dim3(d), dim3(256), 0, st, (const void*)epart, (int)sizeof(T), nb_ln,
                     (int64_t)2 * d, (int64_t)0, d, grad, th("ln_g"));
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_cols, dim3(d), dim3(256), 0, st, (const void*)epart, (int)sizeof(T), nb_ln,
                     (int64_t)2 * d, (int64_t)d, d, grad, th("ln_b"));
  CHECK(hipGetLastError());
  {
    const EnOff eo = en_off(D);
    const size_t en_lds = ((size_t)ENCH * d + ENCH * 5 * D.h1 + D.h1 * D.h2 + D.h2 + D.G) * sizeof(T);
    CHECK(hipFuncSetAttribute((const void*)k_en_bwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)en_lds));
    const int nmc = (D.M + ENCH - 1) / ENCH;
    const int nbx = rows < GBLK ? (int)rows : GBLK;
    hipLaunchKernelGGL(k_en_bwd<T>, dim3(nbx, nmc), dim3(blk), en_lds, st, P, Rc, rows, (const T*)sbar, epart);
    CHECK(hipGetLastError());
    const int nbt = nbx * nmc;
    auto red = [&](int64_t col, int len, int64_t base) {
      hipLaunchKernelGGL(k_reduce_cols, dim3(len), dim3(256), 0, st, (const void*)epart, (int)sizeof(T),
                         nbt, (int64_t)eo.size, col, len, grad, base);
      return hipGetLastError();
    };
    CHECK(red(eo.nuc, D.NT * d, th("nuc_emb")));
    CHECK(red(eo.W1, D.NT * 4 * D.h1, th("en_W1")));
    CHECK(red(eo.b1, D.NT * D.h1, th("en_b1")));
    CHECK(red(eo.W2, D.h1 * D.h2, th("en_W2")));
    CHECK(red(eo.b2, D.h2, th("en_b2")));
    CHECK(red(eo.W3, D.h2 * d, th("en_W3")));
    CHECK(red(eo.Wenv, D.G * d, th("en_Wenv")));
    CHECK(red(eo.sig, D.G, th("en_sig")));
    CHECK(red(eo.Wn, 4 * d, th("en_Wn")));
  }
  return hipSuccess;
}

// Gradient of sum_w c_w log J_cusp,w by the Jastrow parameters q = (w_par,
// a_par, w_anti, a_anti): for u = w a^2/(a + r), du/dw = a^2/(a + r) and
// du/da = w a (a + 2r)/(a + r)^2, summed over the pairs of each walker; one
// workgroup per walker writes c_w times its sums to part[w][0..3] (zeros for a
// flagged walker), which k_jas_sum adds into g in walker order; with
// gstride > 0 the sums go to walker w's own row g + w gstride instead.
__global__ __launch_bounds__(256) void k_jas_grad(const Dims D, int W, const double* __restrict__ R,
                                                  const double* __restrict__ q, const double* __restrict__ coeff,
                                                  const int32_t* __restrict__ status, double* __restrict__ g,
                                                  int64_t gstride, double* __restrict__ part) {
  __shared__ double red[16];
  const int w = blockIdx.x, n = D.n;
  if (status[w] != 0 || coeff[w] == 0.0) {
    if (part && threadIdx.x < 4) part[4 * w + threadIdx.x] = 0.0;
    return;
  }
  if (gstride > 0) g += (int64_t)w * gstride;
  const double* Rw = R + (int64_t)w * n * 3;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t - i * n;
    if (j <= i) continue;
    const double dx = Rw[3 * i] - Rw[3 * j], dy = Rw[3 * i + 1] - Rw[3 * j + 1], dz = Rw[3 * i + 2] - Rw[3 * j + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const int o = (i < D.nu) == (j < D.nu) ? 0 : 2;
    const double wv = q[o], a = q[o + 1], t1 = 1.0 / (a + r);
    s[o] += a * a * t1;
    s[o + 1] += wv * a * (a + 2.0 * r) * t1 * t1;
  }
  for (int k = 0; k < 4; ++k) {
    const double v = block_sum<double>(s[k], red);
    if (threadIdx.x == 0) {
      if (part) part[4 * w + k] = coeff[w] * v;
      else g[k] += coeff[w] * v;
    }
    __syncthreads();
  }
}

// g[k] += sum_w part[w][k], each thread over a fixed stride of walkers and
// the block sum in a fixed order (the result does not depend on scheduling)
__global__ __launch_bounds__(256) void k_jas_sum(int W, const double* __restrict__ part, double* __restrict__ g) {
  __shared__ double red[16];
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int w = threadIdx.x; w < W; w += blockDim.x) s += part[4 * w + k];
    s = block_sum<double>(s, red);
    if (threadIdx.x == 0) g[k] += s;
    __syncthreads();
  }
}

// grad[p] = sum_w coeff[w] O[w][p] over the per-walker gradients
__global__ void k_weighted_rows(int64_t P, int W, const double* __restrict__ O, const double* __restrict__ coeff,
                                double* __restrict__ grad) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int w = 0; w < W; ++w) s += coeff[w] * O[(int64_t)w * P + p];
  grad[p] = s;
}

template <typename T>
static hipError_t grad_impl(fire_handle* h, int W, const double* R, char* state, char* ws, const double* coeff,
                            double* grad, double* per_walker, int32_t* status, hipStream_t st) {
  Net<T> P = make_net<T>(h);
  const GradLayout L = grad_layout(h, W);
  CHECK(fill_i32(status, W, 0, st));
  if (!per_walker) {
    hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)((h->P + 255) / 256)), dim3(256), 0, st, grad, (int64_t)h->P,
                       0.0);
    CHECK(hipGetLastError());
    for (int w0 = 0; w0 < W; w0 += L.Wc) {
      const int wc = W - w0 < L.Wc ? W - w0 : L.Wc;
      CHECK(grad_chunk<T>(h, P, w0, wc, R, state, ws, coeff, grad, status, st));
    }
    double* jpart = (double*)(ws + L.total + align_up((size_t)W * 8));
    hipLaunchKernelGGL(k_jas_grad, dim3(W), dim3(256), 0, st, h->D, W, R, P.jas, coeff, (const int32_t*)status,
                       grad + theta_offset(h, "jas_cusp"), (int64_t)0, jpart);
    CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_jas_sum, dim3(1), dim3(256), 0, st, W, (const double*)jpart,
                       grad + theta_offset(h, "jas_cusp"));
    return hipGetLastError();
  }
  // Per-walker gradients O[w] = d log|psi_w| / d theta: the same adjoint run
  // one walker at a time (coefficient 1) into that walker's row, then
  // grad = sum_w coeff_w O[w].  One-walker chunks keep every reduction of the
  // batched adjoint unchanged; the cost is launch-bound (about 70 launches
  // per walker).
  double* ones = (double*)(ws + L.total);
  hipLaunchKernelGGL(k_fill<double>, dim3((W + 255) / 256), dim3(256), 0, st, ones, (int64_t)W, 1.0);
  CHECK(hipGetLastError());
  const int64_t WP = (int64_t)W * h->P;
  hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)((WP + 255) / 256)), dim3(256), 0, st, per_walker, WP, 0.0);
  CHECK(hipGetLastError());
  for (int w = 0; w < W; ++w)
    CHECK(grad_chunk<T>(h, P, w, 1, R, state, ws, ones, per_walker + (int64_t)w * h->P, status, st));
  hipLaunchKernelGGL(k_jas_grad, dim3(W), dim3(256), 0, st, h->D, W, R, P.jas, (const double*)ones,
                     (const int32_t*)status, per_walker + theta_offset(h, "jas_cusp"), (int64_t)h->P,
                     (double*)nullptr);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_weighted_rows, dim3((unsigned)((h->P + 255) / 256)), dim3(256), 0, st, (int64_t)h->P, W,
                     (const double*)per_walker, coeff, grad);
  return hipGetLastError();
}

hipError_t grad_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* coeff, double* grad,
                     double* per_walker, int32_t* status, hipStream_t s) {
  const Dims& D = h->D;
  if (D.M > 4096 || D.d > 256) return hipErrorInvalidValue;
  return h->tsize == 8 ? grad_impl<double>(h, W, R, state, ws, coeff, grad, per_walker, status, s)
                       : grad_impl<float>(h, W, R, state, ws, coeff, grad, per_walker, status, s);
}

}  // namespace fire
