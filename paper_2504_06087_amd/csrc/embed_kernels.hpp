// Kernels shared by the full evaluation and the single-electron update path.
#pragma once
#include "forward.hpp"

namespace fire {

// ---------------------------------------------------------------------------
// a1: neighbour lists through a cell list.  One workgroup per walker, one
// thread per electron (NMAX = 256 or 512 threads, n <= NMAX): the walker's electrons are binned into a grid over their bounding
// box whose cells are at least c wide along every axis (at most 12 per axis),
// so every pair within c lies in the same or an adjacent cell; electron i
// then tests only the members of its 27 surrounding cells.  The hits are
// kept as a bit set over electron indices and emitted in ascending index,
// same-spin first, then opposite spin: the same lists, in the same order, as
// a test of every pair.
// ---------------------------------------------------------------------------
constexpr int kNbrCellsPerAxis = 12;
constexpr int kNbrCells = kNbrCellsPerAxis * kNbrCellsPerAxis * kNbrCellsPerAxis;

template <int NMAX>
__global__ __launch_bounds__(NMAX) void k_nbr(const double* __restrict__ R, int W, int n, int nu,
                                              double cut2, int cap, int16_t* __restrict__ idx,
                                              int32_t* __restrict__ cnt, int32_t* status) {
  constexpr int NW = NMAX / 64;   // waves; also 64-bit words of the hit set
  __shared__ double pos[NMAX * 3];
  __shared__ int cell_of[NMAX];
  __shared__ int cstart[kNbrCells + 1];
  __shared__ int cfill[kNbrCells];
  __shared__ int16_t members[NMAX];
  __shared__ double red[2][3][NW];
  __shared__ double box_lo[3], box_h[3];
  __shared__ int box_g[3];
  const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Rw = R + (int64_t)w * n * 3;
  for (int t = tid; t < 3 * n; t += blockDim.x) pos[t] = Rw[t];
  for (int t = tid; t < kNbrCells; t += blockDim.x) cfill[t] = 0;
  __syncthreads();
  const bool mine = tid < n;
  double xi = 0, yi = 0, zi = 0;
  bool fin = false;
  if (mine) {
    xi = pos[3 * tid]; yi = pos[3 * tid + 1]; zi = pos[3 * tid + 2];
    fin = isfinite(xi) && isfinite(yi) && isfinite(zi);
    if (!fin) atomicOr(status + w, FIRE_W_NONFINITE);
  }
  // bounding box of the finite positions
  double lo[3] = {fin ? xi : INFINITY, fin ? yi : INFINITY, fin ? zi : INFINITY};
  double hi[3] = {fin ? xi : -INFINITY, fin ? yi : -INFINITY, fin ? zi : -INFINITY};
#pragma unroll
  for (int k = 0; k < 3; ++k)
    for (int o = 32; o > 0; o >>= 1) {
      lo[k] = fmin(lo[k], __shfl_xor(lo[k], o, 64));
      hi[k] = fmax(hi[k], __shfl_xor(hi[k], o, 64));
    }
  if (lane == 0)
    for (int k = 0; k < 3; ++k) { red[0][k][wave] = lo[k]; red[1][k][wave] = hi[k]; }
  __syncthreads();
  if (tid < 3) {
    double l = INFINITY, h = -INFINITY;
    for (int v = 0; v < (int)(blockDim.x >> 6); ++v) { l = fmin(l, red[0][tid][v]); h = fmax(h, red[1][tid][v]); }
    const double c = sqrt(cut2);
    int g = 1;
    double ext = h - l;
    if (!(ext > 0) || !isfinite(ext)) { ext = 0; l = isfinite(l) ? l : 0.0; }
    if (c > 0 && c < 1e300 && ext > 0) {
      const double q = ceil(ext / c);
      g = q < 1 ? 1 : (q > kNbrCellsPerAxis ? kNbrCellsPerAxis : (int)q);
    }
    // cells at least c wide, g of them covering the extent
    const double hw = fmax(c, ext / g);
    box_lo[tid] = l;
    box_h[tid] = hw > 0 && isfinite(hw) ? hw : 1.0;
    box_g[tid] = g;
  }
  __syncthreads();
  const int gx = box_g[0], gy = box_g[1], gz = box_g[2];
  int cx = 0, cy = 0, cz = 0;
  if (mine) {
    if (fin) {
      cx = (int)((xi - box_lo[0]) / box_h[0]); cx = cx < 0 ? 0 : (cx >= gx ? gx - 1 : cx);
      cy = (int)((yi - box_lo[1]) / box_h[1]); cy = cy < 0 ? 0 : (cy >= gy ? gy - 1 : cy);
      cz = (int)((zi - box_lo[2]) / box_h[2]); cz = cz < 0 ? 0 : (cz >= gz ? gz - 1 : cz);
    }
    const int cidx = (cz * gy + cy) * gx + cx;
    cell_of[tid] = cidx;
    atomicAdd(&cfill[cidx], 1);
  }
  __syncthreads();
  // exclusive scan of the cell counts (wave 0; at most 1728 cells)
  const int ncell = gx * gy * gz;
  if (wave == 0) {
    const int per = (ncell + 63) / 64;
    const int b0 = lane * per, b1 = b0 + per < ncell ? b0 + per : ncell;
    int sacc = 0;
    for (int t = b0; t < b1; ++t) sacc += cfill[t];
    int incl = sacc;
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    int run = incl - sacc;
    for (int t = b0; t < b1; ++t) { cstart[t] = run; run += cfill[t]; cfill[t] = 0; }
    if (lane == 63) cstart[ncell] = incl;
  }
  __syncthreads();
  if (mine) {
    const int cidx = cell_of[tid];
    members[cstart[cidx] + atomicAdd(&cfill[cidx], 1)] = (int16_t)tid;
  }
  __syncthreads();
  if (!mine) return;
  uint64_t hit[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) hit[q] = 0;
  if (fin) {
    for (int dz = -1; dz <= 1; ++dz) {
      const int z = cz + dz;
      if (z < 0 || z >= gz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int y = cy + dy;
        if (y < 0 || y >= gy) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = cx + dx;
          if (x < 0 || x >= gx) continue;
          const int cc = (z * gy + y) * gx + x;
          for (int t = cstart[cc]; t < cstart[cc + 1]; ++t) {
            const int j = members[t];
            if (j == tid) continue;
            const double ddx = xi - pos[3 * j], ddy = yi - pos[3 * j + 1], ddz = zi - pos[3 * j + 2];
            if (ddx * ddx + ddy * ddy + ddz * ddz <= cut2) {
#pragma unroll
              for (int q = 0; q < NW; ++q)
                if (q == (j >> 6)) hit[q] |= 1ull << (j & 63);
            }
          }
        }
      }
    }
  }
  // emit: same spin class first, then the other, ascending index
  int16_t* out = idx + ((int64_t)w * n + tid) * cap;
  const int si = tid < nu ? 0 : 1;
  int c[2] = {0, 0};
  int k = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const bool up = (pass == 0) == (si == 0);        // this pass lists spin-up electrons
    const int j0 = up ? 0 : nu, j1 = up ? nu : n;
    for (int q = 0; q < NW; ++q) {
      uint64_t m = hit[q];
      const int base = 64 * q;
      // keep the bits of [j0, j1)
      if (base + 64 <= j0 || base >= j1) continue;
      if (j0 > base) m &= ~0ull << (j0 - base);
      if (j1 < base + 64) m &= (j1 - base) >= 64 ? ~0ull : ((1ull << (j1 - base)) - 1);
      while (m) {
        const int j = base + __builtin_ctzll(m);
        m &= m - 1;
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
  cnt[((int64_t)w * n + tid) * 2 + 0] = c[0];
  cnt[((int64_t)w * n + tid) * 2 + 1] = c[1];
}

// One thread per electron: 256 threads up to 256 electrons, 512 up to 512.
inline void launch_nbr(dim3 grid, hipStream_t st, const double* R, int W, int n, int nu, double cut2, int cap,
                       int16_t* idx, int32_t* cnt, int32_t* status) {
  if (n <= 256)
    hipLaunchKernelGGL(k_nbr<256>, grid, dim3(256), 0, st, R, W, n, nu, cut2, cap, idx, cnt, status);
  else
    hipLaunchKernelGGL(k_nbr<512>, grid, dim3(512), 0, st, R, W, n, nu, cut2, cap, idx, cnt, status);
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

// The same features with the layer-2 and envelope weights of a filter staged
// in LDS (stage_filter: W2 transposed, zero-padded to the compile-time
// maxima) and every weight read where it is used: far fewer live registers
// than pair_features, for kernels whose occupancy its preloaded weights would
// limit.  W1 [4][h1] and b1 [h1] may sit in LDS or in global memory.  Same
// products in the same order, so the results equal pair_features bit for bit.
constexpr int FW_W1 = 0, FW_B1 = 4 * kMaxH1, FW_W2T = FW_B1 + kMaxH1, FW_B2 = FW_W2T + kMaxH1 * kMaxH2,
              FW_SIG = FW_B2 + kMaxH2, FW_SIZE = FW_SIG + kMaxG;
// fw[FW_W1..] = W1 [4][h1] and fw[FW_B1..] = b1 (compact, when W1 is given),
// fw[FW_W2T + k kMaxH1 + j] = W2[j][k], then b2 and the envelope widths.
template <typename T>
FIRE_DEV void stage_filter(const T* W1, const T* b1, const T* W2, const T* b2, const T* sig, const Dims& D, T* fw,
                           int tid, int nt) {
  for (int q = tid; q < FW_SIZE; q += nt) {
    T v = 0;
    if (q < FW_B1) {
      if (W1 && q < 4 * D.h1) v = W1[q];
    } else if (q < FW_W2T) {
      if (W1 && q - FW_B1 < D.h1) v = b1[q - FW_B1];
    } else if (q < FW_B2) {
      const int k = (q - FW_W2T) / kMaxH1, j = (q - FW_W2T) % kMaxH1;
      if (k < D.h2 && j < D.h1) v = W2[j * D.h2 + k];
    } else if (q < FW_SIG) {
      if (q - FW_B2 < D.h2) v = b2[q - FW_B2];
    } else {
      if (q - FW_SIG < D.G) v = sig[q - FW_SIG];
    }
    fw[q] = v;
  }
}
template <typename T>
FIRE_DEV void pair_features_lds(T dx, T dy, T dz, const T* W1, const T* b1, const T* fw, T cut, const Dims& D,
                                T* out) {
  T r = sqrt(dx * dx + dy * dy + dz * dz);
  T e4[4] = {r, dx, dy, dz};
  T lo = log1p_over(r);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = lo * e4[k];
  T z1[kMaxH1];
#pragma unroll
  for (int k = 0; k < kMaxH1; ++k) {
    if (k < D.h1) {
      T a = b1[k];
#pragma unroll
      for (int j = 0; j < 4; ++j) a += e4[j] * W1[j * D.h1 + k];
      z1[k] = silu_(a);
    } else {
      z1[k] = T(0);
    }
  }
#pragma unroll 2
  for (int k = 0; k < kMaxH2; ++k) {
    if (k < D.h2) {
      const T* w2 = fw + FW_W2T + k * kMaxH1;
      T a = fw[FW_B2 + k];
#pragma unroll
      for (int j = 0; j < kMaxH1; ++j) a += z1[j] * w2[j];
      out[4 + k] = silu_(a);
    }
  }
  T fc = fcut_(r / cut);
#pragma unroll 4
  for (int k = 0; k < kMaxG; ++k) {
    const T sg = fw[FW_SIG + k];
    if (k < D.G) out[12 + k] = fc * exp(-(sg * sg) * r * r);
  }
  out[44] = fc;
}

// ---------------------------------------------------------------------------
// a2 + a3 (first half): s_i = sum_m Gamma_m(e_im) * (nuc_emb_m + ebar_im W_n),
// then y_i = LayerNorm(s_i).  Workgroup: one thread per channel, epb
// electrons, ERB of them at a time: the pair features of ERB electrons x up
// to MCH nuclei are formed together (one thread per pair), then every
// channel sums the ERB rows.
// ---------------------------------------------------------------------------
constexpr int EPB = 8;
constexpr int MCH = 64;

// per-value sums over the workgroup (wave sums, then the waves in order)
template <typename T, int NR> FIRE_DEV void block_sums(T (&v)[NR], T* red) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = wave_sum(v[r]);
  __syncthreads();
  if (l == 0)
#pragma unroll
    for (int r = 0; r < NR; ++r) red[w * NR + r] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    T t = 0;
    for (int k = 0; k < nw; ++k) t += red[k * NR + r];
    v[r] = t;
  }
}

// ERB electrons per pass (LDS: ERB x MCH pair features); launches of at most
// two electrons per workgroup take ERB = 2.  The layer-1 weights of the first
// EN_LDS_TYPES nucleus types are staged in LDS with the shared filter weights.
constexpr int EN_LDS_TYPES = 8;
template <typename T> constexpr int en_erb() { return sizeof(T) == 4 ? 4 : 2; }
template <typename T, int ERB = en_erb<T>()>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1) void k_en_embed(Net<T> P, const double* __restrict__ R,
                                                                        int64_t nrows, T* __restrict__ y_out, int epb,
                                                                        const int* __restrict__ nrows_dev) {
  // rows at or beyond a device row count (when given) are inactive
  if (nrows_dev && *nrows_dev < nrows) nrows = *nrows_dev;
  if ((int64_t)blockIdx.x * epb >= nrows) return;
  const Dims& D = P.D;
  __shared__ T feat[ERB * MCH * FEAT];
  __shared__ int ntp[MCH];
  __shared__ T red[4 * ERB];
  __shared__ T fw[FW_SIZE];
  __shared__ T w1t[EN_LDS_TYPES * 5 * kMaxH1];   // per type: W1 [4][h1], then b1 [h1]
  const int c = threadIdx.x, nt = blockDim.x;
  const bool act = c < D.d;
  stage_filter<T>(nullptr, nullptr, P.en_W2, P.en_b2, P.en_sig, D, fw, c, nt);
  {
    const int ntl = D.NT < EN_LDS_TYPES ? D.NT : EN_LDS_TYPES;
    for (int q = c; q < ntl * 5 * D.h1; q += nt) {
      const int t = q / (5 * D.h1), i = q - t * 5 * D.h1;
      w1t[t * 5 * kMaxH1 + i] = i < 4 * D.h1 ? P.en_W1[t * 4 * D.h1 + i] : P.en_b1[t * D.h1 + i - 4 * D.h1];
    }
  }
  T w3[kMaxH2], wenv[kMaxG], wn[4], nemb[4];
  if (act) {
    for (int k = 0; k < D.h2; ++k) w3[k] = P.en_W3[k * D.d + c];
    for (int k = 0; k < D.G; ++k) wenv[k] = P.en_Wenv[k * D.d + c];
    for (int k = 0; k < 4; ++k) wn[k] = P.en_Wn[k * D.d + c];
  }
  // embeddings of the first four nucleus types of this channel
  for (int t = 0; t < 4; ++t) nemb[t] = (act && t < D.NT) ? P.nuc_emb[t * D.d + c] : T(0);
  const int64_t e_beg = (int64_t)blockIdx.x * epb;
  const int64_t e_end = e_beg + epb < nrows ? e_beg + epb : nrows;
  // electrons per pass: one pair per thread (the block has >= MCH threads)
  const int mmax = D.M < MCH ? D.M : MCH;
  const int rpp = nt / mmax < ERB ? (nt / mmax > 0 ? nt / mmax : 1) : ERB;
  for (int64_t eb = e_beg; eb < e_end; eb += rpp) {
    const int nr = e_end - eb < rpp ? (int)(e_end - eb) : rpp;
    T s[ERB];
#pragma unroll
    for (int r = 0; r < ERB; ++r) s[r] = 0;
    for (int m0 = 0; m0 < D.M; m0 += MCH) {
      const int mc = D.M - m0 < MCH ? D.M - m0 : MCH;
      __syncthreads();
      if (threadIdx.x < nr * mc) {
        const int q = threadIdx.x, r = q / mc, k = q - r * mc;
        const int64_t e = eb + r;
        const int m = m0 + k, t = P.ntype[m];
        if (r == 0) ntp[k] = t;
        const T* W1p = t < EN_LDS_TYPES ? w1t + t * 5 * kMaxH1 : P.en_W1 + t * 4 * D.h1;
        const T* b1p = t < EN_LDS_TYPES ? w1t + t * 5 * kMaxH1 + 4 * D.h1 : P.en_b1 + t * D.h1;
        pair_features_lds<T>((T)(R[3 * e] - P.Rn[3 * m]), (T)(R[3 * e + 1] - P.Rn[3 * m + 1]),
                             (T)(R[3 * e + 2] - P.Rn[3 * m + 2]), W1p, b1p, fw, (T)D.cutn, D,
                             feat + (r * MCH + k) * FEAT);
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int r = 0; r < ERB; ++r) {
          if (r < nr) {
#pragma unroll 1
            for (int k = 0; k < mc; ++k) {
              const T* f = feat + (r * MCH + k) * FEAT;
              if (f[44] == T(0)) continue;
              const int tk = ntp[k];
              const T ne = tk == 0 ? nemb[0] : tk == 1 ? nemb[1] : tk == 2 ? nemb[2] : tk == 3 ? nemb[3]
                                                                                     : P.nuc_emb[tk * D.d + c];
              T g1 = 0, g2 = 0;
#pragma unroll
              for (int j = 0; j < kMaxH2; ++j) g1 += f[4 + j] * w3[j];
#pragma unroll
              for (int j = 0; j < kMaxG; ++j) g2 += f[12 + j] * wenv[j];
              T v = ne + f[0] * wn[0] + f[1] * wn[1] + f[2] * wn[2] + f[3] * wn[3];
              s[r] += g1 * g2 * v;
            }
          }
        }
      }
    }
    T mu[ERB], dv[ERB], var[ERB];
#pragma unroll
    for (int r = 0; r < ERB; ++r) mu[r] = act ? s[r] : T(0);
    block_sums<T, ERB>(mu, red);
#pragma unroll
    for (int r = 0; r < ERB; ++r) {
      mu[r] = mu[r] / T(D.d);
      dv[r] = act ? s[r] - mu[r] : T(0);
      var[r] = dv[r] * dv[r];
    }
    block_sums<T, ERB>(var, red);
    if (act)
#pragma unroll
      for (int r = 0; r < ERB; ++r)
        if (r < nr)
          y_out[(eb + r) * D.d + c] = dv[r] / sqrt(var[r] / T(D.d) + T(kLnEps)) * P.ln_g[c] + P.ln_b[c];
  }
}

// GLU gate: t = u * SiLU(g) with [u | g] the two halves of each row of ug.
template <typename T>
__global__ void k_glu(const T* __restrict__ ug, T* __restrict__ out, int64_t nrows, int d,
                      const int* __restrict__ nrows_dev) {
  if (nrows_dev && *nrows_dev < nrows) nrows = *nrows_dev;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nrows * d;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / d;
    const int c = (int)(i % d);
    const T u = ug[r * 2 * d + c], g = ug[r * 2 * d + d + c];
    out[i] = u * silu_(g);
  }
}

// Envelope basis exp(-sigma_me |r_i - R_m|), row e = (w, i), column m*E + k.
template <typename T>
__global__ void k_env_basis(Net<T> P, const double* __restrict__ R, int64_t nrows, T* __restrict__ out,
                            const int* __restrict__ nrows_dev) {
  const Dims& D = P.D;
  if (nrows_dev && *nrows_dev < nrows) nrows = *nrows_dev;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nrows * D.B;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = q / D.B;
    const int b = (int)(q % D.B), m = b / D.E;
    const double dx = R[3 * e] - P.Rn[3 * m], dy = R[3 * e + 1] - P.Rn[3 * m + 1], dz = R[3 * e + 2] - P.Rn[3 * m + 2];
    const T dist = (T)sqrt(dx * dx + dy * dy + dz * dz);
    out[q] = exp(-P.env_sigma[b] * dist);
  }
}


}  // namespace fire
