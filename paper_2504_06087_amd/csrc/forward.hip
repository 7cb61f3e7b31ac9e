// Forward evaluation of log|psi| for all walkers (Methods, wave-function
// ansatz): neighbour lists, electron-nucleus filters and LayerNorm, GLU, one
// message-passing step, the embedding MLP, envelopes and orbitals, FP64
// Gauss-Jordan inversion with partial pivoting and the signed log-sum-exp
// over determinants.
#include <type_traits>

#include "forward.hpp"
#include "jastrow.hpp"
#include "linalg.hpp"
#include "embed_kernels.hpp"

namespace fire {

// ---------------------------------------------------------------------------
// status helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4: m_i = sum_alpha sum_{j in N^alpha_i} Gamma^alpha(e_ij) *
//           SiLU(a^alpha_i + b^alpha_j + ebar_ij W_e^alpha + b^alpha)
// h1_i = h0_i + m_i.  proj rows hold [a^par | a^anti | b^par | b^anti].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_msg(Net<T> P, const double* __restrict__ R, int64_t nrows,
                                             const int16_t* __restrict__ nidx, const int32_t* __restrict__ ncnt,
                                             const char* __restrict__ state, size_t srec, size_t off_h0,
                                             size_t off_proj, size_t off_m, T* __restrict__ h1_out) {
  const Dims& D = P.D;
  __shared__ T feat[MCH * FEAT];
  __shared__ int jn[MCH];
  const int c = threadIdx.x;
  const bool act = c < D.d;
  const int n = D.n;
  T acc[EPB];
  for (int el = 0; el < EPB; ++el) acc[el] = 0;
  for (int a = 0; a < 2; ++a) {
    T w3[kMaxH2], wenv[kMaxG], we[4], bb = 0;
    if (act) {
      for (int k = 0; k < D.h2; ++k) w3[k] = P.ee_W3[(a * D.h2 + k) * D.d + c];
      for (int k = 0; k < D.G; ++k) wenv[k] = P.ee_Wenv[(a * D.G + k) * D.d + c];
      for (int k = 0; k < 4; ++k) we[k] = P.msg_We[(a * 4 + k) * D.d + c];
      bb = P.msg_b[a * D.d + c];
    }
    for (int el = 0; el < EPB; ++el) {
      int64_t e = (int64_t)blockIdx.x * EPB + el;
      if (e >= nrows) break;
      int64_t w = e / n;
      const char* rec = state + w * srec;
      int i = (int)(e % n);
      int c0 = ncnt[2 * e], c1 = ncnt[2 * e + 1];
      int na = a == 0 ? c0 : c1, base = a == 0 ? 0 : c0;
      const T* proj = (const T*)(rec + off_proj);
      T ai = act ? proj[((int64_t)i * 4 + a) * D.d + c] : T(0);
      const double rx = R[3 * e], ry = R[3 * e + 1], rz = R[3 * e + 2];
      const double* Rw = R + w * n * 3;
      for (int j0 = 0; j0 < na; j0 += MCH) {
        int jc = na - j0 < MCH ? na - j0 : MCH;
        __syncthreads();
        if (threadIdx.x < jc) {
          int j = nidx[e * D.cap_nbr + base + j0 + threadIdx.x];
          jn[threadIdx.x] = j;
          pair_features<T>((T)(rx - Rw[3 * j]), (T)(ry - Rw[3 * j + 1]), (T)(rz - Rw[3 * j + 2]),
                           P.ee_W1 + a * 4 * D.h1, P.ee_b1 + a * D.h1, P.ee_W2 + a * D.h1 * D.h2,
                           P.ee_b2 + a * D.h2, P.ee_sig + a * D.G, (T)D.cut, D, feat + threadIdx.x * FEAT);
        }
        __syncthreads();
        if (act) {
          for (int k = 0; k < jc; ++k) {
            const T* f = feat + k * FEAT;
            if (f[44] == T(0)) continue;
            T g1 = 0, g2 = 0;
            for (int q = 0; q < D.h2; ++q) g1 += f[4 + q] * w3[q];
            for (int q = 0; q < D.G; ++q) g2 += f[12 + q] * wenv[q];
            T bj = proj[((int64_t)jn[k] * 4 + 2 + a) * D.d + c];
            T pre = ai + bj + f[0] * we[0] + f[1] * we[1] + f[2] * we[2] + f[3] * we[3] + bb;
            acc[el] += g1 * g2 * silu_(pre);
          }
        }
      }
    }
  }
  if (!act) return;
  for (int el = 0; el < EPB; ++el) {
    int64_t e = (int64_t)blockIdx.x * EPB + el;
    if (e >= nrows) break;
    int64_t w = e / n;
    int i = (int)(e % n);
    char* rec = (char*)state + w * srec;
    T* m = (T*)(rec + off_m);
    const T* h0 = (const T*)(rec + off_h0);
    m[(int64_t)i * D.d + c] = acc[el];
    h1_out[e * D.d + c] = h0[(int64_t)i * D.d + c] + acc[el];
  }
}

// ---------------------------------------------------------------------------
// a7: in-place Gauss-Jordan inversion with partial (row) pivoting in FP64,
// one workgroup per (walker, determinant) block of one spin: Phi^-1 (stored
// as G = Phi^-T in TI), the sign and log|det| of the block from the same
// elimination.
// ---------------------------------------------------------------------------
// a7 with the block in registers: the N x N block (N <= TG NB) is spread
// over a TG x TG grid of threads (TG = 16, or 32 for blocks past 128 rows),
// thread (ty, tx) holding rows ty + TG a and columns tx + TG b (a, b < NB).  The elimination is gj_block's (partial
// pivoting by row swaps, multipliers by division, the inverse formed in
// place, columns permuted back at the end); per step only the pivot column,
// the pivot row and the row it swaps with pass through LDS, and every
// element update is a register FMA.
template <typename TP, typename TI, int NB, int TG>
__global__ __launch_bounds__(TG * TG) void k_gj_inverse_reg(const char* __restrict__ state_in, char* __restrict__ state_out,
                                                        size_t srec, size_t off_phi, size_t off_inv, size_t off_ds,
                                                        size_t off_dl, Dims D, int spin, int32_t* status) {
  __shared__ double prow[TG * NB], krow[TG * NB], pcol[TG * NB];
  __shared__ double cbest[TG];
  __shared__ int cidx[TG], perm[TG * NB], icol[TG * NB];
  __shared__ int pvt;
  const int N = spin == 0 ? D.nu : D.nd;
  const int w = blockIdx.x / D.K, det = blockIdx.x % D.K;
  const int64_t boff = det * phi_per_det(D) + phi_block_off(D, spin);
  const TP* phi = (const TP*)(state_in + (int64_t)w * srec + off_phi) + boff;
  TI* inv = (TI*)(state_out + (int64_t)w * srec + off_inv) + boff;
  double* dsign = (double*)(state_out + (int64_t)w * srec + off_ds);
  double* dlog = (double*)(state_out + (int64_t)w * srec + off_dl);
  const int tid = threadIdx.x, ty = tid / TG, tx = tid % TG;
  if (N == 0) {
    if (tid == 0) { dsign[det * 2 + spin] = 1.0; dlog[det * 2 + spin] = 0.0; }
    return;
  }
  double A[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = ty + TG * a, j = tx + TG * b;
      A[a][b] = (i < N && j < N) ? (double)phi[(int64_t)i * N + j] : 0.0;
    }
  double lsum = 0.0, sgn = 1.0;
  bool sing = false;
  for (int k = 0; k < N; ++k) {
    const int kb = k / TG, kt = k % TG;
    // column k of my rows (meaningful for tx == kt)
    double ck[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      double c = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) c = b == kb ? A[a][b] : c;
      ck[a] = c;
    }
    if (tx == kt) {
      double best = -1.0;
      int bi = k;
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int i = ty + TG * a;
        const double v = fabs(ck[a]);
        if (i >= k && i < N && v > best) { best = v; bi = i; }
      }
      cbest[ty] = best;
      cidx[ty] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double best = -1.0;
      int bi = k;
      for (int t = 0; t < TG; ++t)
        if (cbest[t] > best || (cbest[t] == best && cidx[t] < bi)) { best = cbest[t]; bi = cidx[t]; }
      pvt = bi;
      perm[k] = bi;
    }
    __syncthreads();
    const int p = pvt;
    const int pb = p / TG, pt = p % TG;
    // the old rows k and p, and column k after the swap
    if (ty == kt || ty == pt) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = tx + TG * b;
        double rk = 0.0, rp = 0.0;
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          rk = a == kb ? A[a][b] : rk;
          rp = a == pb ? A[a][b] : rp;
        }
        if (j < N) {
          if (ty == kt) krow[j] = rk;
          if (ty == pt) prow[j] = rp;
        }
      }
    }
    if (tx == kt) {
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int i = ty + TG * a;
        if (i < N) pcol[i == k ? p : (i == p ? k : i)] = ck[a];
      }
    }
    __syncthreads();
    const double piv = prow[k];
    if (piv == 0.0 || !isfinite(piv)) { sing = true; break; }
    if (tid == 0) {
      lsum += log(fabs(piv));
      sgn *= (piv < 0 ? -1.0 : 1.0) * (p != k ? -1.0 : 1.0);
    }
    double pj[NB], kj[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = tx + TG * b;
      pj[b] = j < N ? prow[j] : 0.0;
      kj[b] = j < N ? krow[j] : 0.0;
    }
    const double ip = 1.0 / piv;
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int i = ty + TG * a;
      const bool isk = i == k, isp = i == p && p != k;
      const double f = (isk || i >= N) ? 0.0 : pcol[i] / piv;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = tx + TG * b;
        const double old = isk ? pj[b] : (isp ? kj[b] : A[a][b]);
        double v;
        if (isk) v = j == k ? ip : old / piv;
        else v = j == k ? -f : old - f * pj[b];
        A[a][b] = v;
      }
    }
    __syncthreads();
  }
  if (sing) {
    if (tid == 0) {
      atomicOr(status + w, FIRE_W_SINGULAR);
      dsign[det * 2 + spin] = 0.0;
      dlog[det * 2 + spin] = -INFINITY;
    }
    return;
  }
  // columns permuted back: after undoing the swaps in reverse order, column
  // c holds column col[c] of A; G[c][l] = (Phi^-1)[l][c] = A[l][col[c]]
  if (tid == 0) {
    for (int c = 0; c < N; ++c) icol[c] = c;   // col[] built in place
    for (int k = N - 1; k >= 0; --k) {
      const int q = perm[k];
      const int t = icol[k];
      icol[k] = icol[q];
      icol[q] = t;
    }
    // invert: icol holds col[]; turn it into its inverse in perm[]
    for (int c = 0; c < N; ++c) perm[icol[c]] = c;
    dsign[det * 2 + spin] = sgn;
    dlog[det * 2 + spin] = lsum;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int l = ty + TG * a, m = tx + TG * b;
      if (l < N && m < N) inv[(int64_t)perm[m] * N + l] = (TI)A[a][b];
    }
}

// log J_cusp = sum_{i<j} u(r_ij) per walker (FP64), one workgroup per walker.
__global__ __launch_bounds__(256) void k_jastrow(const Dims D, const double* __restrict__ R,
                                                 const double* __restrict__ q, char* __restrict__ state,
                                                 StateRec S) {
  __shared__ double red[16];
  const int w = blockIdx.x, n = D.n;
  const double* Rw = R + (int64_t)w * n * 3;
  double acc = 0.0;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t - i * n;
    if (j <= i) continue;
    const double dx = Rw[3 * i] - Rw[3 * j], dy = Rw[3 * i + 1] - Rw[3 * j + 1], dz = Rw[3 * i + 2] - Rw[3 * j + 2];
    acc += jas_u(q, (i < D.nu) == (j < D.nu), sqrt(dx * dx + dy * dy + dz * dz));
  }
  const double tot = block_sum<double>(acc, red);
  if (threadIdx.x == 0) *(double*)(state + (int64_t)w * S.stride + S.jas) = tot;
}

// Signed log-sum-exp over determinants: l* + log|sum_d s_d e^(l_d - l*)|
// (cached); the returned log|psi| adds the cached Jastrow log magnitude, and
// with the MLP Jastrow (jm) the sign takes sign(S_2).
__global__ void k_logsumexp(char* __restrict__ state, size_t srec, size_t off_ds, size_t off_dl, size_t off_lp,
                            size_t off_sp, size_t off_jas, int W, int K, double* sign, double* logpsi,
                            int32_t* status, bool jm, size_t off_jms, bool ja, size_t off_ja_node) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  char* rec = state + (int64_t)w * srec;
  const double* ds = (const double*)(rec + off_ds);
  const double* dl = (const double*)(rec + off_dl);
  double lmax = -INFINITY;
  for (int k = 0; k < K; ++k) {
    double l = dl[2 * k] + dl[2 * k + 1];
    if (ds[2 * k] * ds[2 * k + 1] != 0.0 && l > lmax) lmax = l;
  }
  double tot = 0.0;
  for (int k = 0; k < K; ++k) {
    double sg = ds[2 * k] * ds[2 * k + 1];
    if (sg != 0.0) tot += sg * exp(dl[2 * k] + dl[2 * k + 1] - lmax);
  }
  int32_t st = status[w];
  double lp, sp;
  if (tot == 0.0 || !isfinite(lmax)) {
    st |= FIRE_W_DETSUM_ZERO;
    atomicOr(status + w, FIRE_W_DETSUM_ZERO);
  }
  if (!isfinite(tot)) {
    st |= FIRE_W_NONFINITE;
    atomicOr(status + w, FIRE_W_NONFINITE);
  }
  if (st) {
    lp = NAN;
    sp = 0.0;
  } else {
    lp = lmax + log(fabs(tot));
    sp = tot > 0 ? 1.0 : -1.0;
  }
  *(double*)(rec + off_lp) = lp;
  *(double*)(rec + off_sp) = sp;
  if (logpsi) logpsi[w] = lp + *(const double*)(rec + off_jas);
  double sg = jm && ((const double*)(rec + off_jms))[1] < 0.0 ? -sp : sp;
  if (ja && *(const double*)(rec + off_ja_node) < 0.0) sg = -sg;
  if (sign) sign[w] = sg;
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
WsLayout ws_forward(const fire_handle* h, int W) {
  const Dims& D = h->D;
  WsLayout L{};
  size_t o = 0, ts = h->tsize;
  int64_t rows = (int64_t)W * D.n;
  L.nbr_idx = o; o = align_up(o + rows * D.cap_nbr * sizeof(int16_t));
  L.nbr_cnt = o; o = align_up(o + rows * 2 * sizeof(int32_t));
  L.y = o;       o = align_up(o + rows * D.d * ts);
  L.ug = o;      o = align_up(o + rows * 2 * D.d * ts);
  L.hA = o;      o = align_up(o + rows * D.d * ts);
  L.hB = o;      o = align_up(o + rows * D.d * ts);
  L.basis = o;   o = align_up(o + rows * D.B * ts);
  L.jrow = o;    o = align_up(o + (D.Hj > 0 ? rows * 2 * 8 : 0));
  L.jscr = o;    o = align_up(o + jm_rows_ws(h, rows));
  L.ascr = o;    o = align_up(o + ja_eval_ws(h, W));
  L.total = o;
  return L;
}

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

template <typename T>
hipError_t embed_and_orbitals(const fire_handle* h, const Net<T>& P, int W, const double* R, char* state,
                              char* ws, int32_t* status, hipStream_t s) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  const WsLayout L = ws_forward(h, W);
  const int64_t rows = (int64_t)W * D.n;
  const int blk = D.d <= 64 ? 64 : (D.d + 63) / 64 * 64;
  int16_t* nidx = (int16_t*)(ws + L.nbr_idx);
  int32_t* ncnt = (int32_t*)(ws + L.nbr_cnt);
  T* y = (T*)(ws + L.y);
  T* ug = (T*)(ws + L.ug);
  T* hA = (T*)(ws + L.hA);
  T* hB = (T*)(ws + L.hB);
  T* basis = (T*)(ws + L.basis);
  const int64_t srecT = S.stride / sizeof(T);   // record stride in T elements

  launch_nbr(dim3(W), s, R, W, D.n, D.nu, D.cut * D.cut, D.cap_nbr, nidx, ncnt, status);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_en_embed<T>, dim3((unsigned)((rows + EPB - 1) / EPB)), dim3(blk), 0, s, P, R, rows, y, EPB, (const int*)nullptr);
  CHECK(hipGetLastError());
  // GLU: [u | g] = y [W_v | W_g] + [b_v | b_g];  t = u * SiLU(g);  h0 = t W_o + b_o
  {
    GemmArgs g{};
    g.A = y; g.amap = rows_dense(D.d); g.Bt = (const char*)h->params + h->pl.Wvg_t; g.ldb = D.d;
    g.bias = P.b_vg; g.C = ug; g.cmap = rows_dense(2 * D.d); g.ccol = cols_dense();
    g.M = (int)rows; g.N = 2 * D.d; g.K = D.d; g.act = ACT_NONE;
    CHECK(gemm_site(h, SITE_EMB, g, s));
  }
  hipLaunchKernelGGL(k_glu<T>, dim3((unsigned)((rows * D.d + 255) / 256)), dim3(256), 0, s, ug, y, rows, D.d, (const int*)nullptr);
  CHECK(hipGetLastError());
  {
    GemmArgs g{};
    g.A = y; g.amap = rows_dense(D.d); g.Bt = (const char*)h->params + h->pl.Wo_t; g.ldb = D.d;
    g.bias = P.b_o; g.C = state + S.h0; g.cmap = RowMap{D.n, srecT, D.d}; g.ccol = cols_dense();
    g.M = (int)rows; g.N = D.d; g.K = D.d;
    CHECK(gemm_site(h, SITE_EMB, g, s));
  }
  // node projections [a^par | a^anti | b^par | b^anti] = h0 W_proj
  {
    GemmArgs g{};
    g.A = state + S.h0; g.amap = RowMap{D.n, srecT, D.d}; g.Bt = (const char*)h->params + h->pl.Wproj_t;
    g.ldb = D.d; g.C = state + S.proj; g.cmap = RowMap{D.n, srecT, 4 * D.d}; g.ccol = cols_dense();
    g.M = (int)rows; g.N = 4 * D.d; g.K = D.d;
    CHECK(gemm_site(h, SITE_EMB, g, s));
  }
  hipLaunchKernelGGL(k_msg<T>, dim3((unsigned)((rows + EPB - 1) / EPB)), dim3(blk), 0, s, P, R, rows, nidx, ncnt,
                     state, S.stride, S.h0, S.proj, S.m, hA);
  CHECK(hipGetLastError());
  // MLP
  T* hin = hA;
  T* hout = hB;
  for (int k = 0; k < D.L; ++k) {
    GemmArgs g{};
    g.A = hin; g.amap = rows_dense(D.d);
    g.Bt = (const char*)h->params + h->pl.mlp_t + (size_t)k * D.d * D.d * h->gsize; g.ldb = D.d;
    g.bias = P.mlp_b + (int64_t)k * D.d; g.C = hout; g.cmap = rows_dense(D.d); g.ccol = cols_dense();
    g.M = (int)rows; g.N = D.d; g.K = D.d; g.act = ACT_SILU;
    CHECK(gemm_site(h, SITE_EMB, g, s));
    T* t = hin; hin = hout; hout = t;
  }
  // MLP Jastrow readouts of the final embeddings and their sums
  if (D.Hj > 0) {
    double* jrow = (double*)(ws + L.jrow);
    CHECK(jm_rows<T>(h, P, hin, (int)rows, nullptr, ws + L.jscr, jrow, s));
    CHECK(jm_store(h, W, jrow, state, s));
  }
  // attention Jastrow: projections, softmax sums, registers and readouts
  if (D.Ra > 0) CHECK(ja_eval<T>(h, P, W, hin, state, ws + L.ascr, s));
  // envelopes and orbitals per spin block
  hipLaunchKernelGGL(k_env_basis<T>, dim3((unsigned)((rows * D.B + 255) / 256)), dim3(256), 0, s, P, R, rows, basis, (const int*)nullptr);
  CHECK(hipGetLastError());
  for (int sp = 0; sp < 2; ++sp) {
    const int N = D.nsig(sp), e0 = sp == 0 ? 0 : D.nu;
    if (N == 0) continue;
    const int64_t mrows = (int64_t)W * N;
    // env[w][det][sp][i][l] = sum_b basis[w][e0+i][b] pi[(det,l)][b]   (cached in state)
    const RowMap smap{N, srecT, N};
    const ColMap scol{N, phi_per_det(D)};
    GemmArgs g{};
    g.A = basis + (int64_t)e0 * D.B; g.amap = RowMap{N, (int64_t)D.n * D.B, D.B};
    g.Bt = (const char*)h->params + (sp == 0 ? h->pl.pi0 : h->pl.pi1); g.ldb = D.B;
    g.C = state + S.env + phi_block_off(D, sp) * sizeof(T); g.cmap = smap; g.ccol = scol;
    g.M = (int)mrows; g.N = D.K * N; g.K = D.B;
    CHECK(gemm_site(h, SITE_ORB, g, s));
    // Phi[w][det][sp][i][l] = (h_i . W[:, (det,l)]) * env
    GemmArgs o{};
    o.A = hin + (int64_t)e0 * D.d; o.amap = RowMap{N, (int64_t)D.n * D.d, D.d};
    o.Bt = (const char*)h->params + (sp == 0 ? h->pl.orb_t0 : h->pl.orb_t1); o.ldb = D.d;
    o.aux = state + S.env + phi_block_off(D, sp) * sizeof(T); o.xmap = smap; o.xcol = scol;
    o.C = state + S.phi + phi_block_off(D, sp) * sizeof(T);
    o.cmap = smap;
    o.ccol = scol;
    o.M = (int)mrows; o.N = D.K * N; o.K = D.d;
    CHECK(gemm_site(h, SITE_ORB, o, s));
  }
  return hipSuccess;
}

template <typename T>
hipError_t refresh_dets(const fire_handle* h, int W, const double* R, char* state, double* sign, double* logpsi,
                        int32_t* status, hipStream_t s) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  for (int sp = 0; sp < 2; ++sp) {
    const int N = D.nsig(sp);
    // up to 128 rows: a 16 x 16 thread grid (up to 64 values per thread);
    // up to 192: 32 x 32 (up to 36 values per thread: a 1024-thread
    // workgroup holds 128 registers per lane)
    const int nb = N <= 128 ? (N + 15) / 16 : (N + 31) / 32;
    const dim3 g((unsigned)(W * D.K));
    auto go = [&](auto nbc, auto tgc) {
      constexpr int NBC = decltype(nbc)::value, TGC = decltype(tgc)::value;
      if (h->isize == 8)
        hipLaunchKernelGGL((k_gj_inverse_reg<T, double, NBC, TGC>), g, dim3(TGC * TGC), 0, s, state, state, S.stride,
                           S.phi, S.inv, S.dsign, S.dlog, D, sp, status);
      else
        hipLaunchKernelGGL((k_gj_inverse_reg<T, float, NBC, TGC>), g, dim3(TGC * TGC), 0, s, state, state, S.stride,
                           S.phi, S.inv, S.dsign, S.dlog, D, sp, status);
    };
    using I16 = std::integral_constant<int, 16>;
    using I32 = std::integral_constant<int, 32>;
    if (N <= 128) {
      switch (nb) {
        case 0: case 1: go(std::integral_constant<int, 1>{}, I16{}); break;
        case 2: go(std::integral_constant<int, 2>{}, I16{}); break;
        case 3: go(std::integral_constant<int, 3>{}, I16{}); break;
        case 4: go(std::integral_constant<int, 4>{}, I16{}); break;
        case 5: go(std::integral_constant<int, 5>{}, I16{}); break;
        case 6: go(std::integral_constant<int, 6>{}, I16{}); break;
        case 7: go(std::integral_constant<int, 7>{}, I16{}); break;
        default: go(std::integral_constant<int, 8>{}, I16{}); break;
      }
    } else {
      if (nb <= 5) go(std::integral_constant<int, 5>{}, I32{});
      else go(std::integral_constant<int, 6>{}, I32{});
    }
    CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_jastrow, dim3(W), dim3(256), 0, s, D, R, (const double*)((const char*)h->params + h->pl.jas),
                     state, S);
  CHECK(hipGetLastError());
  CHECK(jm_total(h, W, state, status, s));
  CHECK(ja_total(h, W, state, status, s));
  hipLaunchKernelGGL(k_logsumexp, dim3((W + 127) / 128), dim3(128), 0, s, state, S.stride, S.dsign, S.dlog, S.lpsi,
                     S.spsi, S.jas, W, D.K, sign, logpsi, status, D.Hj > 0, S.jms, D.Ra > 0,
                     S.jat + (size_t)(2 * D.Ra + D.NV() + 1) * 8);
  return hipGetLastError();
}

template <typename T>
hipError_t forward(const fire_handle* h, int W, const double* R, char* state, char* ws, double* sign,
                   double* logpsi, int32_t* status, hipStream_t s) {
  Net<T> P = make_net<T>(h);
  CHECK(embed_and_orbitals<T>(h, P, W, R, state, ws, status, s));
  return refresh_dets<T>(h, W, R, state, sign, logpsi, status, s);
}

template hipError_t forward<double>(const fire_handle*, int, const double*, char*, char*, double*, double*,
                                    int32_t*, hipStream_t);
template hipError_t forward<float>(const fire_handle*, int, const double*, char*, char*, double*, double*,
                                   int32_t*, hipStream_t);
template hipError_t refresh_dets<double>(const fire_handle*, int, const double*, char*, double*, double*, int32_t*,
                                         hipStream_t);
template hipError_t refresh_dets<float>(const fire_handle*, int, const double*, char*, double*, double*, int32_t*,
                                        hipStream_t);
template hipError_t embed_and_orbitals<double>(const fire_handle*, const Net<double>&, int, const double*, char*,
                                               char*, int32_t*, hipStream_t);
template hipError_t embed_and_orbitals<float>(const fire_handle*, const Net<float>&, int, const double*, char*,
                                              char*, int32_t*, hipStream_t);

}  // namespace fire
