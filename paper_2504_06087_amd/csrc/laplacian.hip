// Local energy by the sparse forward Laplacian (Methods, efficient
// Laplacian; Hamiltonian and local energy).
//
// Electron i's embedding depends only on r_n for n in S_i = {i} u N_i, so its
// Jacobian has 3|S_i| non-zero rows.  Every stage carries, per electron, the
// value, those tangent rows and one Laplacian row:
//   h0_i:   3 tangents (w.r.t. r_i) + Laplacian           [5-row blocks]
//   h1_i:   3 (self) + 3 per neighbour + Laplacian        [jet blocks]
//   MLP, orbital projections: GEMMs over the stacked jet rows (spin-major)
// and the log-determinant terms use M_{ik,nx} = sum_l d_{nx}Phi_il Phi^-1_lk
// only for i, k in T_n = {n} u N_n (eqs. forward_lap_det_M and
// logdet_lowrank):  d_{nx} log det = sum_i M_ii,  Lap log det =
//   sum_il LapPhi_il Phi^-1_li - sum_{n,x} sum_{i,k in T_n} M_ik M_ki.
#include "laplacian.hpp"
#include "jastrow.hpp"

#include "embed_kernels.hpp"
#include "jets.hpp"

#include <mutex>

namespace fire {

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

static int jet_rows_max(const Dims& D) { return 3 * (1 + D.cap_nbr) + 1; }

LapLayout lap_layout(const fire_handle* h, int W) {
  const Dims& D = h->D;
  LapLayout L{};
  // walkers per chunk: bounded by a workspace budget for the jet tensors
  const size_t ts = h->tsize;
  const int nmax = D.nu > D.nd ? D.nu : D.nd;
  const size_t per_walker = (size_t)D.n * jet_rows_max(D) * ((size_t)2 * D.d + (size_t)D.K * nmax) * ts +
                            (size_t)D.n * 5 * ((size_t)8 * D.d + D.B + (size_t)D.K * nmax) * ts +
                            (D.Hj > 0 ? (size_t)D.n * jet_rows_max(D) * (2 * D.Hj * ts + 16) +
                                            (size_t)D.n * (2 * D.Hj * ts + 24)
                                      : 0) +
                            (D.Ra > 0 ? (size_t)D.n * jet_rows_max(D) * D.NA() * ts +
                                            (size_t)(3 * D.n + 2) * ((size_t)(D.NV() + 2 * D.Ha) * ts + 16) +
                                            (size_t)4 * D.n * D.Ra * 8 + (size_t)D.n * 24
                                      : 0);
  const size_t budget = h->lap_budget;
  int wc = (int)(budget / (per_walker > 0 ? per_walker : 1));
  if (wc < 1) wc = 1;
  if (wc > 512) wc = 512;
  if (wc > W) wc = W;
  L.Wc = wc;
  const int64_t Wl = wc, n = D.n;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  L.nidx = take(Wl * n * D.cap_nbr * 2);
  L.ncnt = take(Wl * n * 2 * 4);
  L.joff = take(Wl * n * 4);
  L.jtot = take(2 * (Wl + 1) * 4 + 64);
  L.yj = take(Wl * n * 5 * D.d * ts);
  L.ugj = take(Wl * n * 5 * 2 * D.d * ts);
  L.h0j = take(Wl * n * 5 * D.d * ts);
  L.projj = take(Wl * n * 5 * 4 * D.d * ts);
  L.hval = take(Wl * n * D.d * ts);
  L.zval = take(Wl * n * D.d * ts);
  L.basisj = take(Wl * n * 5 * D.B * ts);
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s) > 0 ? D.nsig(s) : 1;
    L.rowcap[s] = Wl * (D.nsig(s) > 0 ? D.nsig(s) : 1) * jet_rows_max(D);
    L.jetA[s] = take(L.rowcap[s] * D.d * ts);
    L.jetB[s] = take(L.rowcap[s] * D.d * ts);
    L.envj[s] = take(Wl * N * 5 * D.K * N * ts);
    L.oval[s] = take(Wl * N * D.K * N * ts);
    L.dphi[s] = take(L.rowcap[s] * D.K * N * ts);
  }
  L.gd = take(Wl * D.K * n * 3 * 8);
  L.hd = take(Wl * D.K * n * 8);
  L.tcap = D.cap_nbr + 1;
  L.memb = take(Wl * n * 2 * L.tcap * 4);
  L.mslot = take(Wl * n * 2 * L.tcap * 4);
  L.mcnt = take(Wl * n * 2 * 4);
  if (D.Hj > 0) {
    L.jzv = take(2 * Wl * n * D.Hj * ts);
    for (int s = 0; s < 2; ++s) {
      L.jjx[s] = take(L.rowcap[s] * D.Hj * ts);
      L.jjy[s] = take(L.rowcap[s] * D.Hj * ts);
      L.jjt[s] = take(L.rowcap[s] * 2 * 8);
    }
  }
  if (D.Hj > 0 || D.Ra > 0) {
    L.jgJ = take(Wl * n * 3 * 8);
    L.jlap = take(Wl * 8);
  }
  if (D.Ra > 0) L.jak = take(ja_kin_ws(h, wc, L.rowcap));
  L.total = o;
  return L;
}

// ---------------------------------------------------------------------------
// jet-row offsets: electron (w, i) of spin s owns rows [joff, joff + rows_i)
// of its spin's segment, rows_i = 3 (1 + |N_i|) + 1, walkers in order.
// jtot[s] = rows of segment s.  One workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_jet_offsets(int Wc, int n, int nu, const int32_t* __restrict__ ncnt,
                                                      int* __restrict__ joff, int* __restrict__ jtot) {
  __shared__ int part[2][1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (Wc + nt - 1) / nt;
  const int b = t * per, e = b + per < Wc ? b + per : Wc;
  int s0 = 0, s1 = 0;
  for (int w = b; w < e; ++w)
    for (int i = 0; i < n; ++i) {
      int r = 3 * (1 + ncnt[2 * (w * n + i)] + ncnt[2 * (w * n + i) + 1]) + 1;
      if (i < nu) s0 += r; else s1 += r;
    }
  part[0][t] = s0;
  part[1][t] = s1;
  __syncthreads();
  if (t < 2) {
    int acc = 0;
    for (int k = 0; k < nt; ++k) { int v = part[t][k]; part[t][k] = acc; acc += v; }
    jtot[t] = acc;
  }
  __syncthreads();
  int a0 = part[0][t], a1 = part[1][t];
  for (int w = b; w < e; ++w)
    for (int i = 0; i < n; ++i) {
      int r = 3 * (1 + ncnt[2 * (w * n + i)] + ncnt[2 * (w * n + i) + 1]) + 1;
      if (i < nu) { joff[w * n + i] = a0; a0 += r; }
      else { joff[w * n + i] = a1; a1 += r; }
    }
}

// ---------------------------------------------------------------------------
// h0 jets: s_i and LayerNorm as 3-jets in r_i.  Output rows per electron:
// [value, d/dx, d/dy, d/dz, Laplacian] of y = LN(s).
// ---------------------------------------------------------------------------
constexpr int JCH = 32;   // pairs per LDS chunk

template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void k_en_embed_jet(Net<T> P, const double* __restrict__ R,
                                                                            int64_t nrows, T* __restrict__ yj) {
  const Dims& D = P.D;
  __shared__ T feat[JCH * JFEAT];
  __shared__ T red[16];
  // filter weights staged in LDS as in k_en_embed (shared part, then layer 1
  // of the first EN_LDS_TYPES nucleus types)
  __shared__ T fw[FW_SIZE];
  __shared__ T w1t[EN_LDS_TYPES * 5 * kMaxH1];
  const int c = threadIdx.x;
  const bool act = c < D.d;
  stage_filter<T>(nullptr, nullptr, P.en_W2, P.en_b2, P.en_sig, D, fw, c, blockDim.x);
  {
    const int ntl = D.NT < EN_LDS_TYPES ? D.NT : EN_LDS_TYPES;
    for (int q = c; q < ntl * 5 * D.h1; q += blockDim.x) {
      const int t = q / (5 * D.h1), i = q - t * 5 * D.h1;
      w1t[t * 5 * kMaxH1 + i] = i < 4 * D.h1 ? P.en_W1[t * 4 * D.h1 + i] : P.en_b1[t * D.h1 + i - 4 * D.h1];
    }
  }
  T w3[kMaxH2], wenv[kMaxG], wn[4];
  if (act) {
    for (int k = 0; k < D.h2; ++k) w3[k] = P.en_W3[k * D.d + c];
    for (int k = 0; k < D.G; ++k) wenv[k] = P.en_Wenv[k * D.d + c];
    for (int k = 0; k < 4; ++k) wn[k] = P.en_Wn[k * D.d + c];
  }
  for (int el = 0; el < 4; ++el) {
    const int64_t e = (int64_t)blockIdx.x * 4 + el;
    if (e >= nrows) break;
    const double rx = R[3 * e], ry = R[3 * e + 1], rz = R[3 * e + 2];
    J3<T> s = jconst(T(0));
    for (int m0 = 0; m0 < D.M; m0 += JCH) {
      const int mc = D.M - m0 < JCH ? D.M - m0 : JCH;
      __syncthreads();
      if (threadIdx.x < mc) {
        const int m = m0 + threadIdx.x, t = P.ntype[m];
        const T* W1p = t < EN_LDS_TYPES ? w1t + t * 5 * kMaxH1 : P.en_W1 + t * 4 * D.h1;
        const T* b1p = t < EN_LDS_TYPES ? w1t + t * 5 * kMaxH1 + 4 * D.h1 : P.en_b1 + t * D.h1;
        pair_feature_jets<T>((T)(rx - P.Rn[3 * m]), (T)(ry - P.Rn[3 * m + 1]), (T)(rz - P.Rn[3 * m + 2]), W1p, b1p,
                             fw + FW_W2T, 1, kMaxH1, fw + FW_B2, fw + FW_SIG, (T)D.cutn, D,
                             feat + threadIdx.x * JFEAT);
      }
      __syncthreads();
      if (act)
        for (int k = 0; k < mc; ++k) {
          const T* f = feat + k * JFEAT;
          if (f[44 * 5] == T(0)) continue;
          J3<T> g1 = jconst(T(0)), g2 = jconst(T(0)), v = jconst(P.nuc_emb[P.ntype[m0 + k] * D.d + c]);
          for (int j = 0; j < D.h2; ++j) jaxpy(g1, w3[j], jload(f + 5 * (4 + j)));
          for (int j = 0; j < D.G; ++j) jaxpy(g2, wenv[j], jload(f + 5 * (12 + j)));
          for (int j = 0; j < 4; ++j) jaxpy(v, wn[j], jload(f + 5 * j));
          s = jadd(s, jmul(jmul(g1, g2), v));
        }
    }
    // LayerNorm on jets: mu, d = s - mu, var = mean d^2, y = g * d * (var+eps)^-1/2 + b
    const T inv_d = T(1) / T(D.d);
    J3<T> mu;
    mu.v = block_sum<T>(act ? s.v : T(0), red) * inv_d;
    for (int k = 0; k < 3; ++k) mu.g[k] = block_sum<T>(act ? s.g[k] : T(0), red) * inv_d;
    mu.l = block_sum<T>(act ? s.l : T(0), red) * inv_d;
    J3<T> dv = act ? J3<T>{s.v - mu.v, {s.g[0] - mu.g[0], s.g[1] - mu.g[1], s.g[2] - mu.g[2]}, s.l - mu.l}
                   : jconst(T(0));
    J3<T> var;
    var.v = block_sum<T>(dv.v * dv.v, red) * inv_d;
    for (int k = 0; k < 3; ++k) var.g[k] = T(2) * block_sum<T>(dv.v * dv.g[k], red) * inv_d;
    var.l = T(2) * block_sum<T>(dv.v * dv.l + dv.g[0] * dv.g[0] + dv.g[1] * dv.g[1] + dv.g[2] * dv.g[2], red) * inv_d;
    const T ve = var.v + T(kLnEps);
    const T rs = T(1) / sqrt(ve);
    J3<T> rj = jchain(var, rs, T(-0.5) * rs / ve, T(0.75) * rs / (ve * ve));
    if (act) {
      J3<T> y = jmul(dv, rj);
      const T gam = P.ln_g[c];
      T* o = yj + e * 5 * D.d;
      o[0 * D.d + c] = gam * y.v + P.ln_b[c];
      o[1 * D.d + c] = gam * y.g[0];
      o[2 * D.d + c] = gam * y.g[1];
      o[3 * D.d + c] = gam * y.g[2];
      o[4 * D.d + c] = gam * y.l;
    }
  }
}

// GLU on 5-row jet blocks: t = u * SiLU(g)
template <typename T>
__global__ void k_glu_jet(const T* __restrict__ ugj, T* __restrict__ tj, int64_t nel, int d) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nel * d) return;
  const int64_t e = q / d;
  const int c = (int)(q % d);
  const T* b = ugj + e * 5 * 2 * d;
  J3<T> u{b[c], {b[2 * d + c], b[4 * d + c], b[6 * d + c]}, b[8 * d + c]};
  J3<T> g{b[d + c], {b[3 * d + c], b[5 * d + c], b[7 * d + c]}, b[9 * d + c]};
  J3<T> t = jmul(u, jsilu(g));
  T* o = tj + e * 5 * d;
  o[c] = t.v; o[d + c] = t.g[0]; o[2 * d + c] = t.g[1]; o[3 * d + c] = t.g[2]; o[4 * d + c] = t.l;
}

// ---------------------------------------------------------------------------
// message jets.  For the edge (i, j) the jet has 6 directions (r_i, r_j); the
// filter and rescaled features depend on d = r_i - r_j only, so their
// gradients are +g (r_i) and -g (r_j) and their Laplacian doubles.
// Output: h1 values and the jet block of electron i (self rows, 3 rows per
// neighbour slot in list order, Laplacian row).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void k_msg_jet(Net<T> P, const double* __restrict__ R,
                                                                       int64_t nrows,
                                                 const int16_t* __restrict__ nidx, const int32_t* __restrict__ ncnt,
                                                 const int* __restrict__ joff, const T* __restrict__ h0j,
                                                 const T* __restrict__ projj, T* __restrict__ hval, T* jet0,
                                                 T* jet1) {
  const Dims& D = P.D;
  __shared__ T feat[JCH * JFEAT];
  __shared__ int jn[JCH];
  __shared__ T fw[2 * FW_SIZE];   // filter weights of both pair classes
  const int c = threadIdx.x;
  const bool act = c < D.d;
  const int n = D.n, d = D.d;
  const int64_t e = blockIdx.x;
  if (e >= nrows) return;
  for (int a = 0; a < 2; ++a)
    stage_filter<T>(P.ee_W1 + a * 4 * D.h1, P.ee_b1 + a * D.h1, P.ee_W2 + a * D.h1 * D.h2, P.ee_b2 + a * D.h2,
                    P.ee_sig + a * D.G, D, fw + a * FW_SIZE, c, blockDim.x);
  const int64_t w = e / n;
  const int i = (int)(e % n);
  const int si = i < D.nu ? 0 : 1;
  T* jet = si == 0 ? jet0 : jet1;
  const int64_t base = joff[e];
  const int c0 = ncnt[2 * e], c1 = ncnt[2 * e + 1];
  const int cnt = c0 + c1;
  const int64_t lrow = base + 3 * (1 + cnt);
  const double rx = R[3 * e], ry = R[3 * e + 1], rz = R[3 * e + 2];
  const double* Rw = R + w * n * 3;
  T mv = 0, mg[3] = {0, 0, 0}, ml = 0;
  for (int a = 0; a < 2; ++a) {
    const int na = a == 0 ? c0 : c1, sbase = a == 0 ? 0 : c0;
    T w3[kMaxH2], wenv[kMaxG], we[4], bb = 0;
    J3<T> ai = jconst(T(0));
    if (act) {
      for (int k = 0; k < D.h2; ++k) w3[k] = P.ee_W3[(a * D.h2 + k) * d + c];
      for (int k = 0; k < D.G; ++k) wenv[k] = P.ee_Wenv[(a * D.G + k) * d + c];
      for (int k = 0; k < 4; ++k) we[k] = P.msg_We[(a * 4 + k) * d + c];
      bb = P.msg_b[a * d + c];
      const T* pi = projj + e * 5 * 4 * d + a * d + c;
      ai = J3<T>{pi[0], {pi[4 * d], pi[8 * d], pi[12 * d]}, pi[16 * d]};
    }
    for (int j0 = 0; j0 < na; j0 += JCH) {
      const int jc = na - j0 < JCH ? na - j0 : JCH;
      __syncthreads();
      if (threadIdx.x < jc) {
        const int j = nidx[e * D.cap_nbr + sbase + j0 + threadIdx.x];
        jn[threadIdx.x] = j;
        const T* fa = fw + a * FW_SIZE;
        pair_feature_jets<T>((T)(rx - Rw[3 * j]), (T)(ry - Rw[3 * j + 1]), (T)(rz - Rw[3 * j + 2]), fa + FW_W1,
                             fa + FW_B1, fa + FW_W2T, 1, kMaxH1, fa + FW_B2, fa + FW_SIG, (T)D.cut, D,
                             feat + threadIdx.x * JFEAT);
      }
      __syncthreads();
      if (!act) continue;
      for (int k = 0; k < jc; ++k) {
        const T* f = feat + k * JFEAT;
        const int slot = sbase + j0 + k;
        T* trow = jet + (base + 3 + 3 * slot) * d + c;
        if (f[44 * 5] == T(0)) {
          trow[0] = T(0); trow[d] = T(0); trow[2 * d] = T(0);
          continue;
        }
        J3<T> g1 = jconst(T(0)), g2 = jconst(T(0)), ef = jconst(bb);
        for (int q = 0; q < D.h2; ++q) jaxpy(g1, w3[q], jload(f + 5 * (4 + q)));
        for (int q = 0; q < D.G; ++q) jaxpy(g2, wenv[q], jload(f + 5 * (12 + q)));
        for (int q = 0; q < 4; ++q) jaxpy(ef, we[q], jload(f + 5 * q));
        const J3<T> gam = jmul(g1, g2);
        const T* pj = projj + (w * n + jn[k]) * 5 * 4 * d + (2 + a) * d + c;
        // x over 6 directions: gi = grad a_i + grad ef, gj = grad b_j - grad ef
        const T xv = ai.v + pj[0] + ef.v;
        T xgi[3], xgj[3];
        for (int q = 0; q < 3; ++q) { xgi[q] = ai.g[q] + ef.g[q]; xgj[q] = pj[4 * d * (q + 1)] - ef.g[q]; }
        const T xl = ai.l + pj[16 * d] + T(2) * ef.l;
        T sf, s1, s2;
        silu3(xv, sf, s1, s2);
        const T sq = xgi[0] * xgi[0] + xgi[1] * xgi[1] + xgi[2] * xgi[2] + xgj[0] * xgj[0] + xgj[1] * xgj[1] +
                     xgj[2] * xgj[2];
        const T sl = s1 * xl + s2 * sq;
        // edge = gam * s  (gam's 6-dir gradient: (+g, -g), Laplacian 2 l)
        mv += gam.v * sf;
        T dots = 0;
        for (int q = 0; q < 3; ++q) {
          const T sgi = s1 * xgi[q], sgj = s1 * xgj[q];
          mg[q] += gam.v * sgi + sf * gam.g[q];
          trow[q * d] = gam.v * sgj - sf * gam.g[q];
          dots += gam.g[q] * sgi - gam.g[q] * sgj;
        }
        ml += gam.v * sl + sf * T(2) * gam.l + T(2) * dots;
      }
    }
  }
  if (!act) return;
  const T* h0 = h0j + e * 5 * d + c;
  hval[e * d + c] = h0[0] + mv;
  T* srow = jet + base * d + c;
  for (int q = 0; q < 3; ++q) srow[q * d] = h0[(q + 1) * d] + mg[q];
  jet[lrow * d + c] = h0[4 * d] + ml;
}

// SiLU on jets, in place over one electron's rows: tangent rows t -> f'(z) t,
// Laplacian row l -> f'(z) l + f''(z) sum_t t^2, value -> f(z).
template <typename T>
__global__ __launch_bounds__(256) void k_jet_act(const Dims D, int64_t nrows, const int32_t* __restrict__ ncnt,
                                                 const int* __restrict__ joff, const T* __restrict__ zval,
                                                 T* __restrict__ hval, const T* __restrict__ jin0,
                                                 const T* __restrict__ jin1, T* jout0, T* jout1) {
  const int64_t e = blockIdx.x;
  const int c = threadIdx.x;
  if (e >= nrows || c >= D.d) return;
  const int i = (int)(e % D.n);
  const T* jin = i < D.nu ? jin0 : jin1;
  T* jout = i < D.nu ? jout0 : jout1;
  const int nt = 3 * (1 + ncnt[2 * e] + ncnt[2 * e + 1]);
  const int64_t base = joff[e];
  T f, f1, f2;
  silu3(zval[e * D.d + c], f, f1, f2);
  hval[e * D.d + c] = f;
  T sq = 0;
  for (int r = 0; r < nt; ++r) {
    const T t = jin[(base + r) * D.d + c];
    sq += t * t;
    jout[(base + r) * D.d + c] = f1 * t;
  }
  jout[(base + nt) * D.d + c] = f1 * jin[(base + nt) * D.d + c] + f2 * sq;
}

// envelope basis jets exp(-sigma |r_i - R_m|): rows [v, gx, gy, gz, lap] per electron
template <typename T>
__global__ void k_basis_jet(Net<T> P, const double* __restrict__ R, int64_t nrows, T* __restrict__ out) {
  const Dims& D = P.D;
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nrows * D.B) return;
  const int64_t e = q / D.B;
  const int b = (int)(q % D.B), m = b / D.E;
  const double dx = R[3 * e] - P.Rn[3 * m], dy = R[3 * e + 1] - P.Rn[3 * m + 1], dz = R[3 * e + 2] - P.Rn[3 * m + 2];
  const double rho = sqrt(dx * dx + dy * dy + dz * dz);
  const T sg = P.env_sigma[b];
  const T ex = exp(-sg * (T)rho);
  T* o = out + e * 5 * D.B + b;
  const T ir = rho > 0 ? (T)(1.0 / rho) : T(0);
  o[0] = ex;
  o[D.B] = -sg * ex * (T)dx * ir;
  o[2 * D.B] = -sg * ex * (T)dy * ir;
  o[3 * D.B] = -sg * ex * (T)dz * ir;
  o[4 * D.B] = ex * (sg * sg - T(2) * sg * ir);
}

// Phi jets from projection jets and envelope jets (one spin block), in place:
//   d_n Phi_il = d_n o_il env_il + [n = i] o_il d env_il
//   Lap Phi_il = Lap o_il env_il + 2 grad_i o_il . grad env_il + o_il Lap env_il
template <typename T>
__global__ void k_phi_jet(const Dims D, int s, int Wc, const int32_t* __restrict__ ncnt, const int* __restrict__ joff,
                          const T* __restrict__ oval, const T* __restrict__ envj, T* __restrict__ dphi) {
  const int N = D.nsig(s), KN = D.K * N, e0 = s == 0 ? 0 : D.nu;
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)Wc * N * KN) return;
  const int64_t r = q / KN;                 // (w, iloc)
  const int col = (int)(q % KN);
  const int64_t w = r / N;
  const int iloc = (int)(r % N);
  const int64_t e = w * D.n + e0 + iloc;
  const int nt = 3 * (1 + ncnt[2 * e] + ncnt[2 * e + 1]);
  const int64_t base = joff[e];
  const T o = oval[r * KN + col];
  const T* ej = envj + r * 5 * KN + col;
  const T ev = ej[0], eg0 = ej[KN], eg1 = ej[2 * KN], eg2 = ej[3 * KN], el = ej[4 * KN];
  T* dp = dphi + base * KN + col;
  const T t0 = dp[0], t1 = dp[KN], t2 = dp[2 * KN];
  dp[(int64_t)nt * KN] = dp[(int64_t)nt * KN] * ev + T(2) * (t0 * eg0 + t1 * eg1 + t2 * eg2) + o * el;
  dp[0] = t0 * ev + o * eg0;
  dp[KN] = t1 * ev + o * eg1;
  dp[2 * KN] = t2 * ev + o * eg2;
  for (int k = 3; k < nt; ++k) dp[(int64_t)k * KN] *= ev;
}

// ---------------------------------------------------------------------------
// log-det contraction per (walker, electron n, determinant):
//   grad_{n,x} l_d = sum_{i in T_n} M_ii,   hess_n = sum_x sum_{i,k in T_n} M_ik M_ki
// with M_ik = sum_l d_{n,x}Phi_il G_kl (G = Phi^-T), per spin block, plus the
// Laplacian row term sum_l LapPhi_nl G_nl of electron n itself.
// ---------------------------------------------------------------------------
typedef double d4v_ __attribute__((ext_vector_type(4)));

// Members of T_n = {n} u N_n per spin block, with the slot of n in each
// member's own tangent list (0 for n itself).  One wave per (walker, n);
// members whose list does not hold n (cannot happen for a symmetric
// neighbour relation) are dropped.
__global__ __launch_bounds__(256) void k_lap_members(const Dims D, int Wc, const int16_t* __restrict__ nidx,
                                                     const int32_t* __restrict__ ncnt, int tcap,
                                                     int* __restrict__ memb, int* __restrict__ mslot,
                                                     int* __restrict__ mcnt) {
  const int lane = threadIdx.x & 63;
  const int64_t en = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int n = D.n;
  if (en >= (int64_t)Wc * n) return;
  const int wl = (int)(en / n), nn = (int)(en % n);
  const int cn = ncnt[2 * en] + ncnt[2 * en + 1];
  int c[2] = {0, 0};
  for (int t0 = 0; t0 <= cn; t0 += 64) {
    const int t = t0 + lane;
    int i = -1, sl = -1;
    if (t <= cn) {
      i = t == 0 ? nn : nidx[en * D.cap_nbr + t - 1];
      if (i == nn) {
        sl = 0;
      } else {
        const int64_t ei = (int64_t)wl * n + i;
        const int ci = ncnt[2 * ei] + ncnt[2 * ei + 1];
        for (int p = 0; p < ci; ++p)
          if (nidx[ei * D.cap_nbr + p] == nn) { sl = 1 + p; break; }
      }
    }
    const bool ok = sl >= 0;
    const bool up = i >= 0 && i < D.nu;
    const uint64_t m0 = __ballot(ok && up), m1 = __ballot(ok && !up);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (ok) {
      const int sp = up ? 0 : 1;
      const int pos = c[sp] + __popcll((sp == 0 ? m0 : m1) & below);
      memb[(en * 2 + sp) * tcap + pos] = i;
      mslot[(en * 2 + sp) * tcap + pos] = sl;
    }
    c[0] += __popcll(m0);
    c[1] += __popcll(m1);
  }
  if (lane == 0) {
    mcnt[2 * en] = c[0];
    mcnt[2 * en + 1] = c[1];
  }
}

// log-det contraction per (walker, electron n, determinant), one wave each
// (Methods, efficient Laplacian, eqs. forward_lap_det_M and logdet_lowrank):
//   grad_{n,x} l_d = tr M_x,   hess_n = sum_x sum_{a,b in T_n} (M_x)_ab (M_x)_ba,
// with (M_x)_ab = sum_l d_{n,x}Phi_{a l} G_{b l} (G = Phi^-T) per spin block,
// plus the Laplacian row term sum_l LapPhi_nl G_nl of electron n itself.
// Both M_x = D G^T and M_x^T = G D^T are formed tile by tile on 16x16x4 f64
// MFMA with the same output layout, so sum_ab M_ab M_ba is a lane-wise
// product of the two accumulators.  Rows past |T_n| are zero.
template <typename T, typename TI>
__global__ __launch_bounds__(256, 4) void k_det_lap(const Dims D, int Wc, int w0, const int* __restrict__ memb,
                                                 const int* __restrict__ mslot, const int* __restrict__ mcnt,
                                                 int tcap, const int32_t* __restrict__ ncnt,
                                                 const int* __restrict__ joff, const T* __restrict__ dphi0,
                                                 const T* __restrict__ dphi1, const char* __restrict__ state,
                                                 StateRec S, double* __restrict__ gd, double* __restrict__ hd) {
  const int K = D.K, n = D.n;
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= (int64_t)Wc * n * K) return;
  const int det = (int)(item % K);
  const int64_t en = item / K;
  const int wl = (int)(en / n), nn = (int)(en % n);
  const int r16 = lane & 15, kq = lane >> 4;
  const char* rec = state + (int64_t)(w0 + wl) * S.stride;
  double gx[3] = {0, 0, 0}, hs = 0, lapt = 0;
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s), KN = K * N, e0 = s == 0 ? 0 : D.nu;
    const int t = mcnt[2 * en + s];
    if (t == 0 || N == 0) continue;
    const T* dphi = s == 0 ? dphi0 : dphi1;
    const TI* G = (const TI*)(rec + S.inv) + det * phi_per_det(D) + phi_block_off(D, s);
    const int* mem = memb + (en * 2 + s) * tcap;
    const int* slt = mslot + (en * 2 + s) * tcap;
    // Laplacian-row term of electron n itself
    if ((nn < D.nu ? 0 : 1) == s) {
      const int cn = ncnt[2 * en] + ncnt[2 * en + 1];
      const int64_t lr = joff[en] + 3 * (1 + cn);
      double v = 0;
      for (int l = lane; l < N; l += 64)
        v += (double)dphi[lr * KN + det * N + l] * (double)G[(int64_t)(nn - e0) * N + l];
      lapt += v;
    }
    const int KT = (t + 15) / 16;
    const bool pair = (N & 1) == 0 && ((uintptr_t)dphi & (2 * sizeof(T) - 1)) == 0 &&
                      ((uintptr_t)G & (2 * sizeof(TI) - 1)) == 0;
    for (int x = 0; x < 3; ++x) {
      for (int tx = 0; tx < KT; ++tx) {
        // row of this lane in tile tx: G row and jet row of member a
        const int a = 16 * tx + r16;
        const bool oka = a < t;
        const int ua = oka ? mem[a] : e0;
        const int64_t ra = oka ? ((int64_t)joff[(int64_t)wl * n + ua] + 3 * slt[a] + x) * KN + det * N : 0;
        const TI* ga = G + (int64_t)(ua - e0) * N;
        for (int ty = 0; ty < KT; ++ty) {
          const int b = 16 * ty + r16;
          const bool okb = b < t;
          const int ub = okb ? mem[b] : e0;
          const int64_t rb = okb ? ((int64_t)joff[(int64_t)wl * n + ub] + 3 * slt[b] + x) * KN + det * N : 0;
          const TI* gb = G + (int64_t)(ub - e0) * N;
          d4v_ m1 = {0.0, 0.0, 0.0, 0.0}, m2 = {0.0, 0.0, 0.0, 0.0};
          // unconditional reads (rows past t read member row 0 of the
          // segment and G row e0, columns past N read column N-1; values
          // zeroed after), every MFMA step runs: the reads of a 24-column
          // chunk are all in flight together
          constexpr int CH = 6;
          for (int cb = 0; cb < N; cb += 4 * CH) {
            double dx[CH], gyv[CH], gxv[CH], dyv[CH];
            if (pair) {
              // steps 2v, 2v + 1 of lane group kq: columns cb + 8 v + 2 kq and
              // the next one (N even, rows aligned), one read per pair; the
              // K order is permuted alike in all four operands
#pragma unroll
              for (int v = 0; v < CH / 2; ++v) {
                const int col = cb + 8 * v + 2 * kq;
                const bool cin = col < N;
                const int cc = cin ? col : N - 2;
                const Two<T> a0 = *reinterpret_cast<const Two<T>*>(dphi + ra + cc);
                const Two<TI> a1 = *reinterpret_cast<const Two<TI>*>(ga + cc);
                const Two<TI> a2 = *reinterpret_cast<const Two<TI>*>(gb + cc);
                const Two<T> a3 = *reinterpret_cast<const Two<T>*>(dphi + rb + cc);
                const bool ka = oka && cin, kb = okb && cin;
                dx[2 * v] = ka ? (double)a0.a : 0.0;
                dx[2 * v + 1] = ka ? (double)a0.b : 0.0;
                gxv[2 * v] = ka ? (double)a1.a : 0.0;
                gxv[2 * v + 1] = ka ? (double)a1.b : 0.0;
                gyv[2 * v] = kb ? (double)a2.a : 0.0;
                gyv[2 * v + 1] = kb ? (double)a2.b : 0.0;
                dyv[2 * v] = kb ? (double)a3.a : 0.0;
                dyv[2 * v + 1] = kb ? (double)a3.b : 0.0;
              }
            } else {
#pragma unroll
              for (int u = 0; u < CH; ++u) {
                const int col = cb + 4 * u + kq;
                const bool cin = col < N;
                const int cc = cin ? col : N - 1;
                const double v0 = (double)dphi[ra + cc], v1 = (double)ga[cc];
                const double v2 = (double)gb[cc], v3 = (double)dphi[rb + cc];
                dx[u] = (oka && cin) ? v0 : 0.0;
                gxv[u] = (oka && cin) ? v1 : 0.0;
                gyv[u] = (okb && cin) ? v2 : 0.0;
                dyv[u] = (okb && cin) ? v3 : 0.0;
              }
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
              m1 = __builtin_amdgcn_mfma_f64_16x16x4f64(dx[u], gyv[u], m1, 0, 0, 0);
              m2 = __builtin_amdgcn_mfma_f64_16x16x4f64(gxv[u], dyv[u], m2, 0, 0, 0);
            }
          }
          // output layout: register i of lane l holds row 4 i + l/16, column l%16
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            hs += m1[i] * m2[i];
            if (tx == ty && 4 * i + kq == r16) gx[x] += m1[i];
          }
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    gx[0] += __shfl_xor(gx[0], o, 64);
    gx[1] += __shfl_xor(gx[1], o, 64);
    gx[2] += __shfl_xor(gx[2], o, 64);
    hs += __shfl_xor(hs, o, 64);
    lapt += __shfl_xor(lapt, o, 64);
  }
  if (lane == 0) {
    double* o = gd + (((int64_t)wl * K + det) * n + nn) * 3;
    o[0] = gx[0]; o[1] = gx[1]; o[2] = gx[2];
    hd[((int64_t)wl * K + det) * n + nn] = lapt - hs;
  }
}

// kinetic energy per walker: with psi = e^J D, D = sum_d s_d e^{l_d},
// -1/2 Lap psi / psi = -1/2 [sum_d w_d (Lap l_d + |grad l_d|^2)
//                           + Lap J + |grad J|^2 + 2 grad J . g],
// w_d = s_d e^{l_d} / D, g = sum_d w_d grad l_d; grad log|psi| = g + grad J.
// J = sum_{i<j} u(r_ij) (cusp Jastrow): grad_i J = sum_j u'(r_ij) (r_i - r_j)/r_ij,
// Lap_i J = sum_j (u''(r_ij) + 2 u'(r_ij)/r_ij).
__global__ __launch_bounds__(256) void k_kinetic(const Dims D, int Wc, int w0, const char* __restrict__ state,
                                                 StateRec S, const double* __restrict__ gd,
                                                 const double* __restrict__ hd, const double* __restrict__ R,
                                                 const double* __restrict__ jasq, const double* __restrict__ gJ,
                                                 const double* __restrict__ lapJ, double* __restrict__ kin,
                                                 double* __restrict__ grad) {
  __shared__ double red[16];
  __shared__ double wd[32];
  const int wl = blockIdx.x;
  const int64_t w = w0 + wl;
  const char* rec = state + w * S.stride;
  const double* ds = (const double*)(rec + S.dsign);
  const double* dl = (const double*)(rec + S.dlog);
  const double lp = *(const double*)(rec + S.lpsi), sp = *(const double*)(rec + S.spsi);
  const int K = D.K, n = D.n, tid = threadIdx.x;
  if (tid < K) wd[tid] = ds[2 * tid] * ds[2 * tid + 1] * sp * exp(dl[2 * tid] + dl[2 * tid + 1] - lp);
  __syncthreads();
  const double* Rw = R + w * n * 3;
  const bool jas_on = jasq[0] != 0.0 || jasq[2] != 0.0;   // J = 0 when both weights are
  double acc = 0;
  for (int q = tid; q < 3 * n; q += blockDim.x) {
    double g = 0;
    for (int k = 0; k < K; ++k) {
      const double v = gd[((int64_t)wl * K + k) * n * 3 + q];
      g += wd[k] * v;
      acc += wd[k] * v * v;
    }
    const int i = q / 3, c = q - 3 * i;
    double gj = 0;
    for (int j = 0; j < (jas_on ? n : 0); ++j) {
      if (j == i) continue;
      const double dx = Rw[3 * i] - Rw[3 * j], dy = Rw[3 * i + 1] - Rw[3 * j + 1], dz = Rw[3 * i + 2] - Rw[3 * j + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      double u, u1, u2;
      jas_u3(jasq, (i < D.nu) == (j < D.nu), r, u, u1, u2);
      gj += u1 * (Rw[3 * i + c] - Rw[3 * j + c]) / r;
    }
    if (gJ) gj += gJ[(int64_t)wl * 3 * n + q];
    acc += 2.0 * gj * g + gj * gj;
    if (grad) grad[w * 3 * n + q] = g + gj;
  }
  for (int q = tid; q < n; q += blockDim.x) {
    for (int k = 0; k < K; ++k) acc += wd[k] * hd[((int64_t)wl * K + k) * n + q];
    double lj = 0;
    for (int j = 0; j < (jas_on ? n : 0); ++j) {
      if (j == q) continue;
      const double dx = Rw[3 * q] - Rw[3 * j], dy = Rw[3 * q + 1] - Rw[3 * j + 1], dz = Rw[3 * q + 2] - Rw[3 * j + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      double u, u1, u2;
      jas_u3(jasq, (q < D.nu) == (j < D.nu), r, u, u1, u2);
      lj += u2 + 2.0 * u1 / r;
    }
    acc += lj;
  }
  if (lapJ && tid == 0) acc += lapJ[wl];
  const double tot = block_sum<double>(acc, red);
  if (tid == 0) kin[w] = -0.5 * tot;
}

// V_ee, V_en (bare or erf-smoothed local pseudopotential) and V_nn in FP64
__global__ __launch_bounds__(256) void k_potential(const Dims D, int W, const double* __restrict__ R,
                                                   const double* __restrict__ Rn, const double* __restrict__ Zn,
                                                   const double* __restrict__ ppw, double* __restrict__ out) {
  __shared__ double red[16];
  const int w = blockIdx.x, tid = threadIdx.x, n = D.n, M = D.M;
  const double* Rw = R + (int64_t)w * n * 3;
  double vee = 0, ven = 0, vnn = 0;
  for (int q = tid; q < n * n; q += blockDim.x) {
    const int i = q / n, j = q % n;
    if (j <= i) continue;
    const double dx = Rw[3 * i] - Rw[3 * j], dy = Rw[3 * i + 1] - Rw[3 * j + 1], dz = Rw[3 * i + 2] - Rw[3 * j + 2];
    vee += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  }
  for (int q = tid; q < n * M; q += blockDim.x) {
    const int i = q / M, m = q % M;
    const double dx = Rw[3 * i] - Rn[3 * m], dy = Rw[3 * i + 1] - Rn[3 * m + 1], dz = Rw[3 * i + 2] - Rn[3 * m + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double wv = ppw[m];
    if (wv > 0) ven += r < 1e-10 ? -Zn[m] * 2.0 / (wv * sqrt(M_PI)) : -Zn[m] * erf(r / wv) / r;
    else ven += -Zn[m] / r;
  }
  for (int q = tid; q < M * M; q += blockDim.x) {
    const int a = q / M, b = q % M;
    if (b <= a) continue;
    const double dx = Rn[3 * a] - Rn[3 * b], dy = Rn[3 * a + 1] - Rn[3 * b + 1], dz = Rn[3 * a + 2] - Rn[3 * b + 2];
    vnn += Zn[a] * Zn[b] / sqrt(dx * dx + dy * dy + dz * dz);
  }
  const double a = block_sum<double>(vee, red);
  const double b = block_sum<double>(ven, red);
  const double c = block_sum<double>(vnn, red);
  if (tid == 0) { out[3 * w] = a; out[3 * w + 1] = b; out[3 * w + 2] = c; }
}

// E_L and its parts
__global__ void k_local_energy_sum(int W, const double* __restrict__ kin, const double* __restrict__ pot,
                                   const double* __restrict__ vnl, const int32_t* __restrict__ status,
                                   double* __restrict__ e_loc, double* __restrict__ parts) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double v = vnl ? vnl[w] : 0.0;
  double e = kin[w] + pot[3 * w] + pot[3 * w + 1] + pot[3 * w + 2] + v;
  if (status[w]) e = NAN;
  e_loc[w] = e;
  if (parts) {
    parts[5 * w] = kin[w]; parts[5 * w + 1] = pot[3 * w]; parts[5 * w + 2] = pot[3 * w + 1];
    parts[5 * w + 3] = pot[3 * w + 2]; parts[5 * w + 4] = v;
  }
}

// ---------------------------------------------------------------------------
// host driver: kinetic energy for walkers [w0, w0 + Wc)
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t kinetic_chunk(const fire_handle* h, const Net<T>& P, int w0, int Wc, const double* R, char* state,
                                char* ws, double* kin, double* grad, int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  const LapLayout L = lap_layout(h, Wc);
  const int n = D.n, d = D.d;
  const int64_t rows = (int64_t)Wc * n;
  const double* Rc = R + (int64_t)w0 * n * 3;
  const int blk = d <= 64 ? 64 : (d + 63) / 64 * 64;
  int16_t* nidx = (int16_t*)(ws + L.nidx);
  int32_t* ncnt = (int32_t*)(ws + L.ncnt);
  int* joff = (int*)(ws + L.joff);
  int* jtot = (int*)(ws + L.jtot);
  T* yj = (T*)(ws + L.yj);
  T* ugj = (T*)(ws + L.ugj);
  T* h0j = (T*)(ws + L.h0j);
  T* projj = (T*)(ws + L.projj);
  T* hval = (T*)(ws + L.hval);
  T* zval = (T*)(ws + L.zval);
  T* basisj = (T*)(ws + L.basisj);
  T* jA[2] = {(T*)(ws + L.jetA[0]), (T*)(ws + L.jetA[1])};
  T* jB[2] = {(T*)(ws + L.jetB[0]), (T*)(ws + L.jetB[1])};

  launch_nbr(dim3(Wc), st, Rc, Wc, n, D.nu, D.cut * D.cut, D.cap_nbr, nidx, ncnt,
             status + w0);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_jet_offsets, dim3(1), dim3(1024), 0, st, Wc, n, D.nu, (const int32_t*)ncnt, joff, jtot);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_en_embed_jet<T>, dim3((unsigned)((rows + 3) / 4)), dim3(blk), 0, st, P, Rc, rows, yj);
  CHECK(hipGetLastError());
  {
    GemmArgs g{};
    g.A = yj; g.amap = rows_dense(d); g.Bt = P.Wvg_t; g.ldb = d; g.bias = P.b_vg; g.bias_period = 5;
    g.C = ugj; g.cmap = rows_dense(2 * d); g.ccol = cols_dense(); g.M = (int)(rows * 5); g.N = 2 * d; g.K = d;
    CHECK(gemm_site(h, SITE_JET, g, st));
  }
  hipLaunchKernelGGL(k_glu_jet<T>, dim3((unsigned)((rows * d + 255) / 256)), dim3(256), 0, st, (const T*)ugj, yj,
                     rows, d);
  CHECK(hipGetLastError());
  {
    GemmArgs g{};
    g.A = yj; g.amap = rows_dense(d); g.Bt = P.Wo_t; g.ldb = d; g.bias = P.b_o; g.bias_period = 5;
    g.C = h0j; g.cmap = rows_dense(d); g.ccol = cols_dense(); g.M = (int)(rows * 5); g.N = d; g.K = d;
    CHECK(gemm_site(h, SITE_JET, g, st));
    GemmArgs p{};
    p.A = h0j; p.amap = rows_dense(d); p.Bt = P.Wproj_t; p.ldb = d;
    p.C = projj; p.cmap = rows_dense(4 * d); p.ccol = cols_dense(); p.M = (int)(rows * 5); p.N = 4 * d; p.K = d;
    CHECK(gemm_site(h, SITE_JET, p, st));
  }
  hipLaunchKernelGGL(k_msg_jet<T>, dim3((unsigned)rows), dim3(blk), 0, st, P, Rc, rows, (const int16_t*)nidx,
                     (const int32_t*)ncnt, (const int*)joff, (const T*)h0j, (const T*)projj, hval, jA[0], jA[1]);
  CHECK(hipGetLastError());
  // MLP on values and jet rows
  T** jin = jA;
  T** jout = jB;
  for (int k = 0; k < D.L; ++k) {
    const char* Wk = (const char*)P.mlp_t + (size_t)k * d * d * h->gsize;
    GemmArgs g{};
    g.A = hval; g.amap = rows_dense(d); g.Bt = Wk; g.ldb = d; g.bias = P.mlp_b + (int64_t)k * d;
    g.C = zval; g.cmap = rows_dense(d); g.ccol = cols_dense(); g.M = (int)rows; g.N = d; g.K = d;
    CHECK(gemm_site(h, SITE_EMB, g, st));
    for (int s = 0; s < 2; ++s) {
      if (D.nsig(s) == 0) continue;
      GemmArgs j{};
      j.A = jin[s]; j.amap = rows_dense(d); j.Bt = Wk; j.ldb = d;
      j.C = jout[s]; j.cmap = rows_dense(d); j.ccol = cols_dense(); j.M = (int)L.rowcap[s]; j.N = d; j.K = d;
      j.Mdev = jtot + s;
      CHECK(gemm_site(h, SITE_JET, j, st));
    }
    hipLaunchKernelGGL(k_jet_act<T>, dim3((unsigned)rows), dim3(blk), 0, st, D, rows, (const int32_t*)ncnt,
                       (const int*)joff, (const T*)zval, hval, (const T*)jout[0], (const T*)jout[1], jout[0],
                       jout[1]);
    CHECK(hipGetLastError());
    T** t = jin; jin = jout; jout = t;
  }
  // envelope jets and orbital jets per spin
  hipLaunchKernelGGL(k_basis_jet<T>, dim3((unsigned)((rows * D.B + 255) / 256)), dim3(256), 0, st, P, Rc, rows,
                     basisj);
  CHECK(hipGetLastError());
  T* dph[2] = {(T*)(ws + L.dphi[0]), (T*)(ws + L.dphi[1])};
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s), e0 = s == 0 ? 0 : D.nu;
    if (N == 0) continue;
    const int KN = D.K * N;
    T* envj = (T*)(ws + L.envj[s]);
    T* oval = (T*)(ws + L.oval[s]);
    const void* Wb = s == 0 ? P.orb_t0 : P.orb_t1;
    GemmArgs g{};
    g.A = basisj + (int64_t)e0 * 5 * D.B; g.amap = RowMap{(int64_t)N * 5, (int64_t)n * 5 * D.B, D.B};
    g.Bt = s == 0 ? P.pi0 : P.pi1; g.ldb = D.B; g.C = envj; g.cmap = rows_dense(KN); g.ccol = cols_dense();
    g.M = Wc * N * 5; g.N = KN; g.K = D.B;
    CHECK(gemm_site(h, SITE_JET, g, st));
    GemmArgs o{};
    o.A = hval + (int64_t)e0 * d; o.amap = RowMap{N, (int64_t)n * d, d}; o.Bt = Wb; o.ldb = d;
    o.C = oval; o.cmap = rows_dense(KN); o.ccol = cols_dense(); o.M = Wc * N; o.N = KN; o.K = d;
    CHECK(gemm_site(h, SITE_ORB, o, st));
    GemmArgs j{};
    j.A = jin[s]; j.amap = rows_dense(d); j.Bt = Wb; j.ldb = d; j.C = dph[s]; j.cmap = rows_dense(KN);
    j.ccol = cols_dense(); j.M = (int)L.rowcap[s]; j.N = KN; j.K = d; j.Mdev = jtot + s;
    CHECK(gemm_site(h, SITE_JET, j, st));
    const int64_t tot = (int64_t)Wc * N * KN;
    hipLaunchKernelGGL(k_phi_jet<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, D, s, Wc,
                       (const int32_t*)ncnt, (const int*)joff, (const T*)oval, (const T*)envj, dph[s]);
    CHECK(hipGetLastError());
  }
  // determinant contraction and kinetic energy
  {
    double* gd = (double*)(ws + L.gd);
    double* hd = (double*)(ws + L.hd);
    int* memb = (int*)(ws + L.memb);
    int* mslot = (int*)(ws + L.mslot);
    int* mcnt = (int*)(ws + L.mcnt);
    hipLaunchKernelGGL(k_lap_members, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, D, Wc,
                       (const int16_t*)nidx, (const int32_t*)ncnt, L.tcap, memb, mslot, mcnt);
    CHECK(hipGetLastError());
    const unsigned nblk = (unsigned)((rows * D.K + 3) / 4);
    if (h->isize == 8)
      hipLaunchKernelGGL((k_det_lap<T, double>), dim3(nblk), dim3(256), 0, st, D, Wc, w0, (const int*)memb,
                         (const int*)mslot, (const int*)mcnt, L.tcap, (const int32_t*)ncnt, (const int*)joff,
                         (const T*)dph[0], (const T*)dph[1], (const char*)state, S, gd, hd);
    else
      hipLaunchKernelGGL((k_det_lap<T, float>), dim3(nblk), dim3(256), 0, st, D, Wc, w0, (const int*)memb,
                         (const int*)mslot, (const int*)mcnt, L.tcap, (const int32_t*)ncnt, (const int*)joff,
                         (const T*)dph[0], (const T*)dph[1], (const char*)state, S, gd, hd);
    CHECK(hipGetLastError());
    // MLP Jastrow: its gradient and Laplacian from the jets of h_i (jin
    // and the member lists are still intact; jout is free)
    double* gJ = nullptr;
    double* lapJ = nullptr;
    if (D.Hj > 0 || D.Ra > 0) {
      JmJetArgs a{};
      a.Wc = Wc; a.w0 = w0; a.rowcap[0] = L.rowcap[0]; a.rowcap[1] = L.rowcap[1];
      a.ncnt = ncnt; a.joff = joff; a.jtot = jtot; a.memb = memb; a.mslot = mslot; a.mcnt = mcnt; a.tcap = L.tcap;
      a.hval = hval; a.jin[0] = jin[0]; a.jin[1] = jin[1];
      if (D.Hj > 0) {
        a.zv = ws + L.jzv;
        for (int s = 0; s < 2; ++s) {
          a.jx[s] = ws + L.jjx[s];
          a.jy[s] = ws + L.jjy[s];
          a.jt[s] = (double*)(ws + L.jjt[s]);
        }
      }
      gJ = (double*)(ws + L.jgJ);
      lapJ = (double*)(ws + L.jlap);
      a.gJ = gJ; a.lapJ = lapJ;
      if (D.Hj > 0) CHECK(jm_kinetic<T>(h, P, a, (const char*)state, st));
      if (D.Ra > 0) CHECK(ja_kinetic<T>(h, P, a, (const char*)state, ws + L.jak, D.Hj == 0, st));
    }
    hipLaunchKernelGGL(k_kinetic, dim3(Wc), dim3(256), 0, st, D, Wc, w0, (const char*)state, S, (const double*)gd,
                       (const double*)hd, R, P.jas, (const double*)gJ, (const double*)lapJ, kin, grad);
    CHECK(hipGetLastError());
  }
  return hipSuccess;
}

// dynamic LDS of the Laplacian kernels (the determinant contraction runs in
// registers on MFMA tiles and needs none)
size_t lap_lds_needed(const fire_handle* h) { return 0; }

template <typename T>
static hipError_t local_energy_impl(fire_handle* h, int W, const double* R, char* state, char* ws,
                                    const double* quad_rot, double* e_loc, double* parts, double* grad,
                                    int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  Net<T> P = make_net<T>(h);
  const LapLayout L = lap_layout(h, W);
  // per-walker results first, then the region of the Laplacian chunks, then
  // that of the pseudopotential jobs
  double* kin = (double*)ws;
  double* pot = kin + align_up((size_t)W * 8) / 8;
  double* vnl = pot + align_up((size_t)W * 3 * 8) / 8;
  char* region = (char*)(vnl + align_up((size_t)W * 8) / 8);
  char* region_ecp = region + align_up(L.total);
  CHECK(fill_i32(status, W, 0, st));
  const bool has_ecp = !h->ecp.empty();
  // With a pseudopotential and overlap on, the kinetic energy and the
  // potential run on the handle's second stream, beside the quadrature jobs
  // on the caller's stream:
  // the two read the same state, write disjoint outputs and workspace regions,
  // and meet only in the status flags (atomic OR).  The fork (record on st,
  // wait on the side stream) is atomic under a lock, so concurrent calls
  // cannot swap their fork points; a later record of the join event lies
  // later on the serial side stream, so waiting on it is never too early.
  hipStream_t ks = st;
  const bool fork = has_ecp && h->overlap && h->side;
  AutotuneHold hold(fork);
  if (fork) {
    std::lock_guard<std::mutex> lock(handle_mutex());
    CHECK(hipEventRecord(h->side_fork, st));
    CHECK(hipStreamWaitEvent(h->side, h->side_fork, 0));
    ks = h->side;
  }
  for (int w0 = 0; w0 < W; w0 += L.Wc) {
    const int wc = W - w0 < L.Wc ? W - w0 : L.Wc;
    CHECK(kinetic_chunk<T>(h, P, w0, wc, R, state, region, kin, grad, status, ks));
  }
  hipLaunchKernelGGL(k_potential, dim3(W), dim3(256), 0, ks, D, W, R, P.Rn, P.Zn, P.ppw, pot);
  CHECK(hipGetLastError());
  if (fork) CHECK(hipEventRecord(h->side_join, ks));
  if (has_ecp) CHECK(ecp_into(h, W, R, state, region_ecp, quad_rot, vnl, status, st));
  if (fork) CHECK(hipStreamWaitEvent(st, h->side_join, 0));
  hipLaunchKernelGGL(k_local_energy_sum, dim3((W + 127) / 128), dim3(128), 0, st, W, (const double*)kin,
                     (const double*)pot, has_ecp ? (const double*)vnl : nullptr, (const int32_t*)status, e_loc, parts);
  return hipGetLastError();
}

size_t lap_ws_bytes(const fire_handle* h, int W) {
  const LapLayout L = lap_layout(h, W);
  const size_t reg = align_up(L.total) + align_up(ecp_ws_bytes(h, W));
  return align_up((size_t)W * 8) + align_up((size_t)W * 3 * 8) + align_up((size_t)W * 8) + reg;
}

hipError_t local_energy_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                             double* e_loc, double* parts, double* grad_logpsi, int32_t* status, hipStream_t s) {
  if (lap_lds_needed(h) > 160 * 1024 || h->D.cap_nbr > 128) return hipErrorInvalidValue;
  return h->tsize == 8 ? local_energy_impl<double>(h, W, R, state, ws, quad_rot, e_loc, parts, grad_logpsi, status, s)
                       : local_energy_impl<float>(h, W, R, state, ws, quad_rot, e_loc, parts, grad_logpsi, status, s);
}

}  // namespace fire
