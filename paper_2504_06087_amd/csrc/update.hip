// Single-electron updates (Methods, low-rank wave-function updates) and the
// Metropolis sweep built on them (Methods, improved Monte Carlo sampling).
//
// One step moves electron e of every walker.  The update set is
//   U = {e} u N(r_e) u N(r_e'),
// only h0_e, the messages of U and the MLP / orbital rows of U are recomputed,
// and for every determinant and spin block the ratio comes from
//   A = I + dPhi_U G_U^T,  det Phi' = det Phi det A,
// with G = Phi^-T cached (row k of G is column k of Phi^-1).  Accepted moves
// update G by the Woodbury identity in one read-modify-write pass:
//   G' = G - (G dPhi_U^T) A^-T G_U.
#include "update.hpp"
#include "jastrow.hpp"
#include "rng.hpp"

#include "embed_kernels.hpp"
#include "linalg.hpp"

namespace fire {

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

UpdLayout upd_layout(const fire_handle* h, int W, bool with_woodbury) {
  const Dims& D = h->D;
  UpdLayout L{};
  size_t o = 0, ts = h->tsize, is = h->isize;
  L.capS[0] = D.cap_upd < D.nu ? D.cap_upd : D.nu;
  L.capS[1] = D.cap_upd < D.nd ? D.cap_upd : D.nd;
  L.capmax = L.capS[0] > L.capS[1] ? L.capS[0] : L.capS[1];
  if (L.capmax < 1) L.capmax = 1;
  const int64_t Wl = W;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  L.rnew = take(Wl * 3 * 8);
  L.lqf = take(Wl * 8);
  L.dj = take(Wl * 8);
  L.uidx = take(Wl * 2 * L.capmax * 4);
  L.ucnt = take(Wl * 2 * 4);
  L.off = take((Wl + 1) * 2 * 4);
  L.acc = take(Wl * 4);
  L.detA = take(Wl * D.K * 2 * 2 * 8);
  L.y = take(Wl * D.d * ts);
  L.ug = take(Wl * 2 * D.d * ts);
  L.h0new = take(Wl * D.d * ts);
  L.projnew = take(Wl * 4 * D.d * ts);
  L.basis = take(Wl * D.B * ts);
  int nmax = D.nu > D.nd ? D.nu : D.nd;
  L.envnew = take(Wl * D.K * nmax * ts);
  for (int s = 0; s < 2; ++s) {
    const int per = L.capS[s] < kRowsPerJob ? L.capS[s] : kRowsPerJob;
    int64_t rows = Wl * (per > 0 ? per : 1);
    int N = D.nsig(s) > 0 ? D.nsig(s) : 1;
    L.rowcap[s] = rows;
    L.rowinfo[s] = take(rows * 2 * 4);
    L.hseg[s][0] = take(rows * D.d * ts);
    L.hseg[s][1] = take(rows * D.d * ts);
    L.mseg[s] = take(rows * D.d * ts);
    L.oseg[s] = take(rows * D.K * N * ts);
    // dPhi rows are kept only for the Woodbury update; ratio-only batches
    // form them on the fly
    L.dphi[s] = with_woodbury ? take(rows * D.K * N * ts) : 0;
    L.bbuf[s] = with_woodbury ? take(rows * D.K * N * 8) : 0;
    L.jnew[s] = D.Hj > 0 ? take(rows * 2 * 8) : 0;
  }
  if (D.Hj > 0) {
    L.jsum = take(Wl * 2 * 8);
    L.jscr = take(jm_rows_ws(h, L.rowcap[0] > L.rowcap[1] ? L.rowcap[0] : L.rowcap[1]));
  }
  if (D.Hj > 0 || D.Ra > 0) L.jsg = take(Wl * 8);
  if (D.Ra > 0) {
    for (int s = 0; s < 2; ++s) L.anew[s] = take(L.rowcap[s] * D.NA() * ts);
    L.ja = take(ja_update_ws(h, W));
  }
  L.total = o;
  return L;
}

// Det-lemma block order: eight job groups (jg consecutive jobs, K
// determinants each; a walker's groups are consecutive and read the same
// rows of Phi^-1) form a run of det_run blocks of `per` items; runs are
// dealt to the XCDs in turn (xcd_runs), and the grid is a whole number of
// eight runs.
FIRE_HOST_DEVICE int det_run(int jg, int K, int per) { return (8 * jg * K + per - 1) / per; }
static unsigned det_grid(int64_t blocks, int jg, int K, int per) {
  const int64_t r8 = 8 * det_run(jg, K, per);
  return (unsigned)((blocks + r8 - 1) / r8 * r8);
}

static size_t detA_lds(int k) { return (size_t)(k * (k + 1) + 2 * k + 8) * sizeof(double); }
static size_t wb_rows_lds(int N) { return (size_t)(2 * KS * N + WB_RB * N + WB_RB * KS + 8) * sizeof(double); }
// k_woodbury: G_U/row block, B, A, f in FP64 and dPhi_U in the elementwise type
static size_t wb_fused_lds(int N, int tsize, int ksm = KS) {
  const size_t gu = (size_t)ksm * N > 4 * 16 * 33 ? (size_t)ksm * N : 4 * 16 * 33;
  return (gu + (size_t)ksm * N + ksm * (ksm + 1) + ksm) * sizeof(double) + (size_t)ksm * N * tsize + 16;
}

bool update_fits(const fire_handle* h) {
  UpdLayout L = upd_layout(h, 1);
  const int N = h->D.nu > h->D.nd ? h->D.nu : h->D.nd;
  return L.capmax <= 128 && detA_lds(L.capmax) <= 160 * 1024 && wb_rows_lds(N) <= 160 * 1024 &&
         wb_fused_lds(N, 8) <= 160 * 1024;
}

// log sum_m Z_m exp(-|r - R_m|^2 / (2 tau^2)): log rho_global(r) up to the
// constant -log(sum Z) - 3/2 log(2 pi tau^2), which cancels in the ratio
FIRE_DEV double gmm_log_unnorm(double x, double y, double z, const double* Rn, const double* Zn, int M,
                               double inv2t2) {
  double amax = -INFINITY;
  for (int m = 0; m < M; ++m) {
    const double dx = x - Rn[3 * m], dy = y - Rn[3 * m + 1], dz = z - Rn[3 * m + 2];
    const double a = log(Zn[m]) - (dx * dx + dy * dy + dz * dz) * inv2t2;
    amax = a > amax ? a : amax;
  }
  double sum = 0.0;
  for (int m = 0; m < M; ++m) {
    const double dx = x - Rn[3 * m], dy = y - Rn[3 * m + 1], dz = z - Rn[3 * m + 2];
    sum += exp(log(Zn[m]) - (dx * dx + dy * dy + dz * dz) * inv2t2 - amax);
  }
  return amax + log(sum);
}

// ---------------------------------------------------------------------------
// propose: r_e' = r_e + step * xi (local move) or a draw of the global
// proposal rho_global (SI, improved Monte Carlo sampling), and the update
// set, one wave per walker.
// uidx[w][s][t]: spin-s members in ascending order, e first in its own list.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_propose(const double* __restrict__ R, Jobs jb, int n, int nu, int e,
                                                 double cut2, int cap0, int cap1, int capmax,
                                                 double* __restrict__ rnew, int* __restrict__ uidx,
                                                 int* __restrict__ ucnt, const double* __restrict__ jasq,
                                                 double* __restrict__ dj, int32_t* status) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= jb.J) return;
  if (jb.Jdev && j >= *jb.Jdev) {
    if (lane == 0) { ucnt[2 * j] = 0; ucnt[2 * j + 1] = 0; }
    return;
  }
  const int w = jb.jw ? jb.jw[j] : j;
  const double* Rw = R + (int64_t)w * n * 3;
  const double ox = Rw[3 * e], oy = Rw[3 * e + 1], oz = Rw[3 * e + 2];
  double nx, ny, nz;
  if (jb.rexp) {
    nx = jb.rexp[3 * j]; ny = jb.rexp[3 * j + 1]; nz = jb.rexp[3 * j + 2];
  } else if (jb.pick) {
    // component: the first nucleus whose cumulative charge fraction exceeds
    // the uniform pick; then R_m + gstep * xi
    double tot = 0.0;
    for (int m = 0; m < jb.M; ++m) tot += jb.Zn[m];
    const double pk = jb.pick[j];
    int mc = jb.M - 1;
    double cum = 0.0;
    for (int m = 0; m < jb.M; ++m) {
      cum += jb.Zn[m];
      if (cum / tot > pk) { mc = m; break; }
    }
    nx = jb.Rn[3 * mc] + jb.gstep * jb.xi[3 * j];
    ny = jb.Rn[3 * mc + 1] + jb.gstep * jb.xi[3 * j + 1];
    nz = jb.Rn[3 * mc + 2] + jb.gstep * jb.xi[3 * j + 2];
    if (lane == 0 && jb.lqf) {
      const double inv2t2 = 1.0 / (2.0 * jb.gstep * jb.gstep);
      jb.lqf[j] = gmm_log_unnorm(ox, oy, oz, jb.Rn, jb.Zn, jb.M, inv2t2) -
                  gmm_log_unnorm(nx, ny, nz, jb.Rn, jb.Zn, jb.M, inv2t2);
    }
  } else {
    nx = ox + jb.step * jb.xi[3 * j]; ny = oy + jb.step * jb.xi[3 * j + 1]; nz = oz + jb.step * jb.xi[3 * j + 2];
  }
  if (lane == 0) {
    rnew[3 * j] = nx; rnew[3 * j + 1] = ny; rnew[3 * j + 2] = nz;
    if (!isfinite(nx) || !isfinite(ny) || !isfinite(nz)) atomicOr(status + w, FIRE_W_NONFINITE);
  }
  // change of log J_cusp: sum over i != e of u(|r_e' - r_i|) - u(|r_e - r_i|)
  // (zero without the factor: both weights zero)
  if (jasq[0] == 0.0 && jasq[2] == 0.0) {
    if (lane == 0) dj[j] = 0.0;
  } else {
    double d = 0.0;
    for (int i = lane; i < n; i += 64) {
      if (i == e) continue;
      const double ix = Rw[3 * i], iy = Rw[3 * i + 1], iz = Rw[3 * i + 2];
      const bool same = (i < nu) == (e < nu);
      const double rn = sqrt((nx - ix) * (nx - ix) + (ny - iy) * (ny - iy) + (nz - iz) * (nz - iz));
      const double ro = sqrt((ox - ix) * (ox - ix) + (oy - iy) * (oy - iy) + (oz - iz) * (oz - iz));
      d += jas_u(jasq, same, rn) - jas_u(jasq, same, ro);
    }
    d = wave_sum(d);
    if (lane == 0) dj[j] = d;
  }
  const int se = e < nu ? 0 : 1;
  int cnt[2] = {0, 0};
  cnt[se] = 1;
  int* u0 = uidx + (int64_t)j * 2 * capmax;
  if (lane == 0) u0[se * capmax] = e;
  const int cap[2] = {cap0, cap1};
  bool over = false;
  for (int i0 = 0; i0 < n; i0 += 64) {
    int i = i0 + lane;
    bool in = false;
    if (i < n && i != e) {
      double x = Rw[3 * i], y = Rw[3 * i + 1], z = Rw[3 * i + 2];
      double d0 = (x - ox) * (x - ox) + (y - oy) * (y - oy) + (z - oz) * (z - oz);
      double d1 = (x - nx) * (x - nx) + (y - ny) * (y - ny) + (z - nz) * (z - nz);
      in = d0 <= cut2 || d1 <= cut2;
    }
    const int si = i < nu ? 0 : 1;
    uint64_t m = __ballot(in);
    uint64_t mup = __ballot(in && si == 0);
    uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int pos = si == 0 ? __popcll(mup & below) : __popcll((m & ~mup) & below);
    if (in) {
      int t = cnt[si] + pos;
      if (t < cap[si]) u0[si * capmax + t] = i;
    }
    cnt[0] += __popcll(mup);
    cnt[1] += __popcll(m & ~mup);
  }
  for (int s = 0; s < 2; ++s)
    if (cnt[s] > cap[s]) { over = true; cnt[s] = cap[s]; }
  if (lane == 0) {
    ucnt[2 * j] = cnt[0];
    ucnt[2 * j + 1] = cnt[1];
    if (over) atomicOr(status + w, FIRE_W_UPD_OVERFLOW);
  }
}

// exclusive scan of the per-spin member counts: off[s][w], off[s][W] = total.
// A job whose rows would end beyond the segment capacity gets zero members
// (it is skipped) and its walker is flagged.  Jobs at or beyond a device job
// count (when given) have no members: the scan covers the live ones and the
// rest get the total as their offset.
__global__ __launch_bounds__(1024) void k_scan_counts(int* __restrict__ ucnt, int W, int* __restrict__ off,
                                                      int64_t cap0, int64_t cap1, const int* __restrict__ jw,
                                                      int32_t* __restrict__ status, const int* __restrict__ Jdev) {
  __shared__ int wtot[2][16];
  __shared__ int first_over[2], total[2];
  const int t = threadIdx.x, nt = blockDim.x;   // nt = 1024: 16 full waves
  const int lane = t & 63, wv = t >> 6, nw = nt >> 6;
  const int Wl = Jdev && *Jdev < W ? (*Jdev > 0 ? *Jdev : 0) : W;
  const int per = (Wl + nt - 1) / nt;
  if (t < 2) first_over[t] = 0x7fffffff;
  const int b = t * per, e = b + per < Wl ? b + per : Wl;
  int s0 = 0, s1 = 0;
  for (int w = b; w < e; ++w) { s0 += ucnt[2 * w]; s1 += ucnt[2 * w + 1]; }
  // exclusive scan of the threads' sums: inclusive scans within each wave,
  // then the wave totals in order
  int i0 = s0, i1 = s1;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y0 = __shfl_up(i0, d), y1 = __shfl_up(i1, d);
    if (lane >= d) { i0 += y0; i1 += y1; }
  }
  if (lane == 63) { wtot[0][wv] = i0; wtot[1][wv] = i1; }
  __syncthreads();
  if (t < 2) {
    int acc = 0;
    for (int k = 0; k < nw; ++k) { const int v = wtot[t][k]; wtot[t][k] = acc; acc += v; }
    off[t * (W + 1) + W] = acc;
    total[t] = acc;
  }
  __syncthreads();
  for (int w = Wl + t; w < W; w += nt) {
    off[w] = total[0];
    off[(W + 1) + w] = total[1];
  }
  int a0 = wtot[0][wv] + i0 - s0, a1 = wtot[1][wv] + i1 - s1;
  for (int w = b; w < e; ++w) {
    off[w] = a0;
    off[(W + 1) + w] = a1;
    const int c0 = ucnt[2 * w], c1 = ucnt[2 * w + 1];
    if (a0 + c0 > cap0 || a1 + c1 > cap1) {
      if (c0 + c1 > 0) atomicOr(status + (jw ? jw[w] : w), FIRE_W_UPD_OVERFLOW);
      ucnt[2 * w] = 0;
      ucnt[2 * w + 1] = 0;
      // offsets only grow, so every later job overflows too: the rows in
      // use end at the first dropped job's offsets
      atomicMin(&first_over[0], a0);
      atomicMin(&first_over[1], a1);
    }
    a0 += c0;
    a1 += c1;
  }
  __syncthreads();
  // the row counts that later kernels read on the device (GEMM rows, dPhi
  // rows) cover exactly the rows written: never the rows of a dropped job
  if (t < 2) {
    int tot = off[t * (W + 1) + W];
    if (tot > first_over[t]) tot = first_over[t];
    const int64_t cap = t == 0 ? cap0 : cap1;
    if (tot > cap) tot = (int)cap;
    off[t * (W + 1) + W] = tot;
  }
}

// ---------------------------------------------------------------------------
// messages of the update set.  For u != e:
//   m_u' = m_u - edge(u, e; r_e, b_e) + edge(u, e; r_e', b_e')
// and m_e' is recomputed over the members within c of r_e'.  Writes h1' =
// h0 + m' and m' for every member at its compact row, and the row's (w, u).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1) void k_msg_update(Net<T> P, int W, const int* __restrict__ jw, int e,
                                                    const double* __restrict__ R,
                                                    const double* __restrict__ rnew, const int* __restrict__ uidx,
                                                    int capmax, const int* __restrict__ ucnt,
                                                    const int* __restrict__ off, const char* __restrict__ state,
                                                    StateRec S, const T* __restrict__ h0new,
                                                    const T* __restrict__ projnew, T* hseg0, T* hseg1, T* mseg0,
                                                    T* mseg1, int* rinfo0, int* rinfo1) {
  const Dims& D = P.D;
  constexpr int MPC = 21;               // members per chunk (3 pair feature sets each)
  __shared__ T feat[3 * MPC * FEAT];
  __shared__ int mem[MPC];
  __shared__ T fw[2 * FW_SIZE];   // filter weights of both pair classes
  const int j = blockIdx.x;
  if (ucnt[2 * j] + ucnt[2 * j + 1] == 0) return;   // inactive job
  for (int a = 0; a < 2; ++a)
    stage_filter<T>(P.ee_W1 + a * 4 * D.h1, P.ee_b1 + a * D.h1, P.ee_W2 + a * D.h1 * D.h2, P.ee_b2 + a * D.h2,
                    P.ee_sig + a * D.G, D, fw + a * FW_SIZE, threadIdx.x, blockDim.x);
  const int w = jw ? jw[j] : j;
  const int c = threadIdx.x;
  const bool act = c < D.d;
  const int n = D.n, se = e < D.nu ? 0 : 1;
  const char* rec = state + (int64_t)w * S.stride;
  const T* h0 = (const T*)(rec + S.h0);
  const T* proj = (const T*)(rec + S.proj);
  const T* mold = (const T*)(rec + S.m);
  const double* Rw = R + (int64_t)w * n * 3;
  const double ox = Rw[3 * e], oy = Rw[3 * e + 1], oz = Rw[3 * e + 2];
  const double nx = rnew[3 * j], ny = rnew[3 * j + 1], nz = rnew[3 * j + 2];
  const T* pe_new = projnew + (int64_t)j * 4 * D.d;
  T acc_e = 0;
  for (int s = 0; s < 2; ++s) {
    const int a = (s == se) ? 0 : 1;
    const int cnt = ucnt[2 * j + s];
    const int* lst = uidx + ((int64_t)j * 2 + s) * capmax;
    T w3[kMaxH2], wenv[kMaxG], we[4], bb = 0, be_old = 0, be_new = 0, ae_new = 0;
    if (act) {
      for (int k = 0; k < D.h2; ++k) w3[k] = P.ee_W3[(a * D.h2 + k) * D.d + c];
      for (int k = 0; k < D.G; ++k) wenv[k] = P.ee_Wenv[(a * D.G + k) * D.d + c];
      for (int k = 0; k < 4; ++k) we[k] = P.msg_We[(a * 4 + k) * D.d + c];
      bb = P.msg_b[a * D.d + c];
      be_old = proj[((int64_t)e * 4 + 2 + a) * D.d + c];
      be_new = pe_new[(2 + a) * D.d + c];
      ae_new = pe_new[a * D.d + c];
    }
    T* hseg = s == 0 ? hseg0 : hseg1;
    T* mseg = s == 0 ? mseg0 : mseg1;
    int* rinfo = s == 0 ? rinfo0 : rinfo1;
    const int q0 = off[s * (W + 1) + j];
    for (int t0 = 0; t0 < cnt; t0 += MPC) {
      const int tc = cnt - t0 < MPC ? cnt - t0 : MPC;
      __syncthreads();
      if (threadIdx.x < 3 * tc) {
        const int t = threadIdx.x / 3, kind = threadIdx.x % 3;
        const int u = lst[t0 + t];
        if (kind == 0) mem[t] = u;
        const double ux = Rw[3 * u], uy = Rw[3 * u + 1], uz = Rw[3 * u + 2];
        double dx, dy, dz;
        if (kind == 0) { dx = ux - ox; dy = uy - oy; dz = uz - oz; }        // (u, e) old
        else if (kind == 1) { dx = ux - nx; dy = uy - ny; dz = uz - nz; }   // (u, e) new
        else { dx = nx - ux; dy = ny - uy; dz = nz - uz; }                  // (e, u) new
        const T* fa = fw + a * FW_SIZE;
        pair_features_lds<T>((T)dx, (T)dy, (T)dz, fa + FW_W1, fa + FW_B1, fa, (T)D.cut, D,
                             feat + threadIdx.x * FEAT);
      }
      __syncthreads();
      if (!act) continue;
      // per-member cached values of 8 members are loaded together
      constexpr int MG = 8;
      for (int tg = 0; tg < tc; tg += MG) {
        T mo[MG], au_[MG], bu_[MG], h0u[MG];
#pragma unroll
        for (int v = 0; v < MG; ++v) {
          const int u = tg + v < tc ? mem[tg + v] : e;
          mo[v] = mold[(int64_t)u * D.d + c];
          au_[v] = proj[((int64_t)u * 4 + a) * D.d + c];
          bu_[v] = proj[((int64_t)u * 4 + 2 + a) * D.d + c];
          h0u[v] = h0[(int64_t)u * D.d + c];
        }
#pragma unroll
        for (int v = 0; v < MG; ++v) {
          const int t = tg + v;
          if (t >= tc) break;
          const int u = mem[t];
          if (u == e) continue;
          T mu = mo[v];
          const T au = au_[v];
          for (int kind = 0; kind < 3; ++kind) {
            const T* f = feat + (3 * t + kind) * FEAT;
            if (f[44] == T(0)) continue;
            T g1 = 0, g2 = 0;
#pragma unroll
            for (int q = 0; q < kMaxH2; ++q)
              if (q < D.h2) g1 += f[4 + q] * w3[q];
#pragma unroll
            for (int q = 0; q < kMaxG; ++q)
              if (q < D.G) g2 += f[12 + q] * wenv[q];
            const T ef = f[0] * we[0] + f[1] * we[1] + f[2] * we[2] + f[3] * we[3] + bb;
            if (kind == 0) mu -= g1 * g2 * silu_(au + be_old + ef);
            else if (kind == 1) mu += g1 * g2 * silu_(au + be_new + ef);
            else acc_e += g1 * g2 * silu_(ae_new + bu_[v] + ef);
          }
          const int64_t q = q0 + t0 + t;
          __builtin_nontemporal_store(h0u[v] + mu, hseg + (int64_t)q * D.d + c);
          __builtin_nontemporal_store(mu, mseg + (int64_t)q * D.d + c);
          if (c == 0) { rinfo[2 * q] = j; rinfo[2 * q + 1] = u; }
        }
      }
    }
  }
  if (act) {
    T* hseg = se == 0 ? hseg0 : hseg1;
    T* mseg = se == 0 ? mseg0 : mseg1;
    int* rinfo = se == 0 ? rinfo0 : rinfo1;
    const int64_t q = off[se * (W + 1) + j];   // e is first in its list
    __builtin_nontemporal_store(h0new[(int64_t)j * D.d + c] + acc_e, hseg + (int64_t)q * D.d + c);
    __builtin_nontemporal_store(acc_e, mseg + (int64_t)q * D.d + c);
    if (c == 0) { rinfo[2 * q] = j; rinfo[2 * q + 1] = e; }
  }
}

// Phi' rows = o' * env (cached env, or the moved electron's new env) and
// dPhi = Phi' - Phi in the inverse's precision.  One workgroup per update row
// (rows at or beyond the device row count exit), threads over its K N entries.
template <typename T>
__global__ __launch_bounds__(256) void k_dphi(const Dims D, int s, int e, const int* __restrict__ jw,
                                              const int* __restrict__ rinfo, const int* __restrict__ Mdev,
                                              T* __restrict__ oseg, const char* __restrict__ state, StateRec S,
                                              const T* __restrict__ envnew, T* __restrict__ dphi) {
  const int64_t r = blockIdx.x;
  if (r >= *Mdev) return;
  const int N = D.nsig(s);
  const int KN = D.K * N;
  const int j = rinfo[2 * r], u = rinfo[2 * r + 1];
  const int w = jw ? jw[j] : j;
  const int iloc = s == 0 ? u : u - D.nu;
  const char* rec = state + (int64_t)w * S.stride;
  const int64_t boff = phi_block_off(D, s) + (int64_t)iloc * N;
  const T* envc = (const T*)(rec + S.env) + boff;
  const T* phic = (const T*)(rec + S.phi) + boff;
  const T* envn = envnew + (int64_t)j * KN;
  const bool moved = u == e;
  T* orow = oseg + r * KN;
  T* drow = dphi + r * KN;
  for (int col = threadIdx.x; col < KN; col += blockDim.x) {
    const int det = col / N, l = col - det * N;
    const int64_t idx = (int64_t)det * phi_per_det(D) + l;
    const T env = moved ? envn[col] : envc[idx];
    const T pn = orow[col] * env;
    orow[col] = pn;
    drow[col] = pn - phic[idx];
  }
}

// A = I + dPhi_U G_U^T for one (job, determinant, spin block) into LDS:
// one wave per row a, lanes over the orbital index l, G rows read coalesced.
template <typename TD, typename TI>
FIRE_DEV void build_A(double* A, int LD, int k, int N, const TD* __restrict__ dp_rows, int64_t dp_stride,
                      const TI* __restrict__ G, const int* __restrict__ lst, int e0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int a = wave; a < k; a += nw) {
    const TD* dp = dp_rows + (int64_t)a * dp_stride;
    double x0 = lane < N ? (double)dp[lane] : 0.0;
    double x1 = lane + 64 < N ? (double)dp[lane + 64] : 0.0;
    for (int b = 0; b < k; ++b) {
      const TI* gb = G + (int64_t)(lst[b] - e0) * N;
      double v = x0 * (lane < N ? (double)gb[lane] : 0.0) + x1 * (lane + 64 < N ? (double)gb[lane + 64] : 0.0);
      v = wave_sum(v);
      if (lane == 0) A[a * LD + b] = v + (a == b ? 1.0 : 0.0);
    }
  }
}

// Row a of dPhi_U for one (job, determinant): either read from the dPhi
// segment or formed on the fly as o' env - Phi from the projections, the
// cached envelopes (the new ones for the moved electron) and the cached Phi.
template <typename T> struct DPhiRows {
  const T* dphi;     // [rows][K N], or null when fused
  const T* oseg;     // [rows][K N] projections o'
  const T* envnew;   // [job][K N]
  const T* envc;     // cached envelopes of this (walker, det, spin) block
  const T* phic;     // cached Phi of this block
  int64_t row0, KN, det, N;
  int e, e0, j;
  FIRE_DEV double at(int a, int u, int l) const {
    const int64_t q = (row0 + a) * KN + det * N + l;
    if (dphi) return (double)dphi[q];
    const int iloc = u - e0;
    const T en = u == e ? envnew[(int64_t)j * KN + det * N + l] : envc[(int64_t)iloc * N + l];
    return (double)(oseg[q] * en - phic[(int64_t)iloc * N + l]);
  }
  // base pointers of row a (electron u) for branch-free element reads:
  // x (dPhi, or o' when fused), y (envelope) and z (Phi)
  FIRE_DEV void row_ptrs(int a, int u, const T*& x, const T*& y, const T*& z) const {
    const int64_t q = (row0 + a) * KN + det * N;
    const int iloc = u - e0;
    x = (dphi ? dphi : oseg) + q;
    y = u == e ? envnew + (int64_t)j * KN + det * N : envc + (int64_t)iloc * N;
    z = phic + (int64_t)iloc * N;
  }
};

// det A for update sets with |U_s| > 32 (rare; the wave kernel below takes
// the rest).  One workgroup per (job group, determinant); A = I + dPhi_U G_U^T
// is built one wave per row (lanes over the orbital index, G rows read
// coalesced) into LDS, then Gauss-Jordan with partial pivoting.
template <typename T, typename TI>
__global__ __launch_bounds__(256) void k_detA(const Dims D, int W, const int* __restrict__ jw, int s, int e,
                                              const int* __restrict__ uidx, int capmax,
                                              const int* __restrict__ ucnt, const int* __restrict__ off,
                                              const T* __restrict__ dphi, const T* __restrict__ oseg,
                                              const T* __restrict__ envnew, const char* __restrict__ state,
                                              StateRec S, double* __restrict__ detA, int jg) {
  extern __shared__ double lds[];
  __shared__ double sc[2];
  __shared__ int fl[2];
  // grid-stride over jobs, each checked once: the update sets of more than
  // 32 rows this kernel takes are rare, so a small grid skips the rest
  // cheaply; a job that has one gets all its determinants
  const int N = D.nsig(s), KN = D.K * N;
  const int e0 = s == 0 ? 0 : D.nu;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  double* A = lds;                       // [capmax][capmax+1]
  double* f = A + capmax * (capmax + 1); // [capmax]
  int* pm = (int*)(f + capmax);
  for (int j = blockIdx.x; j < W; j += gridDim.x) {
    const int k = ucnt[2 * j + s];
    if (k <= 32) continue;   // handled by k_detA_wave / k_detA_mid
    const int w = jw ? jw[j] : j;
    for (int det = 0; det < D.K; ++det) {
      double* out = detA + (((int64_t)j * D.K + det) * 2 + s) * 2;
      const int LD = k + 1;
      const int* lst = uidx + ((int64_t)j * 2 + s) * capmax;
      const char* rec = state + (int64_t)w * S.stride;
      const int64_t boff = det * phi_per_det(D) + phi_block_off(D, s);
      const TI* G = (const TI*)(rec + S.inv) + boff;
      DPhiRows<T> dr{dphi, oseg, envnew, (const T*)(rec + S.env) + boff, (const T*)(rec + S.phi) + boff,
                     (int64_t)off[s * (W + 1) + j], (int64_t)KN, (int64_t)det, (int64_t)N, e, e0, j};
      for (int a = wave; a < k; a += nw) {
        const int ua = lst[a];
        const double x0 = lane < N ? dr.at(a, ua, lane) : 0.0;
        const double x1 = lane + 64 < N ? dr.at(a, ua, lane + 64) : 0.0;
        for (int b = 0; b < k; ++b) {
          const TI* gb = G + (int64_t)(lst[b] - e0) * N;
          double v = x0 * (lane < N ? (double)gb[lane] : 0.0) + x1 * (lane + 64 < N ? (double)gb[lane + 64] : 0.0);
          v = wave_sum(v);
          if (lane == 0) A[a * LD + b] = v + (a == b ? 1.0 : 0.0);
        }
      }
      __syncthreads();
      gj_block(A, k, LD, f, pm, sc, fl, false);
      if (tid == 0) {
        if (fl[1]) { out[0] = 0.0; out[1] = -INFINITY; }
        else { out[0] = sc[0]; out[1] = sc[1]; }
      }
      __syncthreads();
    }
  }
}

typedef double d4v_ __attribute__((ext_vector_type(4)));

// a double from one lane (the lane index must be wave-uniform)
FIRE_DEV double readlane_f64(double x, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// max over lanes 0..31 of a 32-bit key, wave-uniform result: DPP row
// shifts give each row's maximum in its lane 15, a row broadcast combines
// rows 0 and 1 in lane 31
FIRE_DEV uint32_t lanes32_max(uint32_t key) {
  uint32_t m = key;
  m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x111, 0xf, 0xf, false));   // row_shr:1
  m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x112, 0xf, 0xf, false));   // row_shr:2
  m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x114, 0xf, 0xf, false));   // row_shr:4
  m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x118, 0xf, 0xf, false));   // row_shr:8
  m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x142, 0xa, 0xf, false));   // row_bcast:15
  return (uint32_t)__builtin_amdgcn_readlane((int)m, 31);
}

// Orders this wave's LDS accesses: everything before it is complete, as
// seen by every lane of the wave, before anything after it.
FIRE_DEV void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// log|det A| and its sign of two matrices, one per half wave: lane 32 h + r
// holds row r of matrix h (columns in registers; rows and columns past the
// half's size kh <= 32 are zero).  Gaussian elimination with partial
// pivoting that never moves rows: the pivot of column p is the largest
// |A_rp| among the rows not yet used (ties to the lower row); the sign of
// the row permutation is counted as inversions, and the product of the
// pivots is carried as a mantissa and a binary exponent, so one logarithm is
// taken at the end.  The pivot lane of each half stores its row (from
// column p on) in LDS (piv: 64 doubles of this wave) and every lane of the
// half reads it back as a broadcast, so one instruction stream eliminates
// both matrices.  Every register index is a compile-time constant; the
// column guards are scalar, from the larger of the two sizes.
FIRE_DEV void halves_lu_det32(double (&row)[32], int kh, double* piv, double& sgn, double& logd, bool& sing) {
  const int lane = threadIdx.x & 63, h = lane >> 5, r = lane & 31;
  const int kmax = __builtin_amdgcn_readfirstlane(max(__builtin_amdgcn_readlane(kh, 0), __builtin_amdgcn_readlane(kh, 32)));
  uint32_t unused = kh >= 32 ? 0xffffffffu : ((1u << kh) - 1u);
  int inv = 0, ex = 0;
  double mant = 1.0;
  sgn = 1.0;
  sing = false;
  double* prow = piv + 32 * h;
#pragma unroll
  for (int p = 0; p < 32; ++p) {
    if (p < kmax) {
      const bool act = p < kh && !sing;
      const bool cand = act && ((unused >> r) & 1u);
      const float av = (float)fabs(row[p]);
      uint32_t m = cand ? ((__float_as_uint(av) & ~31u) | (uint32_t)(31 - r)) : 0u;
      m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x111, 0xf, 0xf, false));   // row_shr:1
      m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x112, 0xf, 0xf, false));   // row_shr:2
      m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x114, 0xf, 0xf, false));   // row_shr:4
      m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x118, 0xf, 0xf, false));   // row_shr:8
      m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x142, 0xa, 0xf, false));   // row_bcast:15
      const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)m, 31);
      const uint32_t b1 = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
      const uint32_t best = h ? b1 : b0;
      const int idx = 31 - (int)(best & 31u);
      if (act && r == idx) {
#pragma unroll
        for (int c0 = p & ~1; c0 < 32; c0 += 2)
          if (c0 < kmax) *reinterpret_cast<double2*>(prow + c0) = make_double2(row[c0], row[c0 + 1]);
      }
      wave_lds_order();
      const double pv = prow[p];
      const bool ok = act && (best & ~31u) != 0u && fabs(pv) > 0.0;
      if (act && !ok) sing = true;
      double f = 0.0;
      if (ok) {
        unused &= ~(1u << idx);
        inv += __popc(unused & ((1u << idx) - 1u));
        int e2;
        mant *= frexp(fabs(pv), &e2);
        ex += e2;
        int e3;
        mant = frexp(mant, &e3);
        ex += e3;
        if (pv < 0) sgn = -sgn;
        if ((unused >> r) & 1u) f = row[p] / pv;
      }
#pragma unroll
      for (int c0 = p & ~1; c0 < 32; c0 += 2) {
        if (c0 < kmax) {
          const double2 q = *reinterpret_cast<const double2*>(prow + c0);
          if (c0 > p) row[c0] -= f * q.x;
          if (c0 + 1 > p) row[c0 + 1] -= f * q.y;
        }
      }
      wave_lds_order();
    }
  }
  logd = log(mant) + (double)ex * 0.69314718055994530942;
  if (inv & 1) sgn = -sgn;
}

// log|det A| and sign of one k x k matrix (k <= 16) per 16-lane group: the
// four groups of a wave factor four matrices at once.  Lane 16 q + r holds
// row r of matrix q; kk is the size of this lane's matrix (0: no matrix).
// Same pivoting as wave_lu_det (largest magnitude among unused rows, no row
// moves, sign from the inversion count); the group maximum comes from DPP
// row shifts (a DPP row is a 16-lane group), rows are broadcast with
// ds_bpermute, which every lane executes.
FIRE_DEV void group_lu_det16(double (&row)[16], int kk, double& sgn, double& logd, bool& sing) {
  const int lane = threadIdx.x & 63, r = lane & 15, base = lane & ~15;
  uint32_t unused = kk >= 16 ? 0xffffu : ((1u << kk) - 1u);
  int inv = 0, ex = 0;
  double mant = 1.0;
  sgn = 1.0;
  sing = false;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const bool act = p < kk && !sing;
    const bool cand = act && ((unused >> r) & 1u);
    const float av = (float)fabs(row[p]);
    const uint32_t key = cand ? ((__float_as_uint(av) & ~15u) | (uint32_t)(15 - r)) : 0u;
    uint32_t m = key;
    m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x111, 0xf, 0xf, false));   // row_shr:1
    m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x112, 0xf, 0xf, false));   // row_shr:2
    m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x114, 0xf, 0xf, false));   // row_shr:4
    m = max(m, (uint32_t)__builtin_amdgcn_update_dpp((int)m, (int)m, 0x118, 0xf, 0xf, false));   // row_shr:8
    const uint32_t best = (uint32_t)__shfl((int)m, base + 15, 64);
    const int idx = 15 - (int)(best & 15u);
    const double pv = __shfl(row[p], base + idx, 64);
    const bool ok = act && (best & ~15u) != 0u && fabs(pv) > 0.0;
    if (act && !ok) sing = true;
    double f = 0.0;
    if (ok) {
      unused &= ~(1u << idx);
      inv += __popc(unused & ((1u << idx) - 1u));
      int e2;
      mant *= frexp(fabs(pv), &e2);
      ex += e2;
      int e3;
      mant = frexp(mant, &e3);
      ex += e3;
      if (pv < 0) sgn = -sgn;
      if ((unused >> r) & 1u) f = row[p] / pv;
    }
#pragma unroll
    for (int c = p + 1; c < 16; ++c) {
      const double pc = __shfl(row[c], base + idx, 64);
      row[c] -= f * pc;
    }
  }
  logd = log(mant) + (double)ex * 0.69314718055994530942;
  if (inv & 1) sgn = -sgn;
}

// The product dPhi_U G_U^T of one (job, determinant) item, 16 KT x 16 KT,
// on 16x16x4 f64 MFMA tiles, into LDS (row stride ld).  Only entries with
// both indices below k are meaningful: rows past k read row 0 (their
// entries are never used by the callers), so the loads need no guards.
// The orbital index runs in chunks of 4 CH columns (CH MFMA steps whose
// reads are all in flight together); each lane's row pointers carry its
// column within a chunk, so the full chunks read at constant offsets, and
// only the last, partial chunk clamps its columns and zeroes those past N.
template <typename T, typename TI, int KT, bool FUSED, bool PAIR>
FIRE_DEV void form_A(const DPhiRows<T>& dr, const TI* G, const int* lst, int k, int N, int e0, double* ab, int ld) {
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  // lane group kq: PAIR steps 2v, 2v + 1 take columns 8 v + 2 kq and the one
  // after it (N even, pairs aligned); otherwise step u takes column 4 u + kq
  const int lo = PAIR ? 2 * kq : kq;
  const T* xr[KT];
  const T* yr[KT];
  const T* zr[KT];
  const TI* gr[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int a = 16 * t + r16;
    const int aa = a < k ? a : 0;
    const int u = lst[aa];
    dr.row_ptrs(aa, u, xr[t], yr[t], zr[t]);
    xr[t] += lo;
    yr[t] += lo;
    zr[t] += lo;
    gr[t] = G + (int64_t)(u - e0) * N + lo;
  }
  d4v_ acc[KT][KT];
#pragma unroll
  for (int x = 0; x < KT; ++x)
#pragma unroll
    for (int y = 0; y < KT; ++y) acc[x][y] = d4v_{0.0, 0.0, 0.0, 0.0};
  constexpr int CH = KT == 2 ? 4 : 8;
  constexpr int CW = 4 * CH;
  auto chunk = [&](int cb, bool tail) {
    double af[CH][KT], bf[CH][KT];
    if constexpr (PAIR) {
#pragma unroll
      for (int v = 0; v < CH / 2; ++v) {
        const bool cok = !tail || cb + 8 * v + lo < N;
        const int o = cok ? cb + 8 * v : N - 2 - lo;
#pragma unroll
        for (int t = 0; t < KT; ++t) {
          const Two<T> x = *reinterpret_cast<const Two<T>*>(xr[t] + o);
          double v0, v1;
          if constexpr (FUSED) {
            const Two<T> y = *reinterpret_cast<const Two<T>*>(yr[t] + o);
            const Two<T> z = *reinterpret_cast<const Two<T>*>(zr[t] + o);
            v0 = (double)(x.a * y.a - z.a);
            v1 = (double)(x.b * y.b - z.b);
          } else {
            v0 = (double)x.a;
            v1 = (double)x.b;
          }
          const Two<TI> g = *reinterpret_cast<const Two<TI>*>(gr[t] + o);
          af[2 * v][t] = cok ? v0 : 0.0;
          af[2 * v + 1][t] = cok ? v1 : 0.0;
          bf[2 * v][t] = (double)g.a;
          bf[2 * v + 1][t] = (double)g.b;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const bool cok = !tail || cb + 4 * u + lo < N;
        const int o = cok ? cb + 4 * u : N - 1 - lo;
#pragma unroll
        for (int t = 0; t < KT; ++t) {
          double v;
          if constexpr (FUSED) v = (double)(xr[t][o] * yr[t][o] - zr[t][o]);
          else v = (double)xr[t][o];
          af[u][t] = cok ? v : 0.0;
          bf[u][t] = (double)gr[t][o];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
      for (int x = 0; x < KT; ++x)
#pragma unroll
        for (int y = 0; y < KT; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[u][x], bf[u][y], acc[x][y], 0, 0, 0);
  };
  const int nfull = N / CW;
#pragma unroll 1
  for (int c = 0; c < nfull; ++c) chunk(c * CW, false);
  if (nfull * CW < N) chunk(nfull * CW, true);
  // f64 16x16x4 output: register i of lane l holds row 4 i + l/16, column l%16
#pragma unroll
  for (int x = 0; x < KT; ++x)
#pragma unroll
    for (int y = 0; y < KT; ++y)
#pragma unroll
      for (int i = 0; i < 4; ++i) ab[(16 * x + 4 * i + kq) * ld + 16 * y + r16] = acc[x][y][i];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// det A = det(I + dPhi_U G_U^T) for (job, determinant) items with
// |U_s| <= 16, four per wave, formed one after another and factored
// together, one per 16-lane group.  Items are ordered (job group,
// determinant, job in group) so that the quadrature points of one
// electron-atom pair, which share most G rows, run side by side.  With FUSED,
// dPhi = o' env - Phi is formed on the fly from the projections, cached
// envelopes and Phi (no dPhi pass); PAIR (chosen on the host) reads two
// consecutive orbital columns at once.  16 < |U_s| <= 32 is left to
// k_detA_mid, |U_s| > 32 to k_detA.  Jobs at or beyond a device job count
// have empty update sets (k_propose clears their counts).
template <typename T, typename TI, bool FUSED, bool PAIR>
__global__ __launch_bounds__(256) void k_detA_wave(const Dims D, int W, const int* __restrict__ jw, int s, int e,
                                                   const int* __restrict__ uidx, int capmax,
                                                   const int* __restrict__ ucnt, const int* __restrict__ off,
                                                   const T* __restrict__ dphi, const T* __restrict__ oseg,
                                                   const T* __restrict__ envnew,
                                                   const char* __restrict__ state, StateRec S,
                                                   double* __restrict__ detA, int jg) {
  __shared__ double abuf[4][4 * 16 * 17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // item counts stay below 2^31: 32-bit index arithmetic
  const unsigned quad = (unsigned)xcd_runs(blockIdx.x, det_run(jg, D.K, 16)) * 4u + (unsigned)wave;
  const unsigned ujg = (unsigned)jg, uK = (unsigned)D.K;
  const unsigned total = ((unsigned)W + ujg - 1u) / ujg * ujg * uK;
  if (quad * 4u >= total) return;
  const int N = D.nsig(s), KN = D.K * N;
  const int e0 = s == 0 ? 0 : D.nu;
  double* ab = abuf[wave];
  int jq[4], dq[4], kqv[4];
  // (group, determinant, job in group) of the quad's first item, then stepped
  {
    unsigned ig = (quad * 4u) % ujg, rest = (quad * 4u) / ujg;
    unsigned id = rest % uK, g = rest / uK;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const unsigned j = g * ujg + ig;
      const bool live = quad * 4u + (unsigned)q < total && j < (unsigned)W;
      jq[q] = live ? (int)j : -1;
      dq[q] = (int)id;
      kqv[q] = live ? ucnt[2 * j + s] : -1;
      if (++ig == ujg) {
        ig = 0;
        if (++id == uK) { id = 0; ++g; }
      }
    }
  }
  auto item_rows = [&](int q, const TI*& G, DPhiRows<T>& dr, const int*& lst) {
    const int j = jq[q], det = dq[q];
    const int w = jw ? jw[j] : j;
    const int q0 = off[s * (W + 1) + j];
    lst = uidx + ((int64_t)j * 2 + s) * capmax;
    const char* rec = state + (int64_t)w * S.stride;
    const int64_t boff = det * phi_per_det(D) + phi_block_off(D, s);
    G = (const TI*)(rec + S.inv) + boff;
    dr = DPhiRows<T>{FUSED ? nullptr : dphi, oseg, envnew, (const T*)(rec + S.env) + boff,
                     (const T*)(rec + S.phi) + boff, (int64_t)q0, (int64_t)KN, (int64_t)det, (int64_t)N, e, e0, j};
  };
  auto out_of = [&](int q) { return detA + (((int64_t)jq[q] * D.K + dq[q]) * 2 + s) * 2; };
  // empty update sets here; 16 < |U_s| <= 32 in k_detA_mid
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (kqv[q] == 0 && lane == 0) {
      double* out = out_of(q);
      out[0] = 1.0;
      out[1] = 0.0;
    }
  }
  // the small ones together
  bool any = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) any = any || (kqv[q] >= 1 && kqv[q] <= 16);
  if (!any) return;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const int k = kqv[q];
    if (k >= 1 && k <= 16) {
      const TI* G;
      DPhiRows<T> dr;
      const int* lst;
      item_rows(q, G, dr, lst);
      double* aq = ab + q * 16 * 17;
      form_A<T, TI, 1, FUSED, PAIR>(dr, G, lst, k, N, e0, aq, 17);
    }
  }
  const int gq = lane >> 4, r = lane & 15;
  int kk = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (gq == q) kk = (kqv[q] >= 1 && kqv[q] <= 16) ? kqv[q] : 0;
  double row[16];
#pragma unroll
  for (int c = 0; c < 16; ++c)
    row[c] = (r < kk && c < kk) ? ab[gq * 16 * 17 + r * 17 + c] + (c == r ? 1.0 : 0.0) : 0.0;
  double sg, ld;
  bool sing;
  group_lu_det16(row, kk, sg, ld, sing);
  if (r == 0 && kk > 0) {
    double* out = detA + (((int64_t)jq[0] * D.K + dq[0]) * 2 + s) * 2;
#pragma unroll
    for (int q = 1; q < 4; ++q)
      if (gq == q) out = detA + (((int64_t)jq[q] * D.K + dq[q]) * 2 + s) * 2;
    if (sing) { out[0] = 0.0; out[1] = -INFINITY; }
    else { out[0] = sg; out[1] = ld; }
  }
}

// det A for items with 16 < |U_s| <= 32: each wave forms one 32 x 32
// product on MFMA tiles into its LDS buffer; then waves 0 and 2 of the
// block factor two matrices each (their own and the next wave's, one per
// half wave; halves_lu_det32).  Items are ordered (job, determinant), so
// the four waves of a block take four determinants of one job (K >= 4) and
// the jobs of a quadrature group (which share most rows of Phi^-1) follow
// one another.  Items of other sizes skip the work; every wave reaches the
// block barrier.
template <typename T, typename TI, bool FUSED, bool PAIR>
__global__ __launch_bounds__(256, 4) void k_detA_mid(const Dims D, int W, const int* __restrict__ jw, int s, int e,
                                                  const int* __restrict__ uidx, int capmax,
                                                  const int* __restrict__ ucnt, const int* __restrict__ off,
                                                  const T* __restrict__ dphi, const T* __restrict__ oseg,
                                                  const T* __restrict__ envnew,
                                                  const char* __restrict__ state, StateRec S,
                                                  double* __restrict__ detA, int jg) {
  __shared__ __align__(16) double abuf[4][32 * 33];
  __shared__ int kb[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // item counts stay below 2^31: 32-bit index arithmetic
  const unsigned item = (unsigned)xcd_runs(blockIdx.x, det_run(jg, D.K, 4)) * 4u + (unsigned)wave;
  const int j = (int)(item / (unsigned)D.K), det = (int)(item % (unsigned)D.K);
  int k = item < (unsigned)W * (unsigned)D.K ? ucnt[2 * j + s] : 0;
  k = (k > 16 && k <= 32) ? k : 0;
  if (lane == 0) kb[wave] = k;
  const int N = D.nsig(s), KN = D.K * N;
  const int e0 = s == 0 ? 0 : D.nu;
  double* ab = abuf[wave];
  if (k > 0) {
    const int w = jw ? jw[j] : j;
    const int q0 = off[s * (W + 1) + j];
    const int* lst = uidx + ((int64_t)j * 2 + s) * capmax;
    const char* rec = state + (int64_t)w * S.stride;
    const int64_t boff = det * phi_per_det(D) + phi_block_off(D, s);
    const TI* G = (const TI*)(rec + S.inv) + boff;
    const DPhiRows<T> dr{FUSED ? nullptr : dphi, oseg, envnew, (const T*)(rec + S.env) + boff,
                         (const T*)(rec + S.phi) + boff, (int64_t)q0, (int64_t)KN, (int64_t)det, (int64_t)N, e, e0, j};
    form_A<T, TI, 2, FUSED, PAIR>(dr, G, lst, k, N, e0, ab, 33);
  }
  __syncthreads();
  if (wave & 1) return;
  const int h = lane >> 5, r = lane & 31;
  const int kh = kb[wave + h];
  if (__builtin_amdgcn_readfirstlane(kb[wave] | kb[wave + 1]) == 0) return;
  const double* src = abuf[wave + h];
  double row[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) row[c] = (r < kh && c < kh) ? src[r * 33 + c] + (c == r ? 1.0 : 0.0) : 0.0;
  wave_lds_order();
  double sg, ld;
  bool sing;
  halves_lu_det32(row, kh, ab, sg, ld, sing);
  if (r == 0 && kh > 0) {
    // item (j, det) at j K + det; the paired wave's item is the next one
    double* out = detA + ((int64_t)(item + h) * 2 + s) * 2;
    if (sing) { out[0] = 0.0; out[1] = -INFINITY; }
    else { out[0] = sg; out[1] = ld; }
  }
}

// The det-lemma kernels by their flags (the signature does not depend on
// the inverse type TI).
template <typename T>
using DetAKernel = void (*)(const Dims, int, const int*, int, int, const int*, int, const int*, const int*,
                            const T*, const T*, const T*, const char*, StateRec, double*, int);
template <typename T, typename TI, bool F, bool P> static DetAKernel<T> detA_pick(bool mid) {
  return mid ? k_detA_mid<T, TI, F, P> : k_detA_wave<T, TI, F, P>;
}
template <typename T, typename TI> static DetAKernel<T> detA_pick(bool mid, bool fused, bool pair) {
  if (fused) return pair ? detA_pick<T, TI, true, true>(mid) : detA_pick<T, TI, true, false>(mid);
  return pair ? detA_pick<T, TI, false, true>(mid) : detA_pick<T, TI, false, false>(mid);
}
template <typename T> static DetAKernel<T> detA_kernel(const fire_handle* h, bool mid, bool fused, bool pair) {
  return h->isize == 8 ? detA_pick<T, double>(mid, fused, pair) : detA_pick<T, float>(mid, fused, pair);
}
// Two-column reads in the det-lemma products need every row of the Phi,
// envelope, inverse, projection and dPhi blocks to start at an even element
// offset of a 16-byte aligned base: both spin blocks even (the blocks of one
// determinant then have even sizes) and the state record, its fields and the
// workspace 16-byte aligned.
static bool detA_pair(const fire_handle* h, const void* state, const void* ws) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  return D.nu % 2 == 0 && D.nd % 2 == 0 && (S.stride | S.inv | S.env | S.phi) % 16 == 0 &&
         (uintptr_t)state % 16 == 0 && (uintptr_t)ws % 16 == 0;
}

// Acceptance: psi'/psi = sum_d s_d e^{l_d} prod_s det A_ds / sum_d s_d e^{l_d};
// accept iff u < (psi'/psi)^2, times rho(r_e)/rho(r_e') = e^lqf for a global
// jump (lqf NULL for local moves).  Updates the determinant logs and log|psi|.
__global__ void k_accept(const Dims D, int W, int e, double* __restrict__ R, const double* __restrict__ rnew,
                         const double* __restrict__ lqf, const double* __restrict__ dj,
                         const double* __restrict__ unif,
                         char* __restrict__ state, StateRec S,
                         const double* __restrict__ detA, int32_t* __restrict__ status, int* __restrict__ acc,
                         int32_t* __restrict__ n_accept) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  char* rec = state + (int64_t)w * S.stride;
  double* ds = (double*)(rec + S.dsign);
  double* dl = (double*)(rec + S.dlog);
  const double lp = *(double*)(rec + S.lpsi);
  const double* dA = detA + (int64_t)w * D.K * 4;
  double lmax = -INFINITY;
  for (int k = 0; k < D.K; ++k) {
    double sg = ds[2 * k] * ds[2 * k + 1] * dA[4 * k] * dA[4 * k + 2];
    double l = dl[2 * k] + dl[2 * k + 1] + dA[4 * k + 1] + dA[4 * k + 3];
    if (sg != 0.0 && l > lmax) lmax = l;
  }
  double tot = 0.0;
  for (int k = 0; k < D.K; ++k) {
    double sg = ds[2 * k] * ds[2 * k + 1] * dA[4 * k] * dA[4 * k + 2];
    if (sg != 0.0) tot += sg * exp(dl[2 * k] + dl[2 * k + 1] + dA[4 * k + 1] + dA[4 * k + 3] - lmax);
  }
  int a = 0;
  double lpn = 0.0;
  if (status[w] == 0 && tot != 0.0 && isfinite(tot) && isfinite(lmax)) {
    lpn = lmax + log(fabs(tot));
    const double ratio2 = exp(2.0 * (lpn - lp + dj[w]) + (lqf ? lqf[w] : 0.0));
    a = unif[w] < ratio2;
  }
  acc[w] = a;
  if (!a) return;
  for (int k = 0; k < D.K; ++k)
    for (int s = 0; s < 2; ++s) {
      ds[2 * k + s] *= dA[4 * k + 2 * s];
      dl[2 * k + s] += dA[4 * k + 2 * s + 1];
    }
  *(double*)(rec + S.lpsi) = lpn;
  *(double*)(rec + S.spsi) = tot > 0 ? 1.0 : -1.0;
  *(double*)(rec + S.jas) += dj[w];
  R[((int64_t)w * D.n + e) * 3 + 0] = rnew[3 * w];
  R[((int64_t)w * D.n + e) * 3 + 1] = rnew[3 * w + 1];
  R[((int64_t)w * D.n + e) * 3 + 2] = rnew[3 * w + 2];
  n_accept[w] += 1;
}

// Woodbury update of G for one accepted (walker, determinant, spin block)
// with |U_s| <= KS, in one workgroup (Methods, low-rank wave function
// updates; with G = Phi^-T the update reads G' = G - (G dPhi_U^T) A^-T G_U):
//   stage dPhi_U and G_U in LDS, A = I + dPhi_U G_U^T, A^-1 by Gauss-Jordan,
//   B = A^-T G_U (kept in LDS), commit the new Phi rows, then stream G in
//   blocks of WB_RB rows: Z = G_blk dPhi_U^T, G_blk -= Z B.
// Larger update sets use k_woodbury_prep + k_woodbury_rows.
template <typename T, typename TI, int KSM>
__global__ __launch_bounds__(256, KSM > 16 ? 3 : 5) void k_woodbury(const Dims D, int W, int s, const int* __restrict__ uidx, int capmax,
                                                  const int* __restrict__ ucnt, const int* __restrict__ off,
                                                  const int* __restrict__ acc, const T* __restrict__ dphi,
                                                  const T* __restrict__ oseg, char* __restrict__ state, StateRec S,
                                                  int32_t* status) {
  extern __shared__ double lds[];
  __shared__ int perm[KSM];
  __shared__ double sc[2];
  __shared__ int fl[2];
  const int w = blockIdx.x / D.K, det = blockIdx.x % D.K;
  const int k = ucnt[2 * w + s];
  // this instance takes update sets of (KSM/2, KSM] rows (KSM = 16: 1..16)
  if (!acc[w] || k == 0 || k > KSM || (KSM > 16 && k <= 16)) return;
  const int N = D.nsig(s);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int LD = k + 1;
  // LDS: GU [KSM][N] (later the per-wave Z tiles), B [KSM][N],
  // A [KSM][KSM+1], f [KSM], P [KSM][N] in T
  double* GU = lds;
  double* B = GU + (KSM * N > 4 * 16 * 33 ? KSM * N : 4 * 16 * 33);
  double* Ai = B + KSM * N;
  double* f = Ai + KSM * (KSM + 1);
  T* P = (T*)(f + KSM);
  const int q0 = off[s * (W + 1) + w];
  const int e0 = s == 0 ? 0 : D.nu;
  const int* lst = uidx + ((int64_t)w * 2 + s) * capmax;
  const int KN = D.K * N;
  char* rec = state + (int64_t)w * S.stride;
  TI* G = (TI*)(rec + S.inv) + det * phi_per_det(D) + phi_block_off(D, s);
  T* phi = (T*)(rec + S.phi) + det * phi_per_det(D) + phi_block_off(D, s);
  const T* dp = dphi + (int64_t)q0 * KN + det * N;
  // staging reads four elements per thread at a time, all issued before the
  // LDS writes (indices clamped into the k x N block, writes guarded)
  const int kN = k * N;
  for (int qs = tid; qs < kN; qs += 4 * nt) {
    T pv[4];
    TI gv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = qs + j * nt < kN ? qs + j * nt : kN - 1;
      const int a = q / N, l = q - a * N;
      pv[j] = dp[(int64_t)a * KN + l];
      gv[j] = G[(int64_t)(lst[a] - e0) * N + l];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = qs + j * nt;
      if (q < kN) {
        P[q] = pv[j];
        GU[q] = (double)gv[j];
      }
    }
  }
  __syncthreads();
  // Z = G_rows dPhi_U^T for the 16 rows from m0 (K = N) on f64 MFMA tiles;
  // f64 MFMA layouts: A lane (r, q) holds A[r][q], B lane (r, q) holds
  // B[q][r], the output register i of lane (r, q) holds C[4 i + q][r]
  const int KT = k > 16 ? 2 : 1;
  auto zrows = [&](int m0, d4v_& z0, d4v_& z1) {
    const int lane = tid & 63, r16 = lane & 15, kq = lane >> 4;
    const int mrow = m0 + r16;
    z0 = d4v_{0.0, 0.0, 0.0, 0.0};
    z1 = d4v_{0.0, 0.0, 0.0, 0.0};
    for (int cb = 0; cb < N; cb += 32) {
      double ga[8], pa0[8], pa1[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int col = cb + 4 * u + kq;
        const bool cin = col < N;
        ga[u] = (cin && mrow < N) ? (double)G[(int64_t)mrow * N + col] : 0.0;
        pa0[u] = (cin && r16 < k) ? (double)P[r16 * N + col] : 0.0;
        pa1[u] = (cin && 16 + r16 < k) ? (double)P[(16 + r16) * N + col] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (cb + 4 * u >= N) break;
        z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[u], pa0[u], z0, 0, 0, 0);
        if (KT > 1) z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[u], pa1[u], z1, 0, 0, 0);
      }
    }
  };
  // Z of row chunk `wave` (waves 1..3), computed while wave 0 is busy below
  d4v_ zp0 = {0.0, 0.0, 0.0, 0.0}, zp1 = {0.0, 0.0, 0.0, 0.0};
  {
    // wave 0 forms A on MFMA, inverts it in registers and forms B on MFMA;
    // waves 1..3 form Z for their first row chunk, then all wait at the
    // barrier below
    constexpr int NT = KSM / 16;          // 16-row tiles of A
    constexpr int LA = KSM + 1;           // row stride of A in LDS
    if (tid >= 64) {
      const int w3 = tid >> 6;
      if (w3 * 16 < N) zrows(w3 * 16, zp0, zp1);
    } else {
      const int lane = tid, r16 = lane & 15, kq = lane >> 4;
      // A = I + P G_U^T (rows and columns past k zero)
      d4v_ am[NT][NT];
#pragma unroll
      for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y) am[x][y] = d4v_{0.0, 0.0, 0.0, 0.0};
      for (int c0 = 0; c0 < N; c0 += 4) {
        const int col = c0 + kq;
        double pv[NT], gv[NT];
#pragma unroll
        for (int x = 0; x < NT; ++x) {
          const int r = 16 * x + r16;
          const bool ok = r < k && col < N;
          pv[x] = ok ? (double)P[r * N + col] : 0.0;
          gv[x] = ok ? GU[r * N + col] : 0.0;
        }
#pragma unroll
        for (int x = 0; x < NT; ++x)
#pragma unroll
          for (int y = 0; y < NT; ++y) am[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(pv[x], gv[y], am[x][y], 0, 0, 0);
      }
#pragma unroll
      for (int x = 0; x < NT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y)
#pragma unroll
          for (int i = 0; i < 4; ++i) Ai[(16 * x + 4 * i + kq) * LA + 16 * y + r16] = am[x][y][i];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      // Gauss-Jordan inversion in place, lane r holds row r of A; pivots are
      // chosen among the unused rows by magnitude (no row moves).  Step p
      // with pivot row i: row i is divided by the pivot, its column p taking
      // 1 / pivot, and every other row subtracts its column-p entry times the
      // new row i, its column p taking minus that entry over the pivot.
      // Columns past k are zero and skipped in groups of four (k is
      // wave-uniform).  Afterwards the row that pivoted column p holds row p
      // of A^-1 with its columns in pivot order: entry c is A^-1[p][piv[c]].
      double row[KSM];
#pragma unroll
      for (int c = 0; c < KSM; ++c)
        row[c] = (lane < k && c < k) ? Ai[lane * LA + c] + (c == lane ? 1.0 : 0.0) : 0.0;
      const int ku = __builtin_amdgcn_readfirstlane(k);
      uint32_t unused = ku >= 32 ? 0xffffffffu : ((1u << ku) - 1u);
      int mycol = 0;
      int piv[KSM];
      bool sing = false;
#pragma unroll
      for (int p = 0; p < KSM; ++p) {
        piv[p] = 0;
        if (p < ku && !sing) {
          const bool cand = lane < 32 && ((unused >> (lane & 31)) & 1u);
          const float av = (float)fabs(row[p]);
          const uint32_t key = cand ? ((__float_as_uint(av) & ~31u) | (uint32_t)(31 - lane)) : 0u;
          const uint32_t best = (uint32_t)__builtin_amdgcn_readfirstlane((int)lanes32_max(key));
          const int idx = 31 - (int)(best & 31u);
          const double pv = readlane_f64(row[p], idx);
          if ((best & ~31u) == 0u || !(fabs(pv) > 0.0)) {
            sing = true;
          } else {
            unused &= ~(1u << idx);
            piv[p] = idx;
            const bool me = lane == idx;
            if (me) mycol = p;
            const double ip = 1.0 / pv;
            if (me) {
#pragma unroll
              for (int c = 0; c < KSM; ++c)
                if ((c & ~3) < ku) row[c] = (c == p ? 1.0 : row[c]) * ip;
            }
            const double fr = (me || lane >= ku) ? 0.0 : row[p];
#pragma unroll
            for (int c0 = 0; c0 < KSM; c0 += 4) {
              if (c0 < ku) {
                double pr[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) pr[t] = readlane_f64(row[c0 + t], idx);
#pragma unroll
                for (int t = 0; t < 4; ++t) row[c0 + t] = ((c0 + t == p && !me) ? 0.0 : row[c0 + t]) - fr * pr[t];
              }
            }
          }
        }
      }
      if (sing) {
        if (lane == 0) { fl[1] = 1; atomicOr(status + w, FIRE_W_SINGULAR); }
      } else {
        if (lane == 0) fl[1] = 0;
        // each pivot lane stores its row of A^-1 transposed (Ai = (A^-1)^T),
        // undoing the pivot order of the columns
        if (lane < ku)
#pragma unroll
          for (int c = 0; c < KSM; ++c) {
            if (c < ku) Ai[piv[c] * LA + mycol] = row[c];
            else Ai[c * LA + mycol] = 0.0;
          }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      if (!sing) {
        // B = (A^-1)^T G_U, 16 columns of N per tile, K = |U_s|
        double at[NT][KSM / 4];
#pragma unroll
        for (int x = 0; x < NT; ++x)
#pragma unroll
          for (int s4 = 0; s4 < KSM / 4; ++s4) {
            const int b = 4 * s4 + kq;
            at[x][s4] = b < k ? Ai[(16 * x + r16) * LA + b] : 0.0;
          }
        for (int c0 = 0; c0 < N; c0 += 16) {
          const int col = c0 + r16;
          double gv[KSM / 4];
#pragma unroll
          for (int s4 = 0; s4 < KSM / 4; ++s4) {
            const int b = 4 * s4 + kq;
            gv[s4] = (b < k && col < N) ? GU[b * N + col] : 0.0;
          }
#pragma unroll
          for (int x = 0; x < NT; ++x) {
            d4v_ bm = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < KSM / 4; ++s4) bm = __builtin_amdgcn_mfma_f64_16x16x4f64(at[x][s4], gv[s4], bm, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int a = 16 * x + 4 * i + kq;
              if (a < k && col < N) B[a * N + col] = bm[i];
            }
          }
        }
      }
    }
    __syncthreads();
    if (fl[1]) return;
  }
  // commit the new Phi rows of this determinant and spin block (reads of
  // four elements per thread issued together)
  for (int qa = tid; qa < kN; qa += 4 * nt) {
    T ov[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = qa + j * nt < kN ? qa + j * nt : kN - 1;
      const int a = q / N, l = q - a * N;
      ov[j] = oseg[(int64_t)(q0 + a) * KN + det * N + l];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = qa + j * nt;
      if (q < kN) {
        const int a = q / N, l = q - a * N;
        phi[(int64_t)(lst[a] - e0) * N + l] = ov[j];
      }
    }
  }
  __syncthreads();
  // G -= Z B in 16-row chunks, one wave per chunk, on 16x16x4 f64 MFMA
  // tiles: Z = G_rows dPhi_U^T (K = N), then each 16x16 tile of G is loaded
  // as the accumulator and Z B subtracted (K = |U_s|).  Chunk c < 4 is wave
  // c's (waves 1..3 already hold its Z); chunks from 4 on go to waves 1..3
  // in turn, since wave 0 spent the precomputation on A and B.
  const int lane = tid & 63, wave = tid >> 6, r16 = lane & 15, kq = lane >> 4;
  double* Zs = GU + wave * (16 * 33);   // this wave's Z tile [16][16 KT]
  const int nch = (N + 15) / 16;
  for (int ch = wave; ch < nch; ch = ch < 4 ? (wave == 0 ? nch : wave + 3) : ch + 3) {
    const int m0 = ch * 16;
    d4v_ z0, z1;
    if (ch == wave && wave > 0) {
      z0 = zp0;
      z1 = zp1;
    } else {
      zrows(m0, z0, z1);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Zs[(4 * i + kq) * 33 + r16] = z0[i];
      Zs[(4 * i + kq) * 33 + 16 + r16] = KT > 1 ? z1[i] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double za[8];
#pragma unroll
    for (int s4 = 0; s4 < 8; ++s4) za[s4] = -Zs[r16 * 33 + 4 * s4 + kq];
    // four 16-column tiles at a time: all their G loads are issued first
    for (int cq = 0; cq < N; cq += 64) {
      d4v_ accs[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = cq + 16 * t + r16;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = m0 + 4 * i + kq;
          accs[t][i] = (r < N && col < N) ? (double)G[(int64_t)r * N + col] : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = cq + 16 * t + r16;
        if (cq + 16 * t >= N) break;
#pragma unroll
        for (int s4 = 0; s4 < 8; ++s4) {
          if (s4 >= 4 * KT) break;
          const int a = 4 * s4 + kq;
          const double bv = (a < k && col < N) ? B[a * N + col] : 0.0;
          accs[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(za[s4], bv, accs[t], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = m0 + 4 * i + kq;
          if (r < N && col < N) G[(int64_t)r * N + col] = (TI)accs[t][i];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

// Woodbury update of G for accepted walkers, in two kernels:
//   k_woodbury_prep (per walker, determinant, spin block): A, A^-1 and
//     B = A^-T G_U (k x N, into the workspace), and the commit of Phi rows;
//   k_woodbury_rows (per block of WB_RB rows of G): Z = G dPhi_U^T and
//     G' = G - Z B, one read and one write of every row of G.
template <typename T, typename TI>
__global__ __launch_bounds__(256) void k_woodbury_prep(const Dims D, int W, int s, const int* __restrict__ uidx,
                                                       int capmax, const int* __restrict__ ucnt,
                                                       const int* __restrict__ off, const int* __restrict__ acc,
                                                       const T* __restrict__ dphi, const T* __restrict__ oseg,
                                                       double* __restrict__ Bbuf, char* __restrict__ state,
                                                       StateRec S, int32_t* status, int kmin) {
  extern __shared__ double lds[];
  __shared__ int perm[128];
  __shared__ double sc[2];
  __shared__ int fl[2];
  const int w = blockIdx.x / D.K, det = blockIdx.x % D.K;
  const int k = ucnt[2 * w + s];
  if (!acc[w] || k == 0 || k < kmin) return;
  const int N = D.nsig(s);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int LD = k + 1;
  double* Ai = lds;               // [k][k+1]
  double* f = Ai + k * LD;        // [k]
  const int q0 = off[s * (W + 1) + w];
  const int e0 = s == 0 ? 0 : D.nu;
  const int* lst = uidx + ((int64_t)w * 2 + s) * capmax;
  const int KN = D.K * N;
  char* rec = state + (int64_t)w * S.stride;
  const TI* G = (const TI*)(rec + S.inv) + det * phi_per_det(D) + phi_block_off(D, s);
  T* phi = (T*)(rec + S.phi) + det * phi_per_det(D) + phi_block_off(D, s);
  build_A<T, TI>(Ai, LD, k, N, dphi + (int64_t)q0 * KN + det * N, KN, G, lst, e0);
  __syncthreads();
  gj_block(Ai, k, LD, f, perm, sc, fl, true);
  if (fl[1]) {
    if (tid == 0) atomicOr(status + w, FIRE_W_SINGULAR);
    return;
  }
  // B[a][l] = sum_b (A^-1)[b][a] G[u_b][l]
  double* B = Bbuf + (int64_t)q0 * KN + det * N;
  for (int q = tid; q < k * N; q += nt) {
    const int a = q / N, l = q % N;
    double v = 0.0;
    for (int b = 0; b < k; ++b) v += Ai[b * LD + a] * (double)G[(int64_t)(lst[b] - e0) * N + l];
    B[(int64_t)a * KN + l] = v;
  }
  // commit the new Phi rows of this determinant and spin block
  for (int q = tid; q < k * N; q += nt) {
    const int a = q / N, l = q % N;
    phi[(int64_t)(lst[a] - e0) * N + l] = oseg[(int64_t)(q0 + a) * KN + det * N + l];
  }
}

template <typename T, typename TI>
FIRE_DEV void woodbury_rows_item(const Dims& D, int W, int s, int rb, int det, int w, const int* __restrict__ ucnt,
                                 const int* __restrict__ off, const int* __restrict__ acc,
                                 const T* __restrict__ dphi, const double* __restrict__ Bbuf,
                                 char* __restrict__ state, const StateRec& S, const int32_t* __restrict__ status,
                                 int kmin, double* lds);
template <typename T, typename TI>
__global__ __launch_bounds__(256) void k_woodbury_rows(const Dims D, int W, int s, const int* __restrict__ ucnt,
                                                       const int* __restrict__ off, const int* __restrict__ acc,
                                                       const T* __restrict__ dphi, const double* __restrict__ Bbuf,
                                                       char* __restrict__ state, StateRec S,
                                                       const int32_t* __restrict__ status, int kmin) {
  extern __shared__ double lds[];
  const int N = D.nsig(s);
  const int nrb = (N + WB_RB - 1) / WB_RB;
  // grid-stride over walkers, each checked once: the large update sets
  // this kernel takes are rare, so a small grid skips the rest cheaply;
  // a walker that has one gets all its (determinant, row block) items
  for (int w = blockIdx.x; w < W; w += gridDim.x) {
    const int k = ucnt[2 * w + s];
    if (!acc[w] || k == 0 || k < kmin || (status[w] & FIRE_W_SINGULAR)) continue;
    for (int t = 0; t < D.K * nrb; ++t) {
      __syncthreads();
      woodbury_rows_item<T, TI>(D, W, s, t % nrb, t / nrb, w, ucnt, off, acc, dphi, Bbuf, state, S, status, kmin,
                                lds);
    }
  }
}

template <typename T, typename TI>
FIRE_DEV void woodbury_rows_item(const Dims& D, int W, int s, int rb, int det, int w, const int* __restrict__ ucnt,
                                 const int* __restrict__ off, const int* __restrict__ acc,
                                 const T* __restrict__ dphi, const double* __restrict__ Bbuf,
                                 char* __restrict__ state, const StateRec& S, const int32_t* __restrict__ status,
                                 int kmin, double* lds) {
  const int N = D.nsig(s);
  const int k = ucnt[2 * w + s];
  if (!acc[w] || k == 0 || k < kmin || (status[w] & FIRE_W_SINGULAR)) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int q0 = off[s * (W + 1) + w];
  const int KN = D.K * N;
  TI* G = (TI*)(state + (int64_t)w * S.stride + S.inv) + det * phi_per_det(D) + phi_block_off(D, s);
  const T* dp = dphi + (int64_t)q0 * KN + det * N;
  const double* B = Bbuf + (int64_t)q0 * KN + det * N;
  const int m0 = rb * WB_RB;
  const int rows = N - m0 < WB_RB ? N - m0 : WB_RB;
  if (k <= KS) {
    double* Ps = lds;                 // [k][N]
    double* Bs = Ps + KS * N;         // [k][N]
    double* Gr = Bs + KS * N;         // [rows][N]
    double* Z = Gr + WB_RB * N;       // [rows][k]
    for (int q = tid; q < k * N; q += nt) {
      const int a = q / N, l = q - a * N;
      Ps[q] = (double)dp[(int64_t)a * KN + l];
      Bs[q] = B[(int64_t)a * KN + l];
    }
    for (int q = tid; q < rows * N; q += nt) Gr[q] = (double)G[(int64_t)m0 * N + q];
    __syncthreads();
    for (int q = tid; q < rows * k; q += nt) {
      const int m = q / k, a = q - m * k;
      double v = 0.0;
      for (int l = 0; l < N; ++l) v += Gr[m * N + l] * Ps[a * N + l];
      Z[q] = v;
    }
    __syncthreads();
    for (int q = tid; q < rows * N; q += nt) {
      const int m = q / N, l = q - m * N;
      double v = Gr[q];
      for (int a = 0; a < k; ++a) v -= Z[m * k + a] * Bs[a * N + l];
      G[(int64_t)m0 * N + q] = (TI)v;
    }
    return;
  }
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (int m = m0 + wave; m < m0 + rows; m += nw) {
    TI* gm = G + (int64_t)m * N;
    double g0 = lane < N ? (double)gm[lane] : 0.0;
    double g1 = lane + 64 < N ? (double)gm[lane + 64] : 0.0;
    double n0 = g0, n1 = g1;
    for (int a = 0; a < k; ++a) {
      const T* pa = dp + (int64_t)a * KN;
      double z = g0 * (lane < N ? (double)pa[lane] : 0.0) + g1 * (lane + 64 < N ? (double)pa[lane + 64] : 0.0);
      z = wave_sum(z);
      const double* ba = B + (int64_t)a * KN;
      if (lane < N) n0 -= z * ba[lane];
      if (lane + 64 < N) n1 -= z * ba[lane + 64];
    }
    if (lane < N) gm[lane] = (TI)n0;
    if (lane + 64 < N) gm[lane + 64] = (TI)n1;
  }
}

// Commit h0_e, projections of e, messages of U and the envelopes of e.
template <typename T>
__global__ __launch_bounds__(256) void k_commit(const Dims D, int W, int e, const int* __restrict__ acc,
                                                const int* __restrict__ uidx, int capmax,
                                                const int* __restrict__ ucnt, const int* __restrict__ off,
                                                const T* __restrict__ h0new, const T* __restrict__ projnew,
                                                const T* __restrict__ mseg0, const T* __restrict__ mseg1,
                                                const T* __restrict__ envnew, char* __restrict__ state, StateRec S) {
  const int w = blockIdx.x;
  if (!acc[w]) return;
  char* rec = state + (int64_t)w * S.stride;
  T* h0 = (T*)(rec + S.h0);
  T* proj = (T*)(rec + S.proj);
  T* m = (T*)(rec + S.m);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int c = tid; c < D.d; c += nt) h0[(int64_t)e * D.d + c] = h0new[(int64_t)w * D.d + c];
  for (int c = tid; c < 4 * D.d; c += nt) proj[(int64_t)e * 4 * D.d + c] = projnew[(int64_t)w * 4 * D.d + c];
  for (int s = 0; s < 2; ++s) {
    const int cnt = ucnt[2 * w + s];
    const int q0 = off[s * (W + 1) + w];
    const int* lst = uidx + ((int64_t)w * 2 + s) * capmax;
    const T* ms = s == 0 ? mseg0 : mseg1;
    for (int q = tid; q < cnt * D.d; q += nt) {
      const int t = q / D.d, c = q % D.d;
      m[(int64_t)lst[t] * D.d + c] = ms[(int64_t)(q0 + t) * D.d + c];
    }
  }
  const int se = e < D.nu ? 0 : 1;
  const int N = D.nsig(se);
  const int iloc = se == 0 ? e : e - D.nu;
  T* env = (T*)(rec + S.env);
  for (int q = tid; q < D.K * N; q += nt) {
    const int det = q / N, l = q % N;
    env[det * phi_per_det(D) + phi_block_off(D, se) + (int64_t)iloc * N + l] = envnew[(int64_t)w * D.K * N + q];
  }
}

__global__ void k_final_outputs(const Dims D, int W, const char* __restrict__ state, StateRec S,
                                const int32_t* __restrict__ status, double* logpsi, double* sign) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const char* rec = state + (int64_t)w * S.stride;
  const bool bad = status[w] != 0;
  if (logpsi) logpsi[w] = bad ? NAN : *(const double*)(rec + S.lpsi) + *(const double*)(rec + S.jas);
  double sp = *(const double*)(rec + S.spsi);
  if (D.Hj > 0 && ((const double*)(rec + S.jms))[1] < 0.0) sp = -sp;
  if (D.Ra > 0 && ((const double*)(rec + S.jat))[2 * D.Ra + D.NV() + 1] < 0.0) sp = -sp;
  if (sign) sign[w] = bad ? 0.0 : sp;
}

__global__ void k_unit_detA(int nwd, int s, double* detA) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nwd) return;
  detA[(int64_t)q * 4 + 2 * s] = 1.0;
  detA[(int64_t)q * 4 + 2 * s + 1] = 0.0;
}

// ---------------------------------------------------------------------------
// one single-electron proposal for all walkers (shared by Metropolis and the
// pseudopotential quadrature, which stops after det A)
// ---------------------------------------------------------------------------
template <typename T>
hipError_t propose_ratio(const fire_handle* h, const Net<T>& P, const Jobs& jb, int e, const double* R,
                         char* state, char* ws, int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  const int W = jb.J;
  const UpdLayout L = upd_layout(h, jb.Jcap > 0 ? jb.Jcap : jb.J, jb.woodbury);
  const int se = e < D.nu ? 0 : 1;
  const int blk = D.d <= 64 ? 64 : (D.d + 63) / 64 * 64;
  double* rnew = (double*)(ws + L.rnew);
  int* uidx = (int*)(ws + L.uidx);
  int* ucnt = (int*)(ws + L.ucnt);
  int* off = (int*)(ws + L.off);
  T* y = (T*)(ws + L.y);
  T* ug = (T*)(ws + L.ug);
  T* h0new = (T*)(ws + L.h0new);
  T* projnew = (T*)(ws + L.projnew);
  T* basis = (T*)(ws + L.basis);
  T* envnew = (T*)(ws + L.envnew);

  hipLaunchKernelGGL(k_propose, dim3((W + 3) / 4), dim3(256), 0, st, R, jb, D.n, D.nu, e, D.cut * D.cut,
                     L.capS[0], L.capS[1], L.capmax, rnew, uidx, ucnt, P.jas, (double*)(ws + L.dj), status);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, ucnt, W, off, L.rowcap[0], L.rowcap[1], jb.jw,
                     status, jb.Jdev);
  CHECK(hipGetLastError());
  // h0 and projections of the moved electron
  const int epb = W >= 16384 ? 4 : (W >= 4096 ? 2 : 1);
  hipLaunchKernelGGL((k_en_embed<T, 2>), dim3((W + epb - 1) / epb), dim3(blk), 0, st, P, (const double*)rnew,
                     (int64_t)W, y, epb, jb.Jdev);
  CHECK(hipGetLastError());
  {
    GemmArgs g{};
    g.A = y; g.amap = rows_dense(D.d); g.Bt = P.Wvg_t; g.ldb = D.d; g.bias = P.b_vg;
    g.C = ug; g.cmap = rows_dense(2 * D.d); g.ccol = cols_dense(); g.M = W; g.N = 2 * D.d; g.K = D.d;
    g.Mdev = jb.Jdev;
    CHECK(gemm_site(h, SITE_EMB, g, st));
  }
  hipLaunchKernelGGL(k_glu<T>, dim3((unsigned)(((int64_t)W * D.d + 255) / 256)), dim3(256), 0, st, ug, y,
                     (int64_t)W, D.d, jb.Jdev);
  CHECK(hipGetLastError());
  {
    GemmArgs g{};
    g.A = y; g.amap = rows_dense(D.d); g.Bt = P.Wo_t; g.ldb = D.d; g.bias = P.b_o;
    g.C = h0new; g.cmap = rows_dense(D.d); g.ccol = cols_dense(); g.M = W; g.N = D.d; g.K = D.d;
    g.Mdev = jb.Jdev;
    CHECK(gemm_site(h, SITE_EMB, g, st));
    GemmArgs p{};
    p.A = h0new; p.amap = rows_dense(D.d); p.Bt = P.Wproj_t; p.ldb = D.d;
    p.C = projnew; p.cmap = rows_dense(4 * D.d); p.ccol = cols_dense(); p.M = W; p.N = 4 * D.d; p.K = D.d;
    p.Mdev = jb.Jdev;
    CHECK(gemm_site(h, SITE_EMB, p, st));
  }
  T* hs[2][2];
  T* ms[2];
  int* ri[2];
  for (int s = 0; s < 2; ++s) {
    hs[s][0] = (T*)(ws + L.hseg[s][0]);
    hs[s][1] = (T*)(ws + L.hseg[s][1]);
    ms[s] = (T*)(ws + L.mseg[s]);
    ri[s] = (int*)(ws + L.rowinfo[s]);
  }
  hipLaunchKernelGGL(k_msg_update<T>, dim3(W), dim3(blk), 0, st, P, W, jb.jw, e, R, (const double*)rnew,
                     (const int*)uidx, L.capmax, (const int*)ucnt, (const int*)off, (const char*)state, S,
                     (const T*)h0new, (const T*)projnew, hs[0][0], hs[1][0], ms[0], ms[1], ri[0], ri[1]);
  CHECK(hipGetLastError());
  // envelopes of the moved electron at r_e'
  hipLaunchKernelGGL(k_env_basis<T>, dim3((unsigned)(((int64_t)W * D.B + 255) / 256)), dim3(256), 0, st, P,
                     (const double*)rnew, (int64_t)W, basis, jb.Jdev);
  CHECK(hipGetLastError());
  {
    const int N = D.nsig(se);
    GemmArgs g{};
    g.A = basis; g.amap = rows_dense(D.B); g.Bt = se == 0 ? P.pi0 : P.pi1; g.ldb = D.B;
    g.C = envnew; g.cmap = rows_dense((int64_t)D.K * N); g.ccol = cols_dense(); g.M = W; g.N = D.K * N; g.K = D.B;
    g.Mdev = jb.Jdev;
    CHECK(gemm_site(h, SITE_ORB, g, st));
  }
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s);
    if (N == 0) continue;
    const int* Mdev = off + s * (W + 1) + W;
    const int rows = (int)L.rowcap[s];
    T* hin = hs[s][0];
    T* hout = hs[s][1];
    for (int k = 0; k < D.L; ++k) {
      GemmArgs g{};
      g.A = hin; g.amap = rows_dense(D.d);
      g.Bt = (const char*)P.mlp_t + (size_t)k * D.d * D.d * h->gsize; g.ldb = D.d;
      g.bias = P.mlp_b + (int64_t)k * D.d; g.C = hout; g.cmap = rows_dense(D.d); g.ccol = cols_dense();
      g.M = rows; g.N = D.d; g.K = D.d; g.act = ACT_SILU; g.Mdev = Mdev;
      CHECK(gemm_site(h, SITE_EMB, g, st));
      T* t = hin; hin = hout; hout = t;
    }
    if (D.Hj > 0) CHECK(jm_rows<T>(h, P, hin, rows, Mdev, ws + L.jscr, (double*)(ws + L.jnew[s]), st));
    if (D.Ra > 0) {
      GemmArgs ga{};
      ga.A = hin; ga.amap = rows_dense(D.d); ga.Bt = P.ja_Pt; ga.ldb = D.d;
      ga.C = ws + L.anew[s]; ga.cmap = rows_dense(D.NA()); ga.ccol = cols_dense(); ga.M = rows; ga.N = D.NA();
      ga.K = D.d; ga.Mdev = Mdev;
      CHECK(gemm_site(h, SITE_EMB, ga, st));
    }
    T* oseg = (T*)(ws + L.oseg[s]);
    GemmArgs o{};
    o.A = hin; o.amap = rows_dense(D.d); o.Bt = s == 0 ? P.orb_t0 : P.orb_t1; o.ldb = D.d;
    o.C = oseg; o.cmap = rows_dense((int64_t)D.K * N); o.ccol = cols_dense();
    o.M = rows; o.N = D.K * N; o.K = D.d; o.Mdev = Mdev;
    CHECK(gemm_site(h, SITE_ORB, o, st));
    const int fused = jb.woodbury ? 0 : 1;   // Metropolis keeps dPhi for the Woodbury update
    if (!fused) {
      hipLaunchKernelGGL((k_dphi<T>), dim3((unsigned)rows), dim3(256), 0, st, D, s, e, jb.jw,
                         (const int*)ri[s], Mdev, oseg, (const char*)state, S, (const T*)envnew,
                         (T*)(ws + L.dphi[s]));
      CHECK(hipGetLastError());
    }
    const int jg = jb.group > 0 ? jb.group : 1;
    const int64_t items = (int64_t)((W + jg - 1) / jg) * jg * D.K;
    const int64_t quads = (items + 3) / 4;
    // grids of whole runs of eight (det_grid) for the run-wise XCD order
    const bool pair = detA_pair(h, state, ws);
    hipLaunchKernelGGL(detA_kernel<T>(h, false, fused, pair), dim3(det_grid((quads + 3) / 4, jg, D.K, 16)), dim3(256),
                       0, st, D, W, jb.jw, s, e, (const int*)uidx, L.capmax, (const int*)ucnt, (const int*)off,
                       (const T*)(ws + L.dphi[s]), (const T*)oseg, (const T*)envnew, (const char*)state, S,
                       (double*)(ws + L.detA), jg);
    CHECK(hipGetLastError());
    if (L.capS[s] > 16) {
      hipLaunchKernelGGL(detA_kernel<T>(h, true, fused, pair), dim3(det_grid((items + 3) / 4, jg, D.K, 4)), dim3(256),
                         0, st, D, W, jb.jw, s, e, (const int*)uidx, L.capmax, (const int*)ucnt, (const int*)off,
                         (const T*)(ws + L.dphi[s]), (const T*)oseg, (const T*)envnew, (const char*)state, S,
                         (double*)(ws + L.detA), jg);
      CHECK(hipGetLastError());
    }
    if (L.capS[s] > 32) {
      const size_t lds = detA_lds(L.capmax);
      const unsigned nblk = (unsigned)(W < 2048 ? W : 2048);
      const T* dp = fused ? nullptr : (const T*)(ws + L.dphi[s]);
      if (h->isize == 8) {
        CHECK(hipFuncSetAttribute((const void*)k_detA<T, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
        hipLaunchKernelGGL((k_detA<T, double>), dim3(nblk), dim3(256), lds, st, D, W, jb.jw, s, e, (const int*)uidx,
                           L.capmax, (const int*)ucnt, (const int*)off, dp, (const T*)oseg, (const T*)envnew,
                           (const char*)state, S, (double*)(ws + L.detA), jg);
      } else {
        CHECK(hipFuncSetAttribute((const void*)k_detA<T, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
        hipLaunchKernelGGL((k_detA<T, float>), dim3(nblk), dim3(256), lds, st, D, W, jb.jw, s, e, (const int*)uidx,
                           L.capmax, (const int*)ucnt, (const int*)off, dp, (const T*)oseg, (const T*)envnew,
                           (const char*)state, S, (double*)(ws + L.detA), jg);
      }
      CHECK(hipGetLastError());
    }
  }
  // a spin block with no electrons contributes det A = 1
  for (int s = 0; s < 2; ++s)
    if (D.nsig(s) == 0) {
      hipLaunchKernelGGL(k_unit_detA, dim3((W * D.K + 255) / 256), dim3(256), 0, st, W * D.K, s,
                         (double*)(ws + L.detA));
      CHECK(hipGetLastError());
    }
  // the change of log|J_MLP| joins the cusp factor's change in dj
  CHECK(jm_delta(h, W, jb.jw, uidx, L.capmax, ucnt, off, (const double*)(ws + L.jnew[0]),
                 (const double*)(ws + L.jnew[1]), state, (double*)(ws + L.dj), (double*)(ws + L.jsg),
                 (double*)(ws + L.jsum), st));
  CHECK(ja_delta<T>(h, P, W, jb.jw, jb.Jdev, uidx, L.capmax, ucnt, off, (const T*)(ws + L.anew[0]),
                    (const T*)(ws + L.anew[1]), state, ws + L.ja, (double*)(ws + L.dj), (double*)(ws + L.jsg),
                    D.Hj == 0, st));
  return hipSuccess;
}

template <typename T>
static hipError_t accept_and_commit(const fire_handle* h, int W, int e, double* R, const double* unif, bool global,
                                    char* state, char* ws, int32_t* n_accept, int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  const UpdLayout L = upd_layout(h, W);
  int* acc = (int*)(ws + L.acc);
  hipLaunchKernelGGL(k_accept, dim3((W + 127) / 128), dim3(128), 0, st, D, W, e, R, (const double*)(ws + L.rnew),
                     global ? (const double*)(ws + L.lqf) : (const double*)nullptr, (const double*)(ws + L.dj),
                     unif, state, S,
                     (const double*)(ws + L.detA), status, acc, n_accept);
  CHECK(hipGetLastError());
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s);
    if (N == 0) continue;
    // update sets up to KS: one fused workgroup per (walker, determinant);
    // sets of up to 16 rows and of 17..32 rows in two instances (LDS sized
    // for each)
    for (int ksm = 16; ksm <= KS; ksm += 16) {
      if (ksm > 16 && L.capS[s] <= 16) break;
      const size_t lfu = wb_fused_lds(N, (int)h->tsize, ksm);
      const void* fn;
      if (h->isize == 8)
        fn = ksm == 16 ? (const void*)k_woodbury<T, double, 16> : (const void*)k_woodbury<T, double, KS>;
      else
        fn = ksm == 16 ? (const void*)k_woodbury<T, float, 16> : (const void*)k_woodbury<T, float, KS>;
      CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lfu));
      if (h->isize == 8 && ksm == 16)
        hipLaunchKernelGGL((k_woodbury<T, double, 16>), dim3(W * D.K), dim3(256), lfu, st, D, W, s,
                           (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt), (const int*)(ws + L.off),
                           (const int*)acc, (const T*)(ws + L.dphi[s]), (const T*)(ws + L.oseg[s]), state, S, status);
      else if (h->isize == 8)
        hipLaunchKernelGGL((k_woodbury<T, double, KS>), dim3(W * D.K), dim3(256), lfu, st, D, W, s,
                           (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt), (const int*)(ws + L.off),
                           (const int*)acc, (const T*)(ws + L.dphi[s]), (const T*)(ws + L.oseg[s]), state, S, status);
      else if (ksm == 16)
        hipLaunchKernelGGL((k_woodbury<T, float, 16>), dim3(W * D.K), dim3(256), lfu, st, D, W, s,
                           (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt), (const int*)(ws + L.off),
                           (const int*)acc, (const T*)(ws + L.dphi[s]), (const T*)(ws + L.oseg[s]), state, S, status);
      else
        hipLaunchKernelGGL((k_woodbury<T, float, KS>), dim3(W * D.K), dim3(256), lfu, st, D, W, s,
                           (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt), (const int*)(ws + L.off),
                           (const int*)acc, (const T*)(ws + L.dphi[s]), (const T*)(ws + L.oseg[s]), state, S, status);
      CHECK(hipGetLastError());
    }
    if (L.capS[s] <= KS) continue;
    // larger update sets (rare): two kernels through a B buffer
    const size_t lds = detA_lds(L.capS[s]);
    double* Bbuf = (double*)(ws + L.bbuf[s]);
    const int nrb = (N + WB_RB - 1) / WB_RB;
    const int kmin = KS + 1;
    const unsigned wr_grid = (unsigned)(W < 2048 ? W : 2048);
    if (h->isize == 8) {
      hipLaunchKernelGGL((k_woodbury_prep<T, double>), dim3(W * D.K), dim3(256), lds, st, D, W, s,
                         (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt), (const int*)(ws + L.off),
                         (const int*)acc, (const T*)(ws + L.dphi[s]), (const T*)(ws + L.oseg[s]), Bbuf, state,
                         S, status, kmin);
      CHECK(hipGetLastError());
      CHECK(hipFuncSetAttribute((const void*)k_woodbury_rows<T, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)wb_rows_lds(N)));
      hipLaunchKernelGGL((k_woodbury_rows<T, double>), dim3(wr_grid), dim3(256), wb_rows_lds(N), st, D, W, s,
                         (const int*)(ws + L.ucnt), (const int*)(ws + L.off), (const int*)acc,
                         (const T*)(ws + L.dphi[s]), (const double*)Bbuf, state, S, (const int32_t*)status, kmin);
    } else {
      hipLaunchKernelGGL((k_woodbury_prep<T, float>), dim3(W * D.K), dim3(256), lds, st, D, W, s,
                         (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt), (const int*)(ws + L.off),
                         (const int*)acc, (const T*)(ws + L.dphi[s]), (const T*)(ws + L.oseg[s]), Bbuf, state,
                         S, status, kmin);
      CHECK(hipGetLastError());
      CHECK(hipFuncSetAttribute((const void*)k_woodbury_rows<T, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)wb_rows_lds(N)));
      hipLaunchKernelGGL((k_woodbury_rows<T, float>), dim3(wr_grid), dim3(256), wb_rows_lds(N), st, D, W, s,
                         (const int*)(ws + L.ucnt), (const int*)(ws + L.off), (const int*)acc,
                         (const T*)(ws + L.dphi[s]), (const double*)Bbuf, state, S, (const int32_t*)status, kmin);
    }
    CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_commit<T>, dim3(W), dim3(256), 0, st, D, W, e, (const int*)acc, (const int*)(ws + L.uidx),
                     L.capmax, (const int*)(ws + L.ucnt), (const int*)(ws + L.off), (const T*)(ws + L.h0new),
                     (const T*)(ws + L.projnew), (const T*)(ws + L.mseg[0]), (const T*)(ws + L.mseg[1]),
                     (const T*)(ws + L.envnew), state, S);
  CHECK(hipGetLastError());
  CHECK(jm_commit(h, W, acc, (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt),
                  (const int*)(ws + L.off), (const double*)(ws + L.jnew[0]), (const double*)(ws + L.jnew[1]),
                  (const double*)(ws + L.jsum), state, st));
  return ja_commit<T>(h, W, acc, (const int*)(ws + L.uidx), L.capmax, (const int*)(ws + L.ucnt),
                      (const int*)(ws + L.off), (const T*)(ws + L.anew[0]), (const T*)(ws + L.anew[1]), ws + L.ja,
                      state, st);
}

// The random numbers of one sweep from the counter-based generator:
// xi [n][W][3] and u [n][W] for sweep counter c.
__global__ void k_sweep_randoms(int n, int W, uint64_t seed, uint64_t c, double* __restrict__ xi,
                                double* __restrict__ u) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * W) return;
  const int e = (int)(q / W), w = (int)(q % W);
  double x[3], a;
  proposal_randoms(seed, c, e, w, x, a);
  xi[3 * q] = x[0];
  xi[3 * q + 1] = x[1];
  xi[3 * q + 2] = x[2];
  u[q] = a;
}

// Workspace of the generated random numbers of one sweep: after the regions
// of the update and of the periodic full re-evaluation, which share the start
// of the workspace.
size_t rng_ws_offset(const fire_handle* h, int W) {
  const size_t a = upd_layout(h, W).total, b = ws_forward(h, W).total;
  return align_up(a > b ? a : b);
}
size_t rng_ws_bytes(const fire_handle* h, int W) { return align_up((size_t)h->D.n * W * 4 * sizeof(double)); }

template <typename T>
static hipError_t sweep_impl(fire_handle* h, int W, double* R, char* state, char* ws, int n_sweeps, double step,
                             double gstep, const int32_t* kinds, const double* noise, const double* unif,
                             const double* pick, uint64_t seed, uint64_t counter, int32_t* n_accept,
                             double* logpsi, double* sign, int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  Net<T> P = make_net<T>(h);
  CHECK(fill_i32(status, W, 0, st));
  const int refresh = h->model.refresh_every;
  // without explicit random numbers each sweep draws its own into the
  // workspace (counter base + sweep index)
  const bool gen = noise == nullptr;
  double* gxi = (double*)(ws + rng_ws_offset(h, W));
  double* gu = gxi + (int64_t)D.n * W * 3;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    if (gen) {
      hipLaunchKernelGGL(k_sweep_randoms, dim3((unsigned)(((int64_t)D.n * W + 255) / 256)), dim3(256), 0, st, D.n, W,
                         seed, counter + (uint64_t)sw, gxi, gu);
      CHECK(hipGetLastError());
    }
    for (int e = 0; e < D.n; ++e) {
      Jobs jb{};
      jb.J = W;
      jb.woodbury = true;
      jb.xi = gen ? gxi + (int64_t)e * W * 3 : noise + ((int64_t)sw * D.n + e) * W * 3;
      jb.step = step;
      const bool global = kinds && kinds[sw] == 1;
      if (global) {
        jb.pick = pick + ((int64_t)sw * D.n + e) * W;
        jb.gstep = gstep;
        jb.Rn = P.Rn;
        jb.Zn = P.Zn;
        jb.M = D.M;
        jb.lqf = (double*)(ws + upd_layout(h, W).lqf);
      }
      const double* u = gen ? gu + (int64_t)e * W : unif + ((int64_t)sw * D.n + e) * W;
      CHECK(propose_ratio<T>(h, P, jb, e, R, state, ws, status, st));
      CHECK(accept_and_commit<T>(h, W, e, R, u, global, state, ws, n_accept, status, st));
    }
    if (refresh > 0 && (sw + 1) % refresh == 0) {
      // full re-evaluation of every cached quantity from the positions (FP64 LU)
      CHECK(embed_and_orbitals<T>(h, P, W, R, state, ws, status, st));
      CHECK(refresh_dets<T>(h, W, R, state, nullptr, nullptr, status, st));
    }
  }
  hipLaunchKernelGGL(k_final_outputs, dim3((W + 127) / 128), dim3(128), 0, st, D, W, (const char*)state, h->st,
                     (const int32_t*)status, logpsi, sign);
  return hipGetLastError();
}

hipError_t mcmc_sweep_path(fire_handle* h, int W, double* R, char* state, char* ws, int n_sweeps, double step,
                           double gstep, const int32_t* kinds, const double* noise, const double* unif,
                           const double* pick, uint64_t seed, uint64_t counter, int32_t* n_accept, double* logpsi,
                           double* sign, int32_t* status, hipStream_t s) {
  if (!update_fits(h)) return hipErrorInvalidValue;
  return h->tsize == 8 ? sweep_impl<double>(h, W, R, state, ws, n_sweeps, step, gstep, kinds, noise, unif, pick,
                                            seed, counter, n_accept, logpsi, sign, status, s)
                       : sweep_impl<float>(h, W, R, state, ws, n_sweeps, step, gstep, kinds, noise, unif, pick,
                                           seed, counter, n_accept, logpsi, sign, status, s);
}

// ---------------------------------------------------------------------------
// Two-electron swaps for the S+ estimator (SI, low-rank updates in S+
// operator): psi(pi_ab r) / psi(r) for the exchange of the positions of an
// up electron a and a down electron b, one job per walker.  After the swap
// the position r_a carries a down electron and r_b an up one: the nuclear
// part of every embedding is unchanged (h0 is a function of the position, so
// the slot of a takes the cached h0 and projections of b and vice versa), the
// electron pairs that change class are those between a third electron and
// either position, and the determinants change in the rows of
// U = {a, b} u N(r_a) u N(r_b) only: a rank-|U_s| update per spin block,
// with a first in the up list and b first in the down list.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_swap_propose(const double* __restrict__ R, int W, int n, int nu, int ea,
                                                      int eb, double cut2, int cap0, int cap1, int capmax,
                                                      double* __restrict__ ra, double* __restrict__ rb,
                                                      int* __restrict__ uidx, int* __restrict__ ucnt,
                                                      const double* __restrict__ jasq, double* __restrict__ dj,
                                                      int32_t* status) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= W) return;
  const double* Rw = R + (int64_t)j * n * 3;
  const double ax = Rw[3 * ea], ay = Rw[3 * ea + 1], az = Rw[3 * ea + 2];
  const double bx = Rw[3 * eb], by = Rw[3 * eb + 1], bz = Rw[3 * eb + 2];
  if (lane == 0) {
    // new positions: the slot of a (up) at r_b, the slot of b (down) at r_a
    ra[3 * j] = bx; ra[3 * j + 1] = by; ra[3 * j + 2] = bz;
    rb[3 * j] = ax; rb[3 * j + 1] = ay; rb[3 * j + 2] = az;
  }
  // change of log J_cusp: the pairs of a third electron i with either position
  if (jasq[0] == 0.0 && jasq[2] == 0.0) {
    if (lane == 0) dj[j] = 0.0;
  } else {
    double d = 0.0;
    for (int i = lane; i < n; i += 64) {
      if (i == ea || i == eb) continue;
      const double ix = Rw[3 * i], iy = Rw[3 * i + 1], iz = Rw[3 * i + 2];
      const bool up = i < nu;
      const double rA = sqrt((ax - ix) * (ax - ix) + (ay - iy) * (ay - iy) + (az - iz) * (az - iz));
      const double rB = sqrt((bx - ix) * (bx - ix) + (by - iy) * (by - iy) + (bz - iz) * (bz - iz));
      d += jas_u(jasq, up, rB) + jas_u(jasq, !up, rA) - jas_u(jasq, up, rA) - jas_u(jasq, !up, rB);
    }
    d = wave_sum(d);
    if (lane == 0) dj[j] = d;
  }
  int cnt[2] = {1, 1};
  int* u0 = uidx + (int64_t)j * 2 * capmax;
  if (lane == 0) { u0[0] = ea; u0[capmax] = eb; }
  const int cap[2] = {cap0, cap1};
  bool over = false;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + lane;
    bool in = false;
    if (i < n && i != ea && i != eb) {
      const double x = Rw[3 * i], y = Rw[3 * i + 1], z = Rw[3 * i + 2];
      const double d0 = (x - ax) * (x - ax) + (y - ay) * (y - ay) + (z - az) * (z - az);
      const double d1 = (x - bx) * (x - bx) + (y - by) * (y - by) + (z - bz) * (z - bz);
      in = d0 <= cut2 || d1 <= cut2;
    }
    const int si = i < nu ? 0 : 1;
    const uint64_t m = __ballot(in);
    const uint64_t mup = __ballot(in && si == 0);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int pos = si == 0 ? __popcll(mup & below) : __popcll((m & ~mup) & below);
    if (in) {
      const int t = cnt[si] + pos;
      if (t < cap[si]) u0[si * capmax + t] = i;
    }
    cnt[0] += __popcll(mup);
    cnt[1] += __popcll(m & ~mup);
  }
  for (int s = 0; s < 2; ++s)
    if (cnt[s] > cap[s]) { over = true; cnt[s] = cap[s]; }
  if (lane == 0) {
    ucnt[2 * j] = cnt[0];
    ucnt[2 * j + 1] = cnt[1];
    if (over) atomicOr(status + j, FIRE_W_UPD_OVERFLOW);
  }
}

// Messages after the swap, one workgroup per job, one thread per channel.
// For a member u of either list: the edges to the two positions change
// class, m_u += sum_{p in {r_a, r_b}} [msg^new(u, p) - msg^old(u, p)] with
// msg^c(u, p) = Gamma^c(r_u - p) * SiLU(a^c_u + b^c_p + e(r_u - p) W_e^c + b^c)
// and b_p the projection of the embedding at p.  The two moved slots get
// their full message: the slot of a (up, at r_b) sums msg over every member
// and the other moved slot, the slot of b (down, at r_a) likewise.
template <typename T>
__global__ __launch_bounds__(256) void k_msg_swap(Net<T> P, int W, int ea, int eb, const double* __restrict__ R,
                                                  const int* __restrict__ uidx, int capmax,
                                                  const int* __restrict__ ucnt, const int* __restrict__ off,
                                                  const char* __restrict__ state, StateRec S, T* hseg0, T* hseg1,
                                                  T* mseg0, T* mseg1, int* rinfo0, int* rinfo1) {
  const Dims& D = P.D;
  constexpr int MPC = 10;               // members per chunk (6 pair feature sets each)
  constexpr int NS = 6;
  __shared__ T feat[NS * MPC * FEAT];
  __shared__ T fab[2 * FEAT];
  __shared__ int mem[MPC];
  const int j = blockIdx.x;
  if (ucnt[2 * j] + ucnt[2 * j + 1] == 0) return;   // dropped job
  const int c = threadIdx.x;
  const bool act = c < D.d;
  const int n = D.n, d = D.d;
  const char* rec = state + (int64_t)j * S.stride;
  const T* h0 = (const T*)(rec + S.h0);
  const T* proj = (const T*)(rec + S.proj);
  const T* mold = (const T*)(rec + S.m);
  const double* Rw = R + (int64_t)j * n * 3;
  const double ax = Rw[3 * ea], ay = Rw[3 * ea + 1], az = Rw[3 * ea + 2];
  const double bx = Rw[3 * eb], by = Rw[3 * eb + 1], bz = Rw[3 * eb + 2];
  // per-channel weights of both pair classes
  T w3[2][kMaxH2], wenv[2][kMaxG], we[2][4], bb[2];
  for (int a = 0; a < 2; ++a) {
    for (int k = 0; k < kMaxH2; ++k) w3[a][k] = (act && k < D.h2) ? P.ee_W3[(a * D.h2 + k) * d + c] : T(0);
    for (int k = 0; k < kMaxG; ++k) wenv[a][k] = (act && k < D.G) ? P.ee_Wenv[(a * D.G + k) * d + c] : T(0);
    for (int k = 0; k < 4; ++k) we[a][k] = act ? P.msg_We[(a * 4 + k) * d + c] : T(0);
    bb[a] = act ? P.msg_b[a * d + c] : T(0);
  }
  auto edge = [&](const T* f, int a, T av, T bv) -> T {
    if (f[44] == T(0)) return T(0);
    T g1 = 0, g2 = 0;
#pragma unroll
    for (int q = 0; q < kMaxH2; ++q) g1 += f[4 + q] * w3[a][q];
#pragma unroll
    for (int q = 0; q < kMaxG; ++q) g2 += f[12 + q] * wenv[a][q];
    const T ef = f[0] * we[a][0] + f[1] * we[a][1] + f[2] * we[a][2] + f[3] * we[a][3] + bb[a];
    return g1 * g2 * silu_(av + bv + ef);
  };
  auto feats = [&](double dx, double dy, double dz, int a, T* out) {
    pair_features<T>((T)dx, (T)dy, (T)dz, P.ee_W1 + a * 4 * D.h1, P.ee_b1 + a * D.h1, P.ee_W2 + a * D.h1 * D.h2,
                     P.ee_b2 + a * D.h2, P.ee_sig + a * D.G, (T)D.cut, D, out);
  };
  // the pair of the two moved slots (opposite spins before and after)
  if (threadIdx.x == 0) feats(bx - ax, by - ay, bz - az, 1, fab);          // slot a at r_b <- slot b at r_a
  else if (threadIdx.x == 1) feats(ax - bx, ay - by, az - bz, 1, fab + FEAT);   // slot b at r_a <- slot a at r_b
  T acc_a = 0, acc_b = 0;
  const T pa_a0 = act ? proj[((int64_t)ea * 4 + 0) * d + c] : T(0), pa_a1 = act ? proj[((int64_t)ea * 4 + 1) * d + c] : T(0);
  const T pa_b0 = act ? proj[((int64_t)ea * 4 + 2) * d + c] : T(0), pa_b1 = act ? proj[((int64_t)ea * 4 + 3) * d + c] : T(0);
  const T pb_a0 = act ? proj[((int64_t)eb * 4 + 0) * d + c] : T(0), pb_a1 = act ? proj[((int64_t)eb * 4 + 1) * d + c] : T(0);
  const T pb_b0 = act ? proj[((int64_t)eb * 4 + 2) * d + c] : T(0), pb_b1 = act ? proj[((int64_t)eb * 4 + 3) * d + c] : T(0);
  __syncthreads();
  if (act) {
    acc_a += edge(fab, 1, pb_a1, pa_b1);          // receiver at r_b with a-proj of r_b, sender at r_a
    acc_b += edge(fab + FEAT, 1, pa_a1, pb_b1);
  }
  for (int s = 0; s < 2; ++s) {
    const int cnt = ucnt[2 * j + s];
    const int* lst = uidx + ((int64_t)j * 2 + s) * capmax;
    T* hseg = s == 0 ? hseg0 : hseg1;
    T* mseg = s == 0 ? mseg0 : mseg1;
    int* rinfo = s == 0 ? rinfo0 : rinfo1;
    const int q0 = off[s * (W + 1) + j];
    // class of an edge between a member of block s and an up / down electron
    const int c_up = s == 0 ? 0 : 1, c_dn = 1 - c_up;
    for (int t0 = 1; t0 < cnt; t0 += MPC) {   // t = 0 is the moved slot
      const int tc = cnt - t0 < MPC ? cnt - t0 : MPC;
      __syncthreads();
      if (threadIdx.x < NS * tc) {
        const int t = threadIdx.x / NS, kind = threadIdx.x % NS;
        const int u = lst[t0 + t];
        if (kind == 0) mem[t] = u;
        const double ux = Rw[3 * u], uy = Rw[3 * u + 1], uz = Rw[3 * u + 2];
        T* out = feat + (NS * t + kind) * FEAT;
        // 0, 1: (u <- r_a) in class 0 / 1;  2, 3: (u <- r_b) in class 0 / 1
        // 4: (slot a at r_b <- u), class c_up;  5: (slot b at r_a <- u), class c_dn
        if (kind < 2) feats(ux - ax, uy - ay, uz - az, kind, out);
        else if (kind < 4) feats(ux - bx, uy - by, uz - bz, kind - 2, out);
        else if (kind == 4) feats(bx - ux, by - uy, bz - uz, c_up, out);
        else feats(ax - ux, ay - uy, az - uz, c_dn, out);
      }
      __syncthreads();
      if (!act) continue;
      for (int t = 0; t < tc; ++t) {
        const int u = mem[t];
        const T* f = feat + NS * t * FEAT;
        const T au[2] = {proj[((int64_t)u * 4 + 0) * d + c], proj[((int64_t)u * 4 + 1) * d + c]};
        const T bu[2] = {proj[((int64_t)u * 4 + 2) * d + c], proj[((int64_t)u * 4 + 3) * d + c]};
        // at r_a: old class c_up (an up electron there), new class c_dn; b-proj of r_a
        const T pa_b[2] = {pa_b0, pa_b1}, pb_b[2] = {pb_b0, pb_b1};
        T dm = edge(f + c_dn * FEAT, c_dn, au[c_dn], pa_b[c_dn]) - edge(f + c_up * FEAT, c_up, au[c_up], pa_b[c_up]);
        // at r_b: old class c_dn, new class c_up; b-proj of r_b
        dm += edge(f + (2 + c_up) * FEAT, c_up, au[c_up], pb_b[c_up]) -
              edge(f + (2 + c_dn) * FEAT, c_dn, au[c_dn], pb_b[c_dn]);
        // the moved slots receive from u
        const T pb_a[2] = {pb_a0, pb_a1}, pa_a[2] = {pa_a0, pa_a1};
        acc_a += edge(f + 4 * FEAT, c_up, pb_a[c_up], bu[c_up]);
        acc_b += edge(f + 5 * FEAT, c_dn, pa_a[c_dn], bu[c_dn]);
        const T mu = mold[(int64_t)u * d + c] + dm;
        const int64_t q = q0 + t0 + t;
        hseg[q * d + c] = h0[(int64_t)u * d + c] + mu;
        mseg[q * d + c] = mu;
        if (c == 0) { rinfo[2 * q] = j; rinfo[2 * q + 1] = u; }
      }
    }
  }
  if (act) {
    // slot a (up list, first) carries the embedding of position r_b
    const int64_t qa = off[j], qb = off[(W + 1) + j];
    hseg0[qa * d + c] = h0[(int64_t)eb * d + c] + acc_a;
    mseg0[qa * d + c] = acc_a;
    hseg1[qb * d + c] = h0[(int64_t)ea * d + c] + acc_b;
    mseg1[qb * d + c] = acc_b;
    if (c == 0) {
      rinfo0[2 * qa] = j; rinfo0[2 * qa + 1] = ea;
      rinfo1[2 * qb] = j; rinfo1[2 * qb + 1] = eb;
    }
  }
}

// ratio[w][a] = e^{dJ} sum_d w_d prod_s det A_ds with w_d the determinant's
// share of the sum (as a pseudopotential ratio, one job per walker)
__global__ void k_swap_ratio(const Dims D, int W, int ea, const double* __restrict__ detA,
                             const double* __restrict__ dj, const double* __restrict__ jsg,
                             const char* __restrict__ state, StateRec S, const int32_t* __restrict__ status,
                             double* __restrict__ ratios) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= W) return;
  const char* rec = state + (int64_t)j * S.stride;
  const double* ds = (const double*)(rec + S.dsign);
  const double* dl = (const double*)(rec + S.dlog);
  const double lp = *(const double*)(rec + S.lpsi), sp = *(const double*)(rec + S.spsi);
  const double* dA = detA + (int64_t)j * D.K * 4;
  double r = 0.0;
  for (int k = 0; k < D.K; ++k) {
    const double sg = ds[2 * k] * ds[2 * k + 1] * sp * dA[4 * k] * dA[4 * k + 2];
    if (sg != 0.0) r += sg * exp(dl[2 * k] + dl[2 * k + 1] - lp + dA[4 * k + 1] + dA[4 * k + 3]);
  }
  ratios[(int64_t)j * D.nu + ea] = status[j] ? NAN : r * exp(dj[j]) * (jsg ? jsg[j] : 1.0);
}

// R_b[w] = 1 - sum_a ratio[w][a]
__global__ void k_splus_rb(int W, int nu, const double* __restrict__ ratios, double* __restrict__ rb) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  double s = 0.0;
  for (int a = 0; a < nu; ++a) s += ratios[(int64_t)w * nu + a];
  rb[w] = 1.0 - s;
}

// workspace of a swap batch: the update layout without the Woodbury buffer,
// then the second moved position and the second envelope row
size_t swap_ws_bytes(const fire_handle* h, int W) {
  const UpdLayout L = upd_layout(h, W, false);
  return L.total + align_up((size_t)W * 24) + align_up((size_t)W * h->D.K * (h->D.nd > 0 ? h->D.nd : 1) * h->tsize);
}

template <typename T>
static hipError_t swap_ratio(const fire_handle* h, const Net<T>& P, int W, int ea, int eb, const double* R,
                             char* state, char* ws, int32_t* status, double* ratios, hipStream_t st) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  const UpdLayout L = upd_layout(h, W, false);
  const int blk = D.d <= 64 ? 64 : (D.d + 63) / 64 * 64;
  double* ra = (double*)(ws + L.rnew);
  double* rb = (double*)(ws + L.total);
  T* env1 = (T*)(ws + L.total + align_up((size_t)W * 24));
  int* uidx = (int*)(ws + L.uidx);
  int* ucnt = (int*)(ws + L.ucnt);
  int* off = (int*)(ws + L.off);
  T* basis = (T*)(ws + L.basis);
  T* env0 = (T*)(ws + L.envnew);
  hipLaunchKernelGGL(k_swap_propose, dim3((W + 3) / 4), dim3(256), 0, st, R, W, D.n, D.nu, ea, eb, D.cut * D.cut,
                     L.capS[0], L.capS[1], L.capmax, ra, rb, uidx, ucnt, P.jas, (double*)(ws + L.dj), status);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, ucnt, W, off, L.rowcap[0], L.rowcap[1],
                     (const int*)nullptr, status, (const int*)nullptr);
  CHECK(hipGetLastError());
  T* hs[2][2];
  T* ms[2];
  int* ri[2];
  for (int s = 0; s < 2; ++s) {
    hs[s][0] = (T*)(ws + L.hseg[s][0]);
    hs[s][1] = (T*)(ws + L.hseg[s][1]);
    ms[s] = (T*)(ws + L.mseg[s]);
    ri[s] = (int*)(ws + L.rowinfo[s]);
  }
  hipLaunchKernelGGL(k_msg_swap<T>, dim3(W), dim3(blk), 0, st, P, W, ea, eb, R, (const int*)uidx, L.capmax,
                     (const int*)ucnt, (const int*)off, (const char*)state, S, hs[0][0], hs[1][0], ms[0], ms[1], ri[0],
                     ri[1]);
  CHECK(hipGetLastError());
  // envelopes of the two moved slots at their new positions
  const T* envs[2] = {env0, env1};
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s);
    hipLaunchKernelGGL(k_env_basis<T>, dim3((unsigned)(((int64_t)W * D.B + 255) / 256)), dim3(256), 0, st, P,
                       (const double*)(s == 0 ? ra : rb), (int64_t)W, basis, (const int*)nullptr);
    CHECK(hipGetLastError());
    GemmArgs g{};
    g.A = basis; g.amap = rows_dense(D.B); g.Bt = s == 0 ? P.pi0 : P.pi1; g.ldb = D.B;
    g.C = (void*)envs[s]; g.cmap = rows_dense((int64_t)D.K * N); g.ccol = cols_dense(); g.M = W; g.N = D.K * N;
    g.K = D.B;
    CHECK(gemm_site(h, SITE_ORB, g, st));
  }
  for (int s = 0; s < 2; ++s) {
    const int N = D.nsig(s);
    const int e_s = s == 0 ? ea : eb;
    const int* Mdev = off + s * (W + 1) + W;
    const int rows = (int)L.rowcap[s];
    T* hin = hs[s][0];
    T* hout = hs[s][1];
    for (int k = 0; k < D.L; ++k) {
      GemmArgs g{};
      g.A = hin; g.amap = rows_dense(D.d);
      g.Bt = (const char*)P.mlp_t + (size_t)k * D.d * D.d * h->gsize; g.ldb = D.d;
      g.bias = P.mlp_b + (int64_t)k * D.d; g.C = hout; g.cmap = rows_dense(D.d); g.ccol = cols_dense();
      g.M = rows; g.N = D.d; g.K = D.d; g.act = ACT_SILU; g.Mdev = Mdev;
      CHECK(gemm_site(h, SITE_EMB, g, st));
      T* t = hin; hin = hout; hout = t;
    }
    if (D.Hj > 0) CHECK(jm_rows<T>(h, P, hin, rows, Mdev, ws + L.jscr, (double*)(ws + L.jnew[s]), st));
    if (D.Ra > 0) {
      GemmArgs ga{};
      ga.A = hin; ga.amap = rows_dense(D.d); ga.Bt = P.ja_Pt; ga.ldb = D.d;
      ga.C = ws + L.anew[s]; ga.cmap = rows_dense(D.NA()); ga.ccol = cols_dense(); ga.M = rows; ga.N = D.NA();
      ga.K = D.d; ga.Mdev = Mdev;
      CHECK(gemm_site(h, SITE_EMB, ga, st));
    }
    T* oseg = (T*)(ws + L.oseg[s]);
    GemmArgs o{};
    o.A = hin; o.amap = rows_dense(D.d); o.Bt = s == 0 ? P.orb_t0 : P.orb_t1; o.ldb = D.d;
    o.C = oseg; o.cmap = rows_dense((int64_t)D.K * N); o.ccol = cols_dense();
    o.M = rows; o.N = D.K * N; o.K = D.d; o.Mdev = Mdev;
    CHECK(gemm_site(h, SITE_ORB, o, st));
    const int64_t items = (int64_t)W * D.K;
    const int64_t quads = (items + 3) / 4;
    const bool pair = detA_pair(h, state, ws);
    hipLaunchKernelGGL(detA_kernel<T>(h, false, true, pair), dim3(det_grid((quads + 3) / 4, 1, D.K, 16)), dim3(256), 0,
                       st, D, W, (const int*)nullptr, s, e_s, (const int*)uidx, L.capmax, (const int*)ucnt,
                       (const int*)off, (const T*)nullptr, (const T*)oseg, envs[s], (const char*)state, S,
                       (double*)(ws + L.detA), 1);
    CHECK(hipGetLastError());
    if (L.capS[s] > 16) {
      hipLaunchKernelGGL(detA_kernel<T>(h, true, true, pair), dim3(det_grid((items + 3) / 4, 1, D.K, 4)), dim3(256), 0,
                         st, D, W, (const int*)nullptr, s, e_s, (const int*)uidx, L.capmax, (const int*)ucnt,
                         (const int*)off, (const T*)nullptr, (const T*)oseg, envs[s], (const char*)state, S,
                         (double*)(ws + L.detA), 1);
      CHECK(hipGetLastError());
    }
    if (L.capS[s] > 32) {
      const size_t lds = detA_lds(L.capmax);
      const unsigned nblk = (unsigned)(W < 2048 ? W : 2048);
      if (h->isize == 8) {
        CHECK(hipFuncSetAttribute((const void*)k_detA<T, double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
        hipLaunchKernelGGL((k_detA<T, double>), dim3(nblk), dim3(256), lds, st, D, W, (const int*)nullptr, s, e_s,
                           (const int*)uidx, L.capmax, (const int*)ucnt, (const int*)off, (const T*)nullptr,
                           (const T*)oseg, envs[s], (const char*)state, S, (double*)(ws + L.detA), 1);
      } else {
        CHECK(hipFuncSetAttribute((const void*)k_detA<T, float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
        hipLaunchKernelGGL((k_detA<T, float>), dim3(nblk), dim3(256), lds, st, D, W, (const int*)nullptr, s, e_s,
                           (const int*)uidx, L.capmax, (const int*)ucnt, (const int*)off, (const T*)nullptr,
                           (const T*)oseg, envs[s], (const char*)state, S, (double*)(ws + L.detA), 1);
      }
      CHECK(hipGetLastError());
    }
  }
  CHECK(jm_delta(h, W, (const int*)nullptr, uidx, L.capmax, ucnt, off, (const double*)(ws + L.jnew[0]),
                 (const double*)(ws + L.jnew[1]), state, (double*)(ws + L.dj), (double*)(ws + L.jsg),
                 (double*)(ws + L.jsum), st));
  CHECK(ja_delta<T>(h, P, W, (const int*)nullptr, (const int*)nullptr, uidx, L.capmax, ucnt, off,
                    (const T*)(ws + L.anew[0]), (const T*)(ws + L.anew[1]), state, ws + L.ja, (double*)(ws + L.dj),
                    (double*)(ws + L.jsg), D.Hj == 0, st));
  hipLaunchKernelGGL(k_swap_ratio, dim3((W + 127) / 128), dim3(128), 0, st, D, W, ea, (const double*)(ws + L.detA),
                     (const double*)(ws + L.dj),
                     D.Hj > 0 || D.Ra > 0 ? (const double*)(ws + L.jsg) : (const double*)nullptr,
                     (const char*)state, S, (const int32_t*)status, ratios);
  return hipGetLastError();
}

template <typename T>
static hipError_t splus_impl(fire_handle* h, int W, const double* R, char* state, char* ws, int eb, double* ratios,
                             double* rb, int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  Net<T> P = make_net<T>(h);
  CHECK(fill_i32(status, W, 0, st));
  for (int ea = 0; ea < D.nu; ++ea) CHECK(swap_ratio<T>(h, P, W, ea, eb, R, state, ws, status, ratios, st));
  hipLaunchKernelGGL(k_splus_rb, dim3((W + 127) / 128), dim3(128), 0, st, W, D.nu, (const double*)ratios, rb);
  return hipGetLastError();
}

hipError_t splus_path(fire_handle* h, int W, const double* R, char* state, char* ws, int eb, double* ratios,
                      double* rb, int32_t* status, hipStream_t s) {
  if (!update_fits(h)) return hipErrorInvalidValue;
  return h->tsize == 8 ? splus_impl<double>(h, W, R, state, ws, eb, ratios, rb, status, s)
                       : splus_impl<float>(h, W, R, state, ws, eb, ratios, rb, status, s);
}

template hipError_t propose_ratio<double>(const fire_handle*, const Net<double>&, const Jobs&, int,
                                          const double*, char*, char*, int32_t*, hipStream_t);
template hipError_t propose_ratio<float>(const fire_handle*, const Net<float>&, const Jobs&, int, const double*,
                                         char*, char*, int32_t*, hipStream_t);

}  // namespace fire
