// Per-electron MLP Jastrow factor (Methods, global electron correlation):
// readouts of the final embeddings, their per-walker sums, the single-
// electron update of the sums, and the jets of log|J_MLP| for the kinetic
// energy (Methods, efficient Laplacian: the readouts ride on the sparse jets
// of h_i, so their gradient and Laplacian use the same neighbourhood rows).
#include "jastrow.hpp"

namespace fire {

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

size_t jm_rows_ws(const fire_handle* h, int64_t M) {
  if (h->D.Hj <= 0 || M <= 0) return 0;
  return 2 * align_up((size_t)M * 2 * h->D.Hj * h->tsize);
}

// out[r] = (w3_0 . z[r][0:Hj] + b3_0, w3_1 . z[r][Hj:2Hj] + b3_1), FP64
// accumulation; one wave per row.
template <typename T>
__global__ __launch_bounds__(256) void k_jm_out(int M, const int* __restrict__ Mdev, int Hj, const T* __restrict__ z,
                                                const T* __restrict__ w3, const T* __restrict__ b3,
                                                double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int m = M;
  if (Mdev && *Mdev < m) m = *Mdev;
  if (r >= m) return;
  const T* zr = z + r * 2 * Hj;
  double a0 = 0.0, a1 = 0.0;
  for (int c = lane; c < Hj; c += 64) {
    a0 += (double)w3[c] * (double)zr[c];
    a1 += (double)w3[Hj + c] * (double)zr[Hj + c];
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if (lane == 0) {
    out[2 * r] = a0 + (double)b3[0];
    out[2 * r + 1] = a1 + (double)b3[1];
  }
}

template <typename T>
hipError_t jm_rows(const fire_handle* h, const Net<T>& P, const T* X, int M, const int* Mdev, char* scratch,
                   double* out, hipStream_t s) {
  const Dims& D = h->D;
  const int Hj = D.Hj;
  if (M <= 0 || Hj <= 0) return hipSuccess;
  T* z1 = (T*)scratch;
  T* z2 = (T*)(scratch + align_up((size_t)M * 2 * Hj * h->tsize));
  GemmArgs g{};
  g.A = X; g.amap = rows_dense(D.d); g.Bt = P.jm_W1t; g.ldb = D.d; g.bias = P.jm_b1;
  g.C = z1; g.cmap = rows_dense(2 * Hj); g.ccol = cols_dense(); g.M = M; g.N = 2 * Hj; g.K = D.d;
  g.act = ACT_SILU; g.Mdev = Mdev;
  CHECK(gemm_site(h, SITE_EMB, g, s));
  for (int k = 0; k < 2; ++k) {
    GemmArgs q{};
    q.A = z1 + (int64_t)k * Hj; q.amap = rows_dense(2 * Hj);
    q.Bt = (const char*)P.jm_W2t + (size_t)k * Hj * Hj * h->gsize; q.ldb = Hj; q.bias = P.jm_b2 + (int64_t)k * Hj;
    q.C = z2 + (int64_t)k * Hj; q.cmap = rows_dense(2 * Hj); q.ccol = cols_dense(); q.M = M; q.N = Hj; q.K = Hj;
    q.act = ACT_SILU; q.Mdev = Mdev;
    CHECK(gemm_site(h, SITE_EMB, q, s));
  }
  hipLaunchKernelGGL(k_jm_out<T>, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, M, Mdev, Hj, (const T*)z2,
                     P.jm_w3, P.jm_b3, out);
  return hipGetLastError();
}

// one workgroup per walker: copy the readouts into the record and sum them
// in a fixed order
__global__ __launch_bounds__(256) void k_jm_store(int n, const double* __restrict__ rows, char* __restrict__ state,
                                                  StateRec S) {
  __shared__ double red[16];
  const int64_t w = blockIdx.x;
  char* rec = state + w * S.stride;
  double* jme = (double*)(rec + S.jme);
  const double* src = rows + w * n * 2;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double u = src[2 * i], v = src[2 * i + 1];
    jme[2 * i] = u;
    jme[2 * i + 1] = v;
    a += u;
    b += v;
  }
  a = block_sum<double>(a, red);
  b = block_sum<double>(b, red);
  if (threadIdx.x == 0) {
    double* jms = (double*)(rec + S.jms);
    jms[0] = a;
    jms[1] = b;
  }
}

hipError_t jm_store(const fire_handle* h, int W, const double* rows, char* state, hipStream_t s) {
  if (h->D.Hj <= 0 || W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jm_store, dim3(W), dim3(256), 0, s, h->D.n, rows, state, h->st);
  return hipGetLastError();
}

__global__ void k_jm_total(int W, char* __restrict__ state, StateRec S, int32_t* __restrict__ status) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  char* rec = state + (int64_t)w * S.stride;
  const double* jms = (const double*)(rec + S.jms);
  const double s1 = jms[0], s2 = jms[1];
  if (!(s2 != 0.0) || !isfinite(s2) || !isfinite(s1)) {
    atomicOr(status + w, FIRE_W_DETSUM_ZERO);
    return;
  }
  *(double*)(rec + S.jas) += s1 + log(fabs(s2));
}

hipError_t jm_total(const fire_handle* h, int W, char* state, int32_t* status, hipStream_t s) {
  if (h->D.Hj <= 0 || W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jm_total, dim3((W + 127) / 128), dim3(128), 0, s, W, state, h->st, status);
  return hipGetLastError();
}

// one thread per job; jobs without update rows (inactive, or dropped for
// overflow, their walker flagged) keep dj and get a unit sign change
__global__ void k_jm_delta(const Dims D, int J, const int* __restrict__ jw, const int* __restrict__ uidx, int capmax,
                           const int* __restrict__ ucnt, const int* __restrict__ off, const double* __restrict__ jnew0,
                           const double* __restrict__ jnew1, const char* __restrict__ state, StateRec S,
                           double* __restrict__ dj, double* __restrict__ jsg, double* __restrict__ jsum) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const int c0 = ucnt[2 * j], c1 = ucnt[2 * j + 1];
  if (c0 + c1 == 0) {
    jsg[j] = 1.0;
    return;
  }
  const int w = jw ? jw[j] : j;
  const char* rec = state + (int64_t)w * S.stride;
  const double* jme = (const double*)(rec + S.jme);
  const double* jms = (const double*)(rec + S.jms);
  double d1 = 0.0, d2 = 0.0;
  for (int s = 0; s < 2; ++s) {
    const int cnt = s == 0 ? c0 : c1;
    const int q0 = off[s * (J + 1) + j];
    const int* lst = uidx + ((int64_t)j * 2 + s) * capmax;
    const double* jn = s == 0 ? jnew0 : jnew1;
    for (int t = 0; t < cnt; ++t) {
      const int u = lst[t];
      d1 += jn[2 * (int64_t)(q0 + t)] - jme[2 * u];
      d2 += jn[2 * (int64_t)(q0 + t) + 1] - jme[2 * u + 1];
    }
  }
  const double s2o = jms[1];
  const double s1 = jms[0] + d1, s2 = s2o + d2;
  jsum[2 * j] = s1;
  jsum[2 * j + 1] = s2;
  if (!(s2 != 0.0) || !isfinite(s2)) {
    dj[j] = -INFINITY;
    jsg[j] = 0.0;
    return;
  }
  dj[j] += d1 + log(fabs(s2)) - log(fabs(s2o));
  jsg[j] = (s2 > 0.0) == (s2o > 0.0) ? 1.0 : -1.0;
}

hipError_t jm_delta(const fire_handle* h, int J, const int* jw, const int* uidx, int capmax, const int* ucnt,
                    const int* off, const double* jnew0, const double* jnew1, const char* state, double* dj,
                    double* jsg, double* jsum, hipStream_t s) {
  if (h->D.Hj <= 0 || J <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jm_delta, dim3((J + 127) / 128), dim3(128), 0, s, h->D, J, jw, uidx, capmax, ucnt, off, jnew0,
                     jnew1, state, h->st, dj, jsg, jsum);
  return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_jm_commit(int W, const int* __restrict__ acc, const int* __restrict__ uidx,
                                                  int capmax, const int* __restrict__ ucnt,
                                                  const int* __restrict__ off, const double* __restrict__ jnew0,
                                                  const double* __restrict__ jnew1, const double* __restrict__ jsum,
                                                  char* __restrict__ state, StateRec S) {
  const int w = blockIdx.x;
  if (!acc[w]) return;
  char* rec = state + (int64_t)w * S.stride;
  double* jme = (double*)(rec + S.jme);
  for (int s = 0; s < 2; ++s) {
    const int cnt = ucnt[2 * w + s];
    const int q0 = off[s * (W + 1) + w];
    const int* lst = uidx + ((int64_t)w * 2 + s) * capmax;
    const double* jn = s == 0 ? jnew0 : jnew1;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      jme[2 * lst[t]] = jn[2 * (int64_t)(q0 + t)];
      jme[2 * lst[t] + 1] = jn[2 * (int64_t)(q0 + t) + 1];
    }
  }
  if (threadIdx.x == 0) {
    double* jms = (double*)(rec + S.jms);
    jms[0] = jsum[2 * w];
    jms[1] = jsum[2 * w + 1];
  }
}

hipError_t jm_commit(const fire_handle* h, int W, const int* acc, const int* uidx, int capmax, const int* ucnt,
                     const int* off, const double* jnew0, const double* jnew1, const double* jsum, char* state,
                     hipStream_t s) {
  if (h->D.Hj <= 0 || W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jm_commit, dim3(W), dim3(64), 0, s, W, acc, uidx, capmax, ucnt, off, jnew0, jnew1, jsum,
                     state, h->st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// jets
// ---------------------------------------------------------------------------
// SiLU on jets of width Hj, in place: value z -> f(z), tangent rows
// t -> f'(z) t, Laplacian row l -> f'(z) l + f''(z) sum_t t^2
template <typename T>
__global__ __launch_bounds__(256) void k_jm_act(int64_t nrows, int n, int nu, int Hj, const int32_t* __restrict__ ncnt,
                                                const int* __restrict__ joff, T* __restrict__ z, T* jet0, T* jet1) {
  const int64_t e = blockIdx.x;
  const int c = threadIdx.x;
  if (e >= nrows || c >= Hj) return;
  const int i = (int)(e % n);
  T* jet = i < nu ? jet0 : jet1;
  const int nt = 3 * (1 + ncnt[2 * e] + ncnt[2 * e + 1]);
  const int64_t base = joff[e];
  T f, f1, f2;
  silu3(z[e * Hj + c], f, f1, f2);
  z[e * Hj + c] = f;
  T sq = 0;
  for (int r = 0; r < nt; ++r) {
    const T t = jet[(base + r) * Hj + c];
    sq += t * t;
    jet[(base + r) * Hj + c] = f1 * t;
  }
  jet[(base + nt) * Hj + c] = f1 * jet[(base + nt) * Hj + c] + f2 * sq;
}

// readout k over every jet row of electron e: jt[row][k] = w3_k . jet[row]
// (the bias has no tangent); one workgroup per electron, a wave per row
template <typename T>
__global__ __launch_bounds__(256) void k_jm_jetdot(int64_t nrows, int n, int nu, int Hj,
                                                   const int32_t* __restrict__ ncnt, const int* __restrict__ joff,
                                                   const T* __restrict__ jet0, const T* __restrict__ jet1,
                                                   const T* __restrict__ w3k, int k, double* jt0, double* jt1) {
  const int64_t e = blockIdx.x;
  if (e >= nrows) return;
  const int i = (int)(e % n);
  const T* jet = i < nu ? jet0 : jet1;
  double* jt = i < nu ? jt0 : jt1;
  const int nt = 3 * (1 + ncnt[2 * e] + ncnt[2 * e + 1]) + 1;
  const int64_t base = joff[e];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int r = wv; r < nt; r += 4) {
    double a = 0.0;
    for (int c = lane; c < Hj; c += 64) a += (double)w3k[c] * (double)jet[(base + r) * Hj + c];
    a = wave_sum(a);
    if (lane == 0) jt[(base + r) * 2 + k] = a;
  }
}

// per walker: d_{n,x} S_k = sum over the members i of T_n = {n} u N_n of the
// tangent row of i at n's slot (the neighbour relation is symmetric), and
//   grad log|J| = dS_1 + dS_2 / S_2,
//   Lap log|J| = sum_i (Lap MLP_1(h_i) + Lap MLP_2(h_i) / S_2)
//                - sum_{n,x} (d_{n,x} S_2 / S_2)^2
__global__ __launch_bounds__(256) void k_jm_kin(const Dims D, int Wc, int w0, const int* __restrict__ memb,
                                                const int* __restrict__ mslot, const int* __restrict__ mcnt, int tcap,
                                                const int32_t* __restrict__ ncnt, const int* __restrict__ joff,
                                                const double* __restrict__ jt0, const double* __restrict__ jt1,
                                                const char* __restrict__ state, StateRec S, double* __restrict__ gJ,
                                                double* __restrict__ lapJ) {
  __shared__ double red[16];
  const int wl = blockIdx.x, n = D.n;
  const char* rec = state + (int64_t)(w0 + wl) * S.stride;
  const double s2 = ((const double*)(rec + S.jms))[1];
  const double inv = s2 != 0.0 && isfinite(s2) ? 1.0 / s2 : 0.0;
  double acc = 0.0;
  for (int nn = threadIdx.x; nn < n; nn += blockDim.x) {
    const int64_t en = (int64_t)wl * n + nn;
    double g1[3] = {0, 0, 0}, g2[3] = {0, 0, 0};
    for (int sp = 0; sp < 2; ++sp) {
      const int t = mcnt[2 * en + sp];
      const int* mem = memb + (en * 2 + sp) * tcap;
      const int* slt = mslot + (en * 2 + sp) * tcap;
      const double* jt = sp == 0 ? jt0 : jt1;
      for (int a = 0; a < t; ++a) {
        const int64_t row = (int64_t)joff[(int64_t)wl * n + mem[a]] + 3 * slt[a];
        for (int x = 0; x < 3; ++x) {
          g1[x] += jt[(row + x) * 2];
          g2[x] += jt[(row + x) * 2 + 1];
        }
      }
    }
    const int cn = ncnt[2 * en] + ncnt[2 * en + 1];
    const int64_t lr = (int64_t)joff[en] + 3 * (1 + cn);
    const double* jts = nn < D.nu ? jt0 : jt1;
    acc += jts[lr * 2] + jts[lr * 2 + 1] * inv;
    for (int x = 0; x < 3; ++x) {
      const double q = g2[x] * inv;
      gJ[en * 3 + x] = g1[x] + q;
      acc -= q * q;
    }
  }
  const double tot = block_sum<double>(acc, red);
  if (threadIdx.x == 0) lapJ[wl] = tot;
}

template <typename T>
hipError_t jm_kinetic(const fire_handle* h, const Net<T>& P, const JmJetArgs& a, const char* state,
                      hipStream_t s) {
  const Dims& D = h->D;
  const int Hj = D.Hj, d = D.d, n = D.n;
  if (Hj <= 0) return hipSuccess;
  const int64_t rows = (int64_t)a.Wc * n;
  T* zv1 = (T*)a.zv;
  T* zv2 = zv1 + rows * Hj;
  const int blk = Hj <= 64 ? 64 : (Hj + 63) / 64 * 64;
  for (int k = 0; k < 2; ++k) {
    const char* W1k = (const char*)P.jm_W1t + (size_t)k * Hj * d * h->gsize;
    const char* W2k = (const char*)P.jm_W2t + (size_t)k * Hj * Hj * h->gsize;
    GemmArgs g{};
    g.A = a.hval; g.amap = rows_dense(d); g.Bt = W1k; g.ldb = d; g.bias = P.jm_b1 + (int64_t)k * Hj;
    g.C = zv1; g.cmap = rows_dense(Hj); g.ccol = cols_dense(); g.M = (int)rows; g.N = Hj; g.K = d;
    CHECK(gemm_site(h, SITE_EMB, g, s));
    for (int sp = 0; sp < 2; ++sp) {
      if (D.nsig(sp) == 0) continue;
      GemmArgs j{};
      j.A = a.jin[sp]; j.amap = rows_dense(d); j.Bt = W1k; j.ldb = d;
      j.C = a.jx[sp]; j.cmap = rows_dense(Hj); j.ccol = cols_dense(); j.M = (int)a.rowcap[sp]; j.N = Hj; j.K = d;
      j.Mdev = a.jtot + sp;
      CHECK(gemm_site(h, SITE_JET, j, s));
    }
    hipLaunchKernelGGL(k_jm_act<T>, dim3((unsigned)rows), dim3(blk), 0, s, rows, n, D.nu, Hj, a.ncnt, a.joff, zv1,
                       (T*)a.jx[0], (T*)a.jx[1]);
    CHECK(hipGetLastError());
    GemmArgs g2{};
    g2.A = zv1; g2.amap = rows_dense(Hj); g2.Bt = W2k; g2.ldb = Hj; g2.bias = P.jm_b2 + (int64_t)k * Hj;
    g2.C = zv2; g2.cmap = rows_dense(Hj); g2.ccol = cols_dense(); g2.M = (int)rows; g2.N = Hj; g2.K = Hj;
    CHECK(gemm_site(h, SITE_EMB, g2, s));
    for (int sp = 0; sp < 2; ++sp) {
      if (D.nsig(sp) == 0) continue;
      GemmArgs j{};
      j.A = a.jx[sp]; j.amap = rows_dense(Hj); j.Bt = W2k; j.ldb = Hj;
      j.C = a.jy[sp]; j.cmap = rows_dense(Hj); j.ccol = cols_dense(); j.M = (int)a.rowcap[sp]; j.N = Hj; j.K = Hj;
      j.Mdev = a.jtot + sp;
      CHECK(gemm_site(h, SITE_JET, j, s));
    }
    hipLaunchKernelGGL(k_jm_act<T>, dim3((unsigned)rows), dim3(blk), 0, s, rows, n, D.nu, Hj, a.ncnt, a.joff, zv2,
                       (T*)a.jy[0], (T*)a.jy[1]);
    CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_jm_jetdot<T>, dim3((unsigned)rows), dim3(256), 0, s, rows, n, D.nu, Hj, a.ncnt, a.joff,
                       (const T*)a.jy[0], (const T*)a.jy[1], P.jm_w3 + (int64_t)k * Hj, k, a.jt[0], a.jt[1]);
    CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_jm_kin, dim3(a.Wc), dim3(256), 0, s, D, a.Wc, a.w0, a.memb, a.mslot, a.mcnt, a.tcap, a.ncnt,
                     a.joff, (const double*)a.jt[0], (const double*)a.jt[1], state, h->st, a.gJ, a.lapJ);
  return hipGetLastError();
}

template hipError_t jm_rows<double>(const fire_handle*, const Net<double>&, const double*, int, const int*, char*,
                                    double*, hipStream_t);
template hipError_t jm_rows<float>(const fire_handle*, const Net<float>&, const float*, int, const int*, char*,
                                   double*, hipStream_t);
template hipError_t jm_kinetic<double>(const fire_handle*, const Net<double>&, const JmJetArgs&, const char*,
                                       hipStream_t);
template hipError_t jm_kinetic<float>(const fire_handle*, const Net<float>&, const JmJetArgs&, const char*,
                                      hipStream_t);

}  // namespace fire
