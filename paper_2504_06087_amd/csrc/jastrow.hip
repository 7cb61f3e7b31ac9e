// Per-electron MLP Jastrow factor (Methods, global electron correlation):
// readouts of the final embeddings, their per-walker sums, the single-
// electron update of the sums, and the jets of log|J_MLP| for the kinetic
// energy (Methods, efficient Laplacian: the readouts ride on the sparse jets
// of h_i, so their gradient and Laplacian use the same neighbourhood rows).
#include "jastrow.hpp"

namespace fire {

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

size_t readout_ws(const fire_handle* h, int64_t M, int H) {
  if (H <= 0 || M <= 0) return 0;
  return 2 * align_up((size_t)M * 2 * H * h->tsize);
}

// out[r] = (w3_0 . z[r][0:H] + b3_0, w3_1 . z[r][H:2H] + b3_1), FP64
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
hipError_t readout_rows(const fire_handle* h, const Readout<T>& Q, const T* X, int M, const int* Mdev,
                        char* scratch, double* out, hipStream_t s) {
  const int H = Q.H;
  if (M <= 0 || H <= 0) return hipSuccess;
  T* z1 = (T*)scratch;
  T* z2 = (T*)(scratch + align_up((size_t)M * 2 * H * h->tsize));
  GemmArgs g{};
  g.A = X; g.amap = rows_dense(Q.in); g.Bt = Q.W1t; g.ldb = Q.in; g.bias = Q.b1;
  g.C = z1; g.cmap = rows_dense(2 * H); g.ccol = cols_dense(); g.M = M; g.N = 2 * H; g.K = Q.in;
  g.act = ACT_SILU; g.Mdev = Mdev;
  CHECK(gemm_site(h, SITE_EMB, g, s));
  for (int k = 0; k < 2; ++k) {
    GemmArgs q{};
    q.A = z1 + (int64_t)k * H; q.amap = rows_dense(2 * H);
    q.Bt = (const char*)Q.W2t + (size_t)k * H * H * h->gsize; q.ldb = H; q.bias = Q.b2 + (int64_t)k * H;
    q.C = z2 + (int64_t)k * H; q.cmap = rows_dense(2 * H); q.ccol = cols_dense(); q.M = M; q.N = H; q.K = H;
    q.act = ACT_SILU; q.Mdev = Mdev;
    CHECK(gemm_site(h, SITE_EMB, q, s));
  }
  hipLaunchKernelGGL(k_jm_out<T>, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, M, Mdev, H, (const T*)z2, Q.w3,
                     Q.b3, out);
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

// ---------------------------------------------------------------------------
// attention-register Jastrow
// ---------------------------------------------------------------------------
// offsets inside the FP64 block jat of a record: m [Ra], Z [Ra], N [NV], o [2]
FIRE_HOST_DEVICE inline int jat_Z(const Dims& D) { return D.Ra; }
FIRE_HOST_DEVICE inline int jat_N(const Dims& D) { return 2 * D.Ra; }
FIRE_HOST_DEVICE inline int jat_o(const Dims& D) { return 2 * D.Ra + D.NV(); }

size_t ja_eval_ws(const fire_handle* h, int W) {
  const Dims& D = h->D;
  if (D.Ra <= 0) return 0;
  return align_up((size_t)W * D.NV() * h->tsize) + align_up((size_t)W * 2 * 8) + readout_ws(h, W, D.Ha);
}

// one workgroup per walker: shifts m_r = max_i l_ri, Z_r, N_r and the
// register embeddings V = N / Z (T, the readout GEMM's input); every sum
// runs over the electrons in order
template <typename T>
__global__ __launch_bounds__(256) void k_ja_sums(const Dims D, char* __restrict__ state, StateRec S,
                                                 T* __restrict__ av) {
  __shared__ double mz[2 * 64];
  const int64_t w = blockIdx.x;
  char* rec = state + w * S.stride;
  const T* a = (const T*)(rec + S.jae);
  double* jt = (double*)(rec + S.jat);
  const int NA = D.NA(), NV = D.NV(), Ra = D.Ra, n = D.n;
  for (int r = threadIdx.x; r < Ra; r += blockDim.x) {
    double m = -INFINITY;
    for (int i = 0; i < n; ++i) m = fmax(m, (double)a[(int64_t)i * NA + r]);
    double z = 0.0;
    for (int i = 0; i < n; ++i) z += exp((double)a[(int64_t)i * NA + r] - m);
    mz[r] = m;
    mz[64 + r] = z;
    jt[r] = m;
    jt[jat_Z(D) + r] = z;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < NV; c += blockDim.x) {
    const int r = c / D.dr;
    const double m = mz[r];
    double acc = 0.0;
    for (int i = 0; i < n; ++i)
      acc += exp((double)a[(int64_t)i * NA + r] - m) * (double)a[(int64_t)i * NA + Ra + c];
    jt[jat_N(D) + c] = acc;
    av[w * NV + c] = (T)(acc / mz[64 + r]);
  }
}

__global__ void k_ja_store(const Dims D, int W, const double* __restrict__ out, char* __restrict__ state, StateRec S) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  double* o = (double*)(state + (int64_t)w * S.stride + S.jat) + jat_o(D);
  o[0] = out[2 * w];
  o[1] = out[2 * w + 1];
}

template <typename T>
hipError_t ja_eval(const fire_handle* h, const Net<T>& P, int W, const T* X, char* state, char* ws, hipStream_t s) {
  const Dims& D = h->D;
  if (D.Ra <= 0 || W <= 0) return hipSuccess;
  const StateRec& S = h->st;
  const int64_t srecT = S.stride / sizeof(T);
  T* av = (T*)ws;
  double* aout = (double*)(ws + align_up((size_t)W * D.NV() * h->tsize));
  char* scr = (char*)aout + align_up((size_t)W * 2 * 8);
  GemmArgs g{};
  g.A = X; g.amap = rows_dense(D.d); g.Bt = P.ja_Pt; g.ldb = D.d;
  g.C = state + S.jae; g.cmap = RowMap{D.n, srecT, D.NA()}; g.ccol = cols_dense();
  g.M = W * D.n; g.N = D.NA(); g.K = D.d;
  CHECK(gemm_site(h, SITE_EMB, g, s));
  hipLaunchKernelGGL(k_ja_sums<T>, dim3(W), dim3(256), 0, s, D, state, S, av);
  CHECK(hipGetLastError());
  CHECK(readout_rows<T>(h, ja_readout<T>(h, P), av, W, nullptr, scr, aout, s));
  hipLaunchKernelGGL(k_ja_store, dim3((W + 127) / 128), dim3(128), 0, s, D, W, (const double*)aout, state, S);
  return hipGetLastError();
}

__global__ void k_ja_total(const Dims D, int W, char* __restrict__ state, StateRec S, int32_t* __restrict__ status) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  char* rec = state + (int64_t)w * S.stride;
  const double* o = (const double*)(rec + S.jat) + jat_o(D);
  if (!(o[1] != 0.0) || !isfinite(o[1]) || !isfinite(o[0])) {
    atomicOr(status + w, FIRE_W_DETSUM_ZERO);
    return;
  }
  *(double*)(rec + S.jas) += o[0] + log(fabs(o[1]));
}

hipError_t ja_total(const fire_handle* h, int W, char* state, int32_t* status, hipStream_t s) {
  if (h->D.Ra <= 0 || W <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ja_total, dim3((W + 127) / 128), dim3(128), 0, s, h->D, W, state, h->st, status);
  return hipGetLastError();
}

// ---- updates
struct JaUpd {
  size_t zs, vv, out, scr, total;
};
static JaUpd ja_upd(const fire_handle* h, int J) {
  const Dims& D = h->D;
  JaUpd L{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  L.zs = take((size_t)J * (D.Ra + D.NV()) * 8);
  L.vv = take((size_t)J * D.NV() * h->tsize);
  L.out = take((size_t)J * 2 * 8);
  L.scr = take(readout_ws(h, J, D.Ha));
  L.total = o;
  return L;
}
size_t ja_update_ws(const fire_handle* h, int J) { return h->D.Ra > 0 ? ja_upd(h, J).total : 0; }

// one workgroup per job: Z' and N' from the cached sums and the old and new
// projections of the job's update rows (shift m_r of the last evaluation),
// then V' = N' / Z'; jobs without rows get zero registers
template <typename T>
__global__ __launch_bounds__(256) void k_ja_delta(const Dims D, int J, const int* __restrict__ jw,
                                                  const int* __restrict__ uidx, int capmax,
                                                  const int* __restrict__ ucnt, const int* __restrict__ off,
                                                  const T* __restrict__ anew0, const T* __restrict__ anew1,
                                                  const char* __restrict__ state, StateRec S, double* __restrict__ zs,
                                                  T* __restrict__ vv) {
  __shared__ double Zs[64];
  const int j = blockIdx.x;
  const int NA = D.NA(), NV = D.NV(), Ra = D.Ra;
  const int c0 = ucnt[2 * j], c1 = ucnt[2 * j + 1];
  T* vr = vv + (int64_t)j * NV;
  if (c0 + c1 == 0) {
    for (int c = threadIdx.x; c < NV; c += blockDim.x) vr[c] = T(0);
    return;
  }
  const int w = jw ? jw[j] : j;
  const char* rec = state + (int64_t)w * S.stride;
  const T* a = (const T*)(rec + S.jae);
  const double* jt = (const double*)(rec + S.jat);
  double* zr = zs + (int64_t)j * NA;
  for (int c = threadIdx.x; c < NA; c += blockDim.x) {
    const bool isz = c < Ra;
    const int r = isz ? c : (c - Ra) / D.dr;
    const double m = jt[r];
    double acc = isz ? jt[jat_Z(D) + r] : jt[jat_N(D) + (c - Ra)];
    for (int s = 0; s < 2; ++s) {
      const int cnt = s == 0 ? c0 : c1;
      const int q0 = off[s * (J + 1) + j];
      const int* lst = uidx + ((int64_t)j * 2 + s) * capmax;
      const T* an = s == 0 ? anew0 : anew1;
      for (int t = 0; t < cnt; ++t) {
        const T* ao = a + (int64_t)lst[t] * NA;
        const T* ar = an + (int64_t)(q0 + t) * NA;
        const double eo = exp((double)ao[r] - m), en = exp((double)ar[r] - m);
        acc += isz ? en - eo : en * (double)ar[c] - eo * (double)ao[c];
      }
    }
    zr[c] = acc;
    if (isz) Zs[r] = acc;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < NV; c += blockDim.x) vr[c] = (T)(zr[Ra + c] / Zs[c / D.dr]);
}

__global__ void k_ja_dj(const Dims D, int J, const int* __restrict__ jw, const int* __restrict__ ucnt,
                        const char* __restrict__ state, StateRec S, const double* __restrict__ out,
                        double* __restrict__ dj, double* __restrict__ jsg, bool first) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  if (ucnt[2 * j] + ucnt[2 * j + 1] == 0) {
    if (first) jsg[j] = 1.0;
    return;
  }
  const int w = jw ? jw[j] : j;
  const double* o = (const double*)(state + (int64_t)w * S.stride + S.jat) + jat_o(D);
  const double o1 = out[2 * j], o2 = out[2 * j + 1];
  const double sg = first ? 1.0 : jsg[j];
  if (!(o2 != 0.0) || !isfinite(o2) || !isfinite(o1)) {
    dj[j] = -INFINITY;
    jsg[j] = 0.0;
    return;
  }
  dj[j] += o1 - o[0] + log(fabs(o2)) - log(fabs(o[1]));
  jsg[j] = sg * ((o2 > 0.0) == (o[1] > 0.0) ? 1.0 : -1.0);
}

template <typename T>
hipError_t ja_delta(const fire_handle* h, const Net<T>& P, int J, const int* jw, const int* Jdev, const int* uidx,
                    int capmax, const int* ucnt, const int* off, const T* anew0, const T* anew1, const char* state,
                    char* ws, double* dj, double* jsg, bool first, hipStream_t s) {
  const Dims& D = h->D;
  if (D.Ra <= 0 || J <= 0) return hipSuccess;
  const JaUpd L = ja_upd(h, J);
  hipLaunchKernelGGL(k_ja_delta<T>, dim3(J), dim3(256), 0, s, D, J, jw, uidx, capmax, ucnt, off, anew0, anew1, state,
                     h->st, (double*)(ws + L.zs), (T*)(ws + L.vv));
  CHECK(hipGetLastError());
  CHECK(readout_rows<T>(h, ja_readout<T>(h, P), (const T*)(ws + L.vv), J, Jdev, ws + L.scr, (double*)(ws + L.out),
                        s));
  hipLaunchKernelGGL(k_ja_dj, dim3((J + 127) / 128), dim3(128), 0, s, D, J, jw, ucnt, state, h->st,
                     (const double*)(ws + L.out), dj, jsg, first);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_ja_commit(const Dims D, int W, const int* __restrict__ acc,
                                                   const int* __restrict__ uidx, int capmax,
                                                   const int* __restrict__ ucnt, const int* __restrict__ off,
                                                   const T* __restrict__ anew0, const T* __restrict__ anew1,
                                                   const double* __restrict__ zs, const double* __restrict__ out,
                                                   char* __restrict__ state, StateRec S) {
  const int w = blockIdx.x;
  if (!acc[w]) return;
  const int NA = D.NA();
  char* rec = state + (int64_t)w * S.stride;
  T* a = (T*)(rec + S.jae);
  double* jt = (double*)(rec + S.jat);
  for (int s = 0; s < 2; ++s) {
    const int cnt = ucnt[2 * w + s];
    const int q0 = off[s * (W + 1) + w];
    const int* lst = uidx + ((int64_t)w * 2 + s) * capmax;
    const T* an = s == 0 ? anew0 : anew1;
    for (int q = threadIdx.x; q < cnt * NA; q += blockDim.x) {
      const int t = q / NA, c = q % NA;
      a[(int64_t)lst[t] * NA + c] = an[(int64_t)(q0 + t) * NA + c];
    }
  }
  for (int c = threadIdx.x; c < NA; c += blockDim.x) jt[jat_Z(D) + c] = zs[(int64_t)w * NA + c];
  if (threadIdx.x == 0) {
    jt[jat_o(D)] = out[2 * w];
    jt[jat_o(D) + 1] = out[2 * w + 1];
  }
}

template <typename T>
hipError_t ja_commit(const fire_handle* h, int W, const int* acc, const int* uidx, int capmax, const int* ucnt,
                     const int* off, const T* anew0, const T* anew1, const char* ws, char* state, hipStream_t s) {
  const Dims& D = h->D;
  if (D.Ra <= 0 || W <= 0) return hipSuccess;
  const JaUpd L = ja_upd(h, W);
  hipLaunchKernelGGL(k_ja_commit<T>, dim3(W), dim3(256), 0, s, D, W, acc, uidx, capmax, ucnt, off, anew0, anew1,
                     (const double*)(ws + L.zs), (const double*)(ws + L.out), state, h->st);
  return hipGetLastError();
}

// ---- kinetic energy
struct JaKin {
  size_t ajet[2], ex, vj, dz, y1, y2, oj, total;
};
static JaKin ja_kin(const fire_handle* h, int Wc, const int64_t rowcap[2]) {
  const Dims& D = h->D;
  JaKin L{};
  size_t o = 0;
  const size_t ts = h->tsize;
  const int64_t rows3 = (int64_t)Wc * (3 * D.n + 2);
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  for (int s = 0; s < 2; ++s) L.ajet[s] = take((size_t)rowcap[s] * D.NA() * ts);
  L.ex = take((size_t)Wc * D.n * D.Ra * 8);
  L.vj = take((size_t)rows3 * D.NV() * ts);
  L.dz = take((size_t)Wc * 3 * D.n * D.Ra * 8);
  L.y1 = take((size_t)rows3 * D.Ha * ts);
  L.y2 = take((size_t)rows3 * D.Ha * ts);
  L.oj = take((size_t)2 * rows3 * 8);
  L.total = o;
  return L;
}
size_t ja_kin_ws(const fire_handle* h, int Wc, const int64_t rowcap[2]) {
  return h->D.Ra > 0 ? ja_kin(h, Wc, rowcap).total : 0;
}

// E_ri = e^{l_ri - m_r} for walkers w0 + [0, Wc)
template <typename T>
__global__ void k_ja_exp(const Dims D, int Wc, int w0, const char* __restrict__ state, StateRec S,
                         double* __restrict__ ex) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = D.n, Ra = D.Ra;
  if (q >= (int64_t)Wc * n * Ra) return;
  const int64_t wl = q / ((int64_t)n * Ra);
  const int i = (int)((q / Ra) % n), r = (int)(q % Ra);
  const char* rec = state + (w0 + wl) * S.stride;
  const T* a = (const T*)(rec + S.jae);
  const double* jt = (const double*)(rec + S.jat);
  ex[q] = exp((double)a[(int64_t)i * D.NA() + r] - jt[r]);
}

// Dense tangents per coordinate (n, x) of walker wl, gathered over the
// members i of T_n (each i's tangent row at n's slot):
//   dZ_r = sum_i E_ri dl_ri,   dN_rc = sum_i E_ri (du_ric + u_ric dl_ri),
// then dV = (dN - V dZ) / Z into row 1 + 3 n + x of the walker's readout
// jet block; dZ (FP64) is kept for the Laplacian's cross term.
template <typename T>
__global__ __launch_bounds__(256) void k_ja_dense(const Dims D, int Wc, int w0, const int* __restrict__ memb,
                                                  const int* __restrict__ mslot, const int* __restrict__ mcnt,
                                                  int tcap, const int* __restrict__ joff, const T* __restrict__ aj0,
                                                  const T* __restrict__ aj1, const double* __restrict__ ex,
                                                  const char* __restrict__ state, StateRec S, T* __restrict__ vj,
                                                  double* __restrict__ dz) {
  __shared__ double sh[64 + 1024];
  const int n = D.n, Ra = D.Ra, NA = D.NA(), NV = D.NV();
  const int64_t en = blockIdx.x;
  const int64_t wl = en / n;
  const int nn = (int)(en % n);
  const char* rec = state + (w0 + wl) * S.stride;
  const T* av = (const T*)(rec + S.jae);
  const double* jt = (const double*)(rec + S.jat);
  for (int x = 0; x < 3; ++x) {
    for (int c = threadIdx.x; c < NA; c += blockDim.x) {
      const bool isz = c < Ra;
      const int r = isz ? c : (c - Ra) / D.dr;
      double acc = 0.0;
      for (int sp = 0; sp < 2; ++sp) {
        const int t = mcnt[2 * en + sp];
        const int* mem = memb + (en * 2 + sp) * tcap;
        const int* slt = mslot + (en * 2 + sp) * tcap;
        const T* aj = sp == 0 ? aj0 : aj1;
        for (int b = 0; b < t; ++b) {
          const int i = mem[b];
          const int64_t row = (int64_t)joff[wl * n + i] + 3 * slt[b] + x;
          const double E = ex[(wl * n + i) * Ra + r];
          const double tl = (double)aj[row * NA + r];
          acc += isz ? E * tl : E * ((double)aj[row * NA + c] + (double)av[(int64_t)i * NA + c] * tl);
        }
      }
      sh[c] = acc;
    }
    __syncthreads();
    const int64_t vrow = wl * (3 * n + 2) + 1 + 3 * nn + x;
    for (int c = threadIdx.x; c < NV; c += blockDim.x) {
      const int r = c / D.dr;
      const double Z = jt[Ra + r], V = jt[2 * Ra + c] / Z;
      vj[vrow * NV + c] = (T)((sh[Ra + c] - V * sh[r]) / Z);
    }
    for (int r = threadIdx.x; r < Ra; r += blockDim.x) dz[((wl * 3 * n) + 3 * nn + x) * Ra + r] = sh[r];
    __syncthreads();
  }
}

// Laplacians per walker: each electron's own rows give
//   Lap Z_r = sum_i E_ri (Lap l_ri + |dl_ri|^2),
//   Lap N_rc = sum_i E_ri (Lap u_ric + 2 dl_ri . du_ric + u_ric (Lap l_ri + |dl_ri|^2)),
// then Lap V = (Lap N - V Lap Z - 2 sum_k d_k V d_k Z) / Z into the last row
// of the walker's jet block, and V itself into its first row.
template <typename T>
__global__ __launch_bounds__(256) void k_ja_lap(const Dims D, int Wc, int w0, const int32_t* __restrict__ ncnt,
                                                const int* __restrict__ joff, const T* __restrict__ aj0,
                                                const T* __restrict__ aj1, const double* __restrict__ ex,
                                                const char* __restrict__ state, StateRec S, T* __restrict__ vj,
                                                const double* __restrict__ dz) {
  __shared__ double sh[64 + 1024];
  const int n = D.n, Ra = D.Ra, NA = D.NA(), NV = D.NV();
  const int64_t wl = blockIdx.x;
  const char* rec = state + (w0 + wl) * S.stride;
  const T* av = (const T*)(rec + S.jae);
  const double* jt = (const double*)(rec + S.jat);
  for (int c = threadIdx.x; c < NA; c += blockDim.x) {
    const bool isz = c < Ra;
    const int r = isz ? c : (c - Ra) / D.dr;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
      const int64_t en = wl * n + i;
      const T* aj = i < D.nu ? aj0 : aj1;
      const int64_t base = joff[en];
      const int nt = 3 * (1 + ncnt[2 * en] + ncnt[2 * en + 1]);
      double sll = 0.0, slu = 0.0;
      for (int q = 0; q < nt; ++q) {
        const double tl = (double)aj[(base + q) * NA + r];
        sll += tl * tl;
        if (!isz) slu += tl * (double)aj[(base + q) * NA + c];
      }
      const double ll = (double)aj[(base + nt) * NA + r];
      const double E = ex[en * Ra + r];
      if (isz) acc += E * (ll + sll);
      else acc += E * ((double)aj[(base + nt) * NA + c] + 2.0 * slu + (double)av[(int64_t)i * NA + c] * (ll + sll));
    }
    sh[c] = acc;
  }
  __syncthreads();
  const int64_t b0 = wl * (3 * n + 2);
  for (int c = threadIdx.x; c < NV; c += blockDim.x) {
    const int r = c / D.dr;
    const double Z = jt[Ra + r], V = jt[2 * Ra + c] / Z;
    double cross = 0.0;
    for (int k = 0; k < 3 * n; ++k) cross += (double)vj[(b0 + 1 + k) * NV + c] * dz[(wl * 3 * n + k) * Ra + r];
    vj[(b0 + 3 * n + 1) * NV + c] = (T)((sh[Ra + c] - V * sh[r] - 2.0 * cross) / Z);
    vj[b0 * NV + c] = (T)V;
  }
}

// SiLU on the dense jet block of each walker (rows: value, 3n tangents,
// Laplacian), in place, width H
template <typename T>
__global__ __launch_bounds__(256) void k_ja_jact(int rows_per, int H, T* __restrict__ y) {
  const int64_t wl = blockIdx.x;
  const int c = threadIdx.x;
  if (c >= H) return;
  const int64_t b0 = wl * rows_per;
  T f, f1, f2;
  silu3(y[b0 * H + c], f, f1, f2);
  y[b0 * H + c] = f;
  T sq = 0;
  for (int k = 1; k < rows_per - 1; ++k) {
    const T t = y[(b0 + k) * H + c];
    sq += t * t;
    y[(b0 + k) * H + c] = f1 * t;
  }
  y[(b0 + rows_per - 1) * H + c] = f1 * y[(b0 + rows_per - 1) * H + c] + f2 * sq;
}

// oj[row] = w3 . y[row] (FP64), one wave per row
template <typename T>
__global__ __launch_bounds__(256) void k_ja_odot(int64_t nrows, int H, const T* __restrict__ y,
                                                 const T* __restrict__ w3, double* __restrict__ oj) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= nrows) return;
  double a = 0.0;
  for (int c = lane; c < H; c += 64) a += (double)w3[c] * (double)y[r * H + c];
  a = wave_sum(a);
  if (lane == 0) oj[r] = a;
}

// grad log|J_att| = do_1 + do_2 / o_2 and Lap = Lap o_1 + Lap o_2 / o_2 -
// |do_2 / o_2|^2 per walker, into (or onto) gJ and lapJ
__global__ __launch_bounds__(256) void k_ja_kinsum(const Dims D, int Wc, int w0, const char* __restrict__ state,
                                                   StateRec S, const double* __restrict__ oj, int64_t nrows,
                                                   double* __restrict__ gJ, double* __restrict__ lapJ, bool first) {
  __shared__ double red[16];
  const int64_t wl = blockIdx.x;
  const int n3 = 3 * D.n;
  const double o2 = ((const double*)(state + (w0 + wl) * S.stride + S.jat))[2 * D.Ra + D.NV() + 1];
  const double inv = o2 != 0.0 && isfinite(o2) ? 1.0 / o2 : 0.0;
  const int64_t b0 = wl * (n3 + 2);
  double acc = 0.0;
  for (int k = threadIdx.x; k < n3; k += blockDim.x) {
    const double t2 = oj[nrows + b0 + 1 + k] * inv;
    const double g = oj[b0 + 1 + k] + t2;
    gJ[wl * n3 + k] = first ? g : gJ[wl * n3 + k] + g;
    acc -= t2 * t2;
  }
  const double tot = block_sum<double>(acc, red);
  if (threadIdx.x == 0) {
    const double lap = oj[b0 + n3 + 1] + oj[nrows + b0 + n3 + 1] * inv + tot;
    lapJ[wl] = first ? lap : lapJ[wl] + lap;
  }
}

template <typename T>
hipError_t ja_kinetic(const fire_handle* h, const Net<T>& P, const JmJetArgs& a, const char* state, char* ws,
                      bool first, hipStream_t s) {
  const Dims& D = h->D;
  if (D.Ra <= 0) return hipSuccess;
  const JaKin L = ja_kin(h, a.Wc, a.rowcap);
  const int n = D.n, NA = D.NA(), NV = D.NV(), Ha = D.Ha;
  T* aj[2] = {(T*)(ws + L.ajet[0]), (T*)(ws + L.ajet[1])};
  for (int sp = 0; sp < 2; ++sp) {
    if (D.nsig(sp) == 0) continue;
    GemmArgs j{};
    j.A = a.jin[sp]; j.amap = rows_dense(D.d); j.Bt = P.ja_Pt; j.ldb = D.d;
    j.C = aj[sp]; j.cmap = rows_dense(NA); j.ccol = cols_dense(); j.M = (int)a.rowcap[sp]; j.N = NA; j.K = D.d;
    j.Mdev = a.jtot + sp;
    CHECK(gemm_site(h, SITE_JET, j, s));
  }
  double* ex = (double*)(ws + L.ex);
  T* vj = (T*)(ws + L.vj);
  double* dz = (double*)(ws + L.dz);
  const int64_t nex = (int64_t)a.Wc * n * D.Ra;
  hipLaunchKernelGGL(k_ja_exp<T>, dim3((unsigned)((nex + 255) / 256)), dim3(256), 0, s, D, a.Wc, a.w0, state, h->st,
                     ex);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_ja_dense<T>, dim3((unsigned)((int64_t)a.Wc * n)), dim3(256), 0, s, D, a.Wc, a.w0, a.memb,
                     a.mslot, a.mcnt, a.tcap, a.joff, (const T*)aj[0], (const T*)aj[1], (const double*)ex, state,
                     h->st, vj, dz);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_ja_lap<T>, dim3(a.Wc), dim3(256), 0, s, D, a.Wc, a.w0, a.ncnt, a.joff, (const T*)aj[0],
                     (const T*)aj[1], (const double*)ex, state, h->st, vj, (const double*)dz);
  CHECK(hipGetLastError());
  const int rp = 3 * n + 2;
  const int64_t rows3 = (int64_t)a.Wc * rp;
  T* y1 = (T*)(ws + L.y1);
  T* y2 = (T*)(ws + L.y2);
  double* oj = (double*)(ws + L.oj);
  const int blk = Ha <= 64 ? 64 : (Ha + 63) / 64 * 64;
  for (int k = 0; k < 2; ++k) {
    GemmArgs g{};
    g.A = vj; g.amap = rows_dense(NV); g.Bt = (const char*)P.ja_W1t + (size_t)k * Ha * NV * h->gsize; g.ldb = NV;
    g.bias = P.ja_b1 + (int64_t)k * Ha; g.bias_period = rp;
    g.C = y1; g.cmap = rows_dense(Ha); g.ccol = cols_dense(); g.M = (int)rows3; g.N = Ha; g.K = NV;
    CHECK(gemm_site(h, SITE_JET, g, s));
    hipLaunchKernelGGL(k_ja_jact<T>, dim3(a.Wc), dim3(blk), 0, s, rp, Ha, y1);
    CHECK(hipGetLastError());
    GemmArgs g2{};
    g2.A = y1; g2.amap = rows_dense(Ha); g2.Bt = (const char*)P.ja_W2t + (size_t)k * Ha * Ha * h->gsize; g2.ldb = Ha;
    g2.bias = P.ja_b2 + (int64_t)k * Ha; g2.bias_period = rp;
    g2.C = y2; g2.cmap = rows_dense(Ha); g2.ccol = cols_dense(); g2.M = (int)rows3; g2.N = Ha; g2.K = Ha;
    CHECK(gemm_site(h, SITE_JET, g2, s));
    hipLaunchKernelGGL(k_ja_jact<T>, dim3(a.Wc), dim3(blk), 0, s, rp, Ha, y2);
    CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_ja_odot<T>, dim3((unsigned)((rows3 + 3) / 4)), dim3(256), 0, s, rows3, Ha, (const T*)y2,
                       P.ja_w3 + (int64_t)k * Ha, oj + (int64_t)k * rows3);
    CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_ja_kinsum, dim3(a.Wc), dim3(256), 0, s, D, a.Wc, a.w0, state, h->st, (const double*)oj, rows3,
                     a.gJ, a.lapJ, first);
  return hipGetLastError();
}

template hipError_t ja_kinetic<double>(const fire_handle*, const Net<double>&, const JmJetArgs&, const char*, char*,
                                       bool, hipStream_t);
template hipError_t ja_kinetic<float>(const fire_handle*, const Net<float>&, const JmJetArgs&, const char*, char*,
                                      bool, hipStream_t);

template hipError_t ja_eval<double>(const fire_handle*, const Net<double>&, int, const double*, char*, char*,
                                    hipStream_t);
template hipError_t ja_eval<float>(const fire_handle*, const Net<float>&, int, const float*, char*, char*,
                                   hipStream_t);
template hipError_t ja_delta<double>(const fire_handle*, const Net<double>&, int, const int*, const int*, const int*,
                                     int, const int*, const int*, const double*, const double*, const char*, char*,
                                     double*, double*, bool, hipStream_t);
template hipError_t ja_delta<float>(const fire_handle*, const Net<float>&, int, const int*, const int*, const int*,
                                    int, const int*, const int*, const float*, const float*, const char*, char*,
                                    double*, double*, bool, hipStream_t);
template hipError_t ja_commit<double>(const fire_handle*, int, const int*, const int*, int, const int*, const int*,
                                      const double*, const double*, const char*, char*, hipStream_t);
template hipError_t ja_commit<float>(const fire_handle*, int, const int*, const int*, int, const int*, const int*,
                                     const float*, const float*, const char*, char*, hipStream_t);

template hipError_t readout_rows<double>(const fire_handle*, const Readout<double>&, const double*, int, const int*,
                                         char*, double*, hipStream_t);
template hipError_t readout_rows<float>(const fire_handle*, const Readout<float>&, const float*, int, const int*,
                                        char*, double*, hipStream_t);
template hipError_t jm_kinetic<double>(const fire_handle*, const Net<double>&, const JmJetArgs&, const char*,
                                       hipStream_t);
template hipError_t jm_kinetic<float>(const fire_handle*, const Net<float>&, const JmJetArgs&, const char*,
                                      hipStream_t);

}  // namespace fire
