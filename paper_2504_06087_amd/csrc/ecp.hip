// Nonlocal pseudopotential energy by angular quadrature of psi ratios
// (Methods, effective core potential; low-rank wave-function updates):
//   V_NL = sum_{i, I: |r_i - R_I| < r_max} sum_l v_l(r_iI) (2l+1)
//          (1/N_q) sum_q P_l(rhat_iI . Q e_q) psi(r_i -> R_I + r_iI Q e_q) / psi
// with the N_q vertices e_q of the species' rule (4 tetrahedron, 6
// octahedron, 12 icosahedron).  Every ratio is one single-electron update
// (neighbour recompute + det A), never a full re-evaluation.
#include <mutex>
#include <vector>

#include "laplacian.hpp"
#include "update.hpp"

namespace fire {

#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

constexpr int NQ = 12;          // the largest rule
constexpr int ECP_PMAX = 8;     // pseudo-atoms within r_max of one electron

struct EcpTables {
  int nchan;
  int species[8], l[8], nterms[8], nq[8];
  double a[8][4], alpha[8][4];
  double rmax;
};

static EcpTables tables(const fire_handle* h) {
  EcpTables t{};
  t.nchan = (int)h->ecp.size() < 8 ? (int)h->ecp.size() : 8;
  for (int k = 0; k < t.nchan; ++k) {
    const EcpChan& c = h->ecp[k];
    t.species[k] = c.species; t.l[k] = c.l; t.nterms[k] = c.nterms; t.nq[k] = c.nquad;
    for (int j = 0; j < 4; ++j) { t.a[k][j] = c.a[j]; t.alpha[k][j] = c.alpha[j]; }
  }
  t.rmax = h->ecp_rmax;
  return t;
}

// icosahedron vertices: cyclic permutations of (0, +-1, +-phi), normalised
FIRE_DEV void ico_vertex(int q, double v[3]) {
  const double phi = 1.6180339887498948482, nrm = 1.0 / sqrt(1.0 + phi * phi);
  const int cyc = q % 3, pair = q / 3;   // pair 0..3 -> the signs of (1, phi)
  const double a = (pair & 2) ? -1.0 : 1.0, b = (pair & 1) ? -phi : phi;
  double t[3];
  if (cyc == 0) { t[0] = 0; t[1] = a; t[2] = b; }
  else if (cyc == 1) { t[0] = a; t[1] = b; t[2] = 0; }
  else { t[0] = b; t[1] = 0; t[2] = a; }
  v[0] = t[0] * nrm; v[1] = t[1] * nrm; v[2] = t[2] * nrm;
}

// tetrahedron (4) and octahedron (6) vertices
FIRE_DEV void quad_vertex(int nq, int q, double v[3]) {
  if (nq == 12) {
    ico_vertex(q, v);
  } else if (nq == 6) {
    v[0] = v[1] = v[2] = 0.0;
    v[q >> 1] = (q & 1) ? -1.0 : 1.0;
  } else {
    const double s = 0.57735026918962576451;   // 1/sqrt(3)
    v[0] = s;
    v[1] = (q == 1 || q == 3) ? -s : s;
    v[2] = (q == 1 || q == 2) ? -s : s;
    if (q >= 2) v[0] = -s;
  }
}

// quadrature points of species sp (0: no nonlocal channel)
FIRE_DEV int nq_of(const EcpTables& t, int sp) {
  for (int k = 0; k < t.nchan; ++k)
    if (t.species[k] == sp) return t.nq[k];
  return 0;
}
FIRE_DEV bool is_ecp_species(const EcpTables& t, int sp) { return nq_of(t, sp) > 0; }

// number of pseudo-atoms within r_max of electron e, per (e, w): cnt[e][w]
__global__ void k_ecp_count(const Dims D, int W, const double* __restrict__ R, const double* __restrict__ Rn,
                            const int* __restrict__ species, EcpTables t, int* __restrict__ cnt,
                            int32_t* __restrict__ status) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= (int64_t)W * D.n) return;
  const int w = (int)(q / D.n), e = (int)(q % D.n);
  const double* r = R + q * 3;
  // jobs of the first ECP_PMAX pseudo-atoms within r_max, N_q per atom
  int c = 0, jobs = 0;
  for (int m = 0; m < D.M; ++m) {
    const int nq = nq_of(t, species[m]);
    if (nq == 0) continue;
    const double dx = r[0] - Rn[3 * m], dy = r[1] - Rn[3 * m + 1], dz = r[2] - Rn[3 * m + 2];
    if (dx * dx + dy * dy + dz * dz < t.rmax * t.rmax) {
      if (c < ECP_PMAX) jobs += nq;
      ++c;
    }
  }
  if (c > ECP_PMAX) atomicOr(status + w, FIRE_W_UPD_OVERFLOW);
  cnt[(int64_t)e * W + w] = jobs;
}

// per electron e: exclusive scan over walkers of the job counts; tot[e]
__global__ __launch_bounds__(1024) void k_ecp_scan(int W, const int* __restrict__ cnt, int* __restrict__ off,
                                                   int* __restrict__ tot) {
  __shared__ int part[1024];
  const int e = blockIdx.x;
  const int* c = cnt + (int64_t)e * W;
  int* o = off + (int64_t)e * (W + 1);
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (W + nt - 1) / nt;
  const int b = t * per, en = b + per < W ? b + per : W;
  int s = 0;
  for (int w = b; w < en; ++w) s += c[w];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int k = 0; k < nt; ++k) { int v = part[k]; part[k] = acc; acc += v; }
    o[W] = acc;
    tot[e] = acc;
  }
  __syncthreads();
  int a = part[t];
  for (int w = b; w < en; ++w) { o[w] = a; a += c[w]; }
}

// jobs [j0, j0 + Jc) of electron e: walker, new position and quadrature
// weight.  The chunk's live job count min(max(tot_e - j0, 0), Jc) comes from
// the device total tot_e and is written to *jdev for the kernels that follow;
// jobs beyond it are inactive (walker 0, weight 0).
__global__ void k_ecp_jobs(const Dims D, int W, int e, int j0, int Jc, const int* __restrict__ tot_e,
                           int* __restrict__ jdev, const double* __restrict__ R,
                           const double* __restrict__ Rn, const int* __restrict__ species, EcpTables t,
                           const double* __restrict__ quad_rot, const int* __restrict__ off, int* __restrict__ jw,
                           double* __restrict__ rexp, double* __restrict__ cf) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Jc) return;
  int J = *tot_e - j0;
  J = J < 0 ? 0 : (J > Jc ? Jc : J);
  if (j == 0) *jdev = J;
  if (j >= J) {
    jw[j] = 0;
    rexp[3 * j] = R[3 * e]; rexp[3 * j + 1] = R[3 * e + 1]; rexp[3 * j + 2] = R[3 * e + 2];
    cf[j] = 0.0;
    return;
  }
  const int jg = j0 + j;
  // walker: last w with off[w] <= jg
  int lo = 0, hi = W - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (off[mid] <= jg) lo = mid; else hi = mid - 1;
  }
  const int w = lo;
  // the pseudo-atom and point of this job: walk the atoms within r_max in
  // the order k_ecp_count counted them, N_q jobs each
  int loc = jg - off[w];
  const double* r = R + ((int64_t)w * D.n + e) * 3;
  int c = 0, I = -1, q = 0, nqI = NQ;
  for (int m = 0; m < D.M && I < 0 && c < ECP_PMAX; ++m) {
    const int nq = nq_of(t, species[m]);
    if (nq == 0) continue;
    const double dx = r[0] - Rn[3 * m], dy = r[1] - Rn[3 * m + 1], dz = r[2] - Rn[3 * m + 2];
    if (dx * dx + dy * dy + dz * dz < t.rmax * t.rmax) {
      if (loc < nq) { I = m; q = loc; nqI = nq; }
      else loc -= nq;
      ++c;
    }
  }
  jw[j] = w;
  if (I < 0) {   // cannot happen when the counts are consistent: a no-op job
    rexp[3 * j] = r[0]; rexp[3 * j + 1] = r[1]; rexp[3 * j + 2] = r[2];
    cf[j] = 0.0;
    return;
  }
  const double dx = r[0] - Rn[3 * I], dy = r[1] - Rn[3 * I + 1], dz = r[2] - Rn[3 * I + 2];
  const double rr = sqrt(dx * dx + dy * dy + dz * dz);
  double v[3], u[3];
  quad_vertex(nqI, q, v);
  if (quad_rot) {
    const double* Q = quad_rot + (int64_t)w * 9;
    for (int k = 0; k < 3; ++k) u[k] = Q[3 * k] * v[0] + Q[3 * k + 1] * v[1] + Q[3 * k + 2] * v[2];
  } else {
    u[0] = v[0]; u[1] = v[1]; u[2] = v[2];
  }
  rexp[3 * j] = Rn[3 * I] + rr * u[0];
  rexp[3 * j + 1] = Rn[3 * I + 1] + rr * u[1];
  rexp[3 * j + 2] = Rn[3 * I + 2] + rr * u[2];
  const double cs = rr > 0 ? (dx * u[0] + dy * u[1] + dz * u[2]) / rr : 0.0;
  double coef = 0.0;
  for (int k = 0; k < t.nchan; ++k) {
    if (t.species[k] != species[I]) continue;
    double vl = 0.0;
    for (int m = 0; m < t.nterms[k]; ++m) vl += t.a[k][m] * exp(-t.alpha[k][m] * rr * rr);
    const double Pl = t.l[k] == 0 ? 1.0 : cs;
    coef += vl * (2 * t.l[k] + 1) * Pl / nqI;
  }
  cf[j] = coef;
}

// contribution of each job: coefficient * psi'/psi with
// psi'/psi = e^{dJ} sum_d w_d prod_s det A_ds,  w_d = s_d e^{l_d} / sum_d s_d e^{l_d}
// (dJ: the job's change of the Jastrow log magnitude; jsg, when set, the
// sign change of the MLP Jastrow's node factor)
__global__ void k_ecp_ratio(const Dims D, int J, int j0, const int* __restrict__ jdev, const int* __restrict__ jw,
                            const double* __restrict__ cf, const double* __restrict__ detA,
                            const double* __restrict__ dj, const double* __restrict__ jsg,
                            const char* __restrict__ state, StateRec S, double* __restrict__ contrib) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J || j >= *jdev) return;
  const int w = jw[j];
  const char* rec = state + (int64_t)w * S.stride;
  const double* ds = (const double*)(rec + S.dsign);
  const double* dl = (const double*)(rec + S.dlog);
  const double lp = *(const double*)(rec + S.lpsi), sp = *(const double*)(rec + S.spsi);
  const double* dA = detA + (int64_t)j * D.K * 4;
  double r = 0.0;
  for (int k = 0; k < D.K; ++k) {
    const double sg = ds[2 * k] * ds[2 * k + 1] * sp * dA[4 * k] * dA[4 * k + 2];
    if (sg != 0.0) r += sg * exp(dl[2 * k] + dl[2 * k + 1] - lp + dA[4 * k + 1] + dA[4 * k + 3]);
  }
  contrib[j0 + j] = cf[j] * r * exp(dj[j]) * (jsg ? jsg[j] : 1.0);
}

__global__ void k_ecp_reduce(int W, const int* __restrict__ off, const double* __restrict__ contrib,
                             double* __restrict__ vnl) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  double s = 0.0;
  for (int j = off[w]; j < off[w + 1]; ++j) s += contrib[j];
  vnl[w] += s;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

std::mutex& handle_mutex() {
  static std::mutex m;
  return m;
}

__global__ void k_add_f64(double* p, const double* q, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] += q[i];
}

// Shared job counts, then one or two lanes of job buffers.  With overlap on,
// electrons alternate between two lanes, which run on two streams; otherwise
// one lane of twice the chunk takes them all on the caller's stream.  Both
// layouts take about the same bytes; the workspace holds the larger.
struct EcpLayout {
  int Jc;
  size_t cnt, off, tot;
  size_t lane[2];                                  // lane bases
  size_t jw, rexp, cf, contrib, vnl, jdev, upd;    // offsets within a lane
  size_t total;
};

// Jobs per electron are at most W * ecp_pmax * (largest rule): an electron
// lies within r_max of at most ecp_pmax pseudo-atoms (a bound fixed by the
// geometry at handle creation).
static int64_t ecp_job_bound(const fire_handle* h, int W) {
  int nqmax = 0;
  for (const EcpChan& c : h->ecp) nqmax = c.nquad > nqmax ? c.nquad : nqmax;
  const int pm = h->ecp_pmax < ECP_PMAX ? h->ecp_pmax : ECP_PMAX;
  const int64_t b = (int64_t)W * (pm > 0 ? pm : 1) * (nqmax > 0 ? nqmax : 1);
  return b > 0 ? b : 1;
}

static EcpLayout ecp_layout(const fire_handle* h, int W, int lanes) {
  EcpLayout L{};
  const Dims& D = h->D;
  // Jobs per chunk and lane.  A chunk's update segments hold kRowsPerJob
  // rows per job and spin of K N_s orbital values each: the cap keeps every
  // element index of a segment below 2^31 and a lane's segments within
  // 24 GiB.  The chunks of an electron's bound are made equal and a
  // multiple of 12 (the sizes of the 4-, 6- and 12-point rules divide it).
  const UpdLayout u1k = upd_layout(h, 1024, false);
  int64_t per_row = 1;
  for (int s = 0; s < 2; ++s) {
    const int64_t r = (u1k.rowcap[s] / 1024) * D.K * (D.nsig(s) > 0 ? D.nsig(s) : 1);
    per_row = r > per_row ? r : per_row;
  }
  const int64_t cap_idx = (int64_t)0x7fffffff / per_row;
  const int64_t cap_mem = ((int64_t)24 << 30) / (int64_t)(u1k.total / 1024 + 64);
  int64_t cap = (cap_idx < cap_mem ? cap_idx : cap_mem) / lanes;
  if (h->ecp_chunk_cap > 0 && h->ecp_chunk_cap < cap) cap = h->ecp_chunk_cap;
  cap = cap / 12 * 12;
  if (cap < 12) cap = 12;
  const int64_t bound = ecp_job_bound(h, W);
  const int64_t nch = (bound + cap - 1) / cap;
  const int64_t jc = ((bound + nch - 1) / nch + 11) / 12 * 12;
  L.Jc = (int)(jc < cap ? jc : cap);
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align_up(o + b); return r; };
  L.cnt = take((size_t)D.n * W * 4);
  L.off = take((size_t)D.n * (W + 1) * 4);
  L.tot = take((size_t)D.n * 4);
  size_t q = 0;
  auto ltake = [&](size_t b) { size_t r = q; q = align_up(q + b); return r; };
  L.jw = ltake((size_t)L.Jc * 4);
  L.rexp = ltake((size_t)L.Jc * 3 * 8);
  L.cf = ltake((size_t)L.Jc * 8);
  L.contrib = ltake((size_t)W * ECP_PMAX * NQ * 8);
  L.vnl = ltake((size_t)W * 8);
  L.jdev = ltake(4);
  L.upd = q;
  q = align_up(q + upd_layout(h, L.Jc, false).total);
  L.lane[0] = o;
  L.lane[1] = o + (lanes == 2 ? q : 0);
  L.total = align_up(o + lanes * q);
  return L;
}

size_t ecp_ws_bytes(const fire_handle* h, int W) {
  if (h->ecp.empty()) return 0;
  const size_t a = ecp_layout(h, W, 1).total, b = ecp_layout(h, W, 2).total;
  return a > b ? a : b;
}

// Chunks per electron: the chunk loop covers the job bound and each chunk
// reads its live job count on the device, so no count is read back to the
// host.
static int ecp_chunks(const fire_handle* h, int W, int Jc) {
  return (int)((ecp_job_bound(h, W) + Jc - 1) / Jc);
}

template <typename T>
static hipError_t ecp_impl(const fire_handle* h, int W, const double* R, char* state, char* ws,
                           const double* quad_rot, double* vnl, int32_t* status, hipStream_t st) {
  const Dims& D = h->D;
  const StateRec& S = h->st;
  Net<T> P = make_net<T>(h);
  const int lanes = (h->overlap && h->side_ecp) ? 2 : 1;
  AutotuneHold hold(lanes == 2);
  const EcpLayout L = ecp_layout(h, W, lanes);
  const EcpTables tb = tables(h);
  const UpdLayout U = upd_layout(h, L.Jc, false);
  int* cnt = (int*)(ws + L.cnt);
  int* off = (int*)(ws + L.off);
  int* tot = (int*)(ws + L.tot);
  const int* sp_dev = (const int*)((const char*)h->params + h->pl.species);
  // lane 0 accumulates into vnl on the caller's stream, lane 1 into its own
  // sum on the handle's pseudopotential stream, which starts after the
  // counts (fork event)
  double* vl[2] = {vnl, (double*)(ws + L.lane[1] + L.vnl)};
  for (int l = 0; l < lanes; ++l) {
    hipLaunchKernelGGL(k_fill_f64, dim3((W + 255) / 256), dim3(256), 0, st, vl[l], (int64_t)W, 0.0);
    CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_ecp_count, dim3((unsigned)(((int64_t)W * D.n + 255) / 256)), dim3(256), 0, st, D, W, R, P.Rn,
                     sp_dev, tb, cnt, status);
  CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_ecp_scan, dim3(D.n), dim3(1024), 0, st, W, (const int*)cnt, off, tot);
  CHECK(hipGetLastError());
  hipStream_t ls[2] = {st, st};
  if (lanes == 2) {
    // record and wait as one step, so that concurrent calls on other streams
    // cannot move the fork point
    std::lock_guard<std::mutex> lock(handle_mutex());
    CHECK(hipEventRecord(h->side_ecp_fork, st));
    CHECK(hipStreamWaitEvent(h->side_ecp, h->side_ecp_fork, 0));
    ls[1] = h->side_ecp;
  }
  const int nch = ecp_chunks(h, W, L.Jc);
  for (int e = 0; e < D.n; ++e) {
    const int ln = lanes == 2 ? (e & 1) : 0;
    hipStream_t ss = ls[ln];
    char* lb = ws + L.lane[ln];
    int* jw = (int*)(lb + L.jw);
    double* rexp = (double*)(lb + L.rexp);
    double* cf = (double*)(lb + L.cf);
    double* contrib = (double*)(lb + L.contrib);
    int* jdev = (int*)(lb + L.jdev);
    char* uws = lb + L.upd;
    const int* offe = off + (int64_t)e * (W + 1);
    for (int c = 0; c < nch; ++c) {
      const int j0 = c * L.Jc;
      hipLaunchKernelGGL(k_ecp_jobs, dim3((L.Jc + 255) / 256), dim3(256), 0, ss, D, W, e, j0, L.Jc,
                         (const int*)(tot + e), jdev, R, P.Rn, sp_dev, tb, quad_rot, offe, jw, rexp, cf);
      CHECK(hipGetLastError());
      Jobs jb{};
      jb.J = L.Jc;
      jb.Jcap = L.Jc;
      jb.Jdev = jdev;
      jb.group = tb.nq[0];   // the jobs of one (electron, pseudo-atom) pair are consecutive
      jb.jw = jw;
      jb.rexp = rexp;
      CHECK(propose_ratio<T>(h, P, jb, e, R, state, uws, status, ss));
      hipLaunchKernelGGL(k_ecp_ratio, dim3((L.Jc + 255) / 256), dim3(256), 0, ss, D, L.Jc, j0, (const int*)jdev,
                         (const int*)jw, (const double*)cf, (const double*)(uws + U.detA),
                         (const double*)(uws + U.dj),
                         h->D.Hj > 0 || h->D.Ra > 0 ? (const double*)(uws + U.jsg) : (const double*)nullptr,
                         (const char*)state,
                         S, contrib);
      CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ecp_reduce, dim3((W + 255) / 256), dim3(256), 0, ss, W, offe, (const double*)contrib, vl[ln]);
    CHECK(hipGetLastError());
  }
  // join lane 1 (a later record of the join event lies later on the serial
  // lane-1 stream, so the wait is never too early) and add its sum
  if (lanes == 2) {
    CHECK(hipEventRecord(h->side_ecp_join, ls[1]));
    CHECK(hipStreamWaitEvent(st, h->side_ecp_join, 0));
    hipLaunchKernelGGL(k_add_f64, dim3((W + 255) / 256), dim3(256), 0, st, vnl, (const double*)vl[1], (int64_t)W);
  }
  return hipGetLastError();
}

hipError_t ecp_into(const fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                    double* vnl, int32_t* status, hipStream_t st) {
  if (!update_fits(h)) return hipErrorInvalidValue;
  return h->tsize == 8 ? ecp_impl<double>(h, W, R, state, ws, quad_rot, vnl, status, st)
                       : ecp_impl<float>(h, W, R, state, ws, quad_rot, vnl, status, st);
}

hipError_t ecp_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                    double* v_nl, int32_t* status, hipStream_t s) {
  CHECK(fill_i32(status, W, 0, s));
  if (h->ecp.empty()) {
    hipLaunchKernelGGL(k_fill_f64, dim3((W + 255) / 256), dim3(256), 0, s, v_nl, (int64_t)W, 0.0);
    return hipGetLastError();
  }
  return ecp_into(h, W, R, state, ws, quad_rot, v_nl, status, s);
}

}  // namespace fire
