// Uneven multi-system batches: several molecules with different electron
// counts advanced together, one step = full evaluation, Metropolis sweeps,
// local energy, energy-gradient coefficients and the parameter gradient, for
// every system, enqueued as one fork/join DAG over a few streams and
// optionally captured once into HIP graphs (one per stream branch) that
// replay the whole step with one call.  The embedding parameters (filters, per-species nuclear
// tables, GLU, messages, MLP) are shared by all systems; orbital weights and
// envelopes are per system (Methods, wave function ansatz: the embedding
// network is molecule-agnostic, the orbital layer depends on the molecule).
#include <algorithm>
#include <vector>

#include "forward.hpp"
#include "handle.hpp"

struct fire_batch {
  int n = 0;
  std::vector<fire_handle*> sys;
  std::vector<int> n_el;
  int64_t P_shared = 0;            // leading theta entries shared by every system
  std::vector<int64_t> P_sys;      // full theta size of each system
  std::vector<int64_t> priv_off;   // offset of system s's private block in the batch theta
  int64_t P_total = 0;
  int n_branch = 0;
  std::vector<hipStream_t> streams;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
};


namespace fire {

size_t workspace_bytes_for(const fire_handle* h, int W);

constexpr int kMaxSystems = 32;

// Byte offsets of one system's regions inside the batch buffers.
struct SysOff {
  size_t params, state, ws, gtmp, coeff, sign, lpsi, st[4];
  int64_t walker0, r0, noise0, unif0;
};

// Systems are dealt to the branches longest-first onto the least-loaded
// branch, with cost ~ W n^2 (sweep and Laplacian both scale so).
static std::vector<int> schedule(const fire_batch* b, const int* W, std::vector<int>* order) {
  std::vector<int> idx(b->n), br(b->n, 0);
  for (int s = 0; s < b->n; ++s) idx[s] = s;
  auto cost = [&](int s) { return (double)W[s] * b->n_el[s] * b->n_el[s]; };
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<double> load(b->n_branch, 0.0);
  for (int s : idx) {
    int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    br[s] = k;
    load[k] += cost(s);
  }
  if (order) *order = idx;
  return br;
}

// The systems of one branch run one after another on its stream, so they
// share one scratch workspace (the largest they need); the per-system
// results that outlive a system's turn (gradient, coefficients, status) have
// regions of their own.
static std::vector<SysOff> batch_offsets(const fire_batch* b, const int* W, int n_sweeps, size_t* params_total,
                                         size_t* state_total, size_t* ws_total) {
  std::vector<SysOff> o(b->n);
  const std::vector<int> br = schedule(b, W, nullptr);
  std::vector<size_t> branch_ws(b->n_branch, 0);
  for (int s = 0; s < b->n; ++s) branch_ws[br[s]] = std::max(branch_ws[br[s]], workspace_bytes_for(b->sys[s], W[s]));
  std::vector<size_t> branch_off(b->n_branch, 0);
  size_t pa = 0, sa = 0, wa = 0;
  for (int k = 0; k < b->n_branch; ++k) {
    branch_off[k] = wa;
    wa = align_up(wa + branch_ws[k]);
  }
  int64_t w0 = 0, r0 = 0, n0 = 0, u0 = 0;
  for (int s = 0; s < b->n; ++s) {
    const fire_handle* h = b->sys[s];
    SysOff& x = o[s];
    x.params = pa;
    pa = align_up(pa + h->pl.total);
    x.state = sa;
    sa = align_up(sa + h->st.stride * (size_t)W[s]);
    x.ws = branch_off[br[s]];
    x.gtmp = wa;
    wa = align_up(wa + (size_t)h->P * 8);
    x.coeff = wa;
    wa = align_up(wa + (size_t)W[s] * 8);
    x.sign = wa;
    wa = align_up(wa + (size_t)W[s] * 8);
    x.lpsi = wa;
    wa = align_up(wa + (size_t)W[s] * 8);
    for (int k = 0; k < 4; ++k) {
      x.st[k] = wa;
      wa = align_up(wa + (size_t)W[s] * 4);
    }
    x.walker0 = w0;
    x.r0 = r0;
    x.noise0 = n0;
    x.unif0 = u0;
    w0 += W[s];
    r0 += (int64_t)W[s] * b->n_el[s] * 3;
    n0 += (int64_t)n_sweeps * b->n_el[s] * W[s] * 3;
    u0 += (int64_t)n_sweeps * b->n_el[s] * W[s];
  }
  if (params_total) *params_total = pa;
  if (state_total) *state_total = sa;
  if (ws_total) *ws_total = wa;
  return o;
}

// c_w = (E_L,w - mean E_L) / W over the walkers of one system (Methods,
// energy gradient).  Flagged walkers (non-finite E_L) are left out of the
// mean and get c_w = 0.  One workgroup.
__global__ __launch_bounds__(256) void k_energy_coeff(const double* __restrict__ e, int W, double* __restrict__ c) {
  __shared__ double ssum[256];
  __shared__ int scnt[256];
  double a = 0.0;
  int k = 0;
  for (int w = threadIdx.x; w < W; w += 256) {
    const double v = e[w];
    if (isfinite(v)) { a += v; ++k; }
  }
  ssum[threadIdx.x] = a;
  scnt[threadIdx.x] = k;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ssum[threadIdx.x] += ssum[threadIdx.x + o];
      scnt[threadIdx.x] += scnt[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double mean = scnt[0] > 0 ? ssum[0] / scnt[0] : 0.0;
  for (int w = threadIdx.x; w < W; w += 256) {
    const double v = e[w];
    c[w] = isfinite(v) ? (v - mean) / W : 0.0;
  }
}

__global__ void k_or_status(int W, const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                            const int32_t* __restrict__ c, const int32_t* __restrict__ d, int32_t* __restrict__ out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < W) out[w] = a[w] | b[w] | c[w] | d[w];
}

struct BatchGrad {
  int n;
  int64_t P_shared;
  const double* g[kMaxSystems];
  int64_t priv_off[kMaxSystems + 1];
};

}  // namespace fire

// A captured batch step: one graph per stream branch (its systems in order),
// replayed on the batch's branch streams, then the gradient combine.  A graph
// with parallel branches is replayed one branch after another by the
// runtime, so the branches are captured and launched separately.
struct fire_graph {
  fire_batch* b = nullptr;
  std::vector<hipGraph_t> g;
  std::vector<hipGraphExec_t> x;
  std::vector<int> branch;      // stream branch of graph k
  fire::BatchGrad tail{};
  int64_t P_total = 0;
  double* grad = nullptr;
};

namespace fire {

// batch gradient: shared entries summed over systems in system order,
// private entries copied from their system
__global__ void k_batch_grad(BatchGrad a, int64_t P_total, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= P_total) return;
  if (i < a.P_shared) {
    double v = 0.0;
    for (int s = 0; s < a.n; ++s) v += a.g[s][i];
    out[i] = v;
    return;
  }
  int s = 0;
  while (s + 1 < a.n && i >= a.priv_off[s + 1]) ++s;
  out[i] = a.g[s][a.P_shared + (i - a.priv_off[s])];
}

struct StepArgs {
  const int* W;
  double* R;
  char* state;
  char* ws;
  int n_sweeps;
  double step;
  const double* noise;
  const double* unif;
  int32_t* n_accept;
  double* e_loc;
  double* grad;
  int32_t* status;
};

static fire_status enqueue_system(fire_batch* b, int s, const SysOff& o, const StepArgs& a, hipStream_t st) {
  fire_handle* h = b->sys[s];
  const int W = a.W[s];
  double* R = a.R + o.r0;
  char* state = a.state + o.state;
  char* ws = a.ws + o.ws;
  char* wb = a.ws;
  int32_t* s0 = (int32_t*)(wb + o.st[0]);
  int32_t* s1 = (int32_t*)(wb + o.st[1]);
  int32_t* s2 = (int32_t*)(wb + o.st[2]);
  int32_t* s3 = (int32_t*)(wb + o.st[3]);
  double* sign = (double*)(wb + o.sign);
  double* lpsi = (double*)(wb + o.lpsi);
  double* coeff = (double*)(wb + o.coeff);
  double* e = a.e_loc + o.walker0;
  fire_status r = fire_eval_logpsi(h, W, R, state, ws, sign, lpsi, s0, st);
  if (r != FIRE_OK) return r;
  if (a.n_sweeps > 0) {
    r = fire_mcmc_sweep(h, W, R, state, ws, a.n_sweeps, a.step, a.noise + o.noise0, a.unif + o.unif0, 0, 0,
                        a.n_accept + o.walker0, lpsi, sign, s1, st);
    if (r != FIRE_OK) return r;
  } else if (fill_i32(s1, W, 0, st) != hipSuccess) {
    return FIRE_ERR_HIP;
  }
  r = fire_local_energy(h, W, R, state, ws, nullptr, e, nullptr, nullptr, s2, st);
  if (r != FIRE_OK) return r;
  hipLaunchKernelGGL(k_energy_coeff, dim3(1), dim3(256), 0, st, (const double*)e, W, coeff);
  if (hipGetLastError() != hipSuccess) return FIRE_ERR_HIP;
  r = fire_grad_params(h, W, R, state, ws, coeff, (double*)(wb + o.gtmp), nullptr, s3, st);
  if (r != FIRE_OK) return r;
  hipLaunchKernelGGL(k_or_status, dim3((W + 255) / 256), dim3(256), 0, st, W, (const int32_t*)s0,
                     (const int32_t*)s1, (const int32_t*)s2, (const int32_t*)s3, a.status + o.walker0);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

static fire_status check_sizes(const fire_batch* b, const StepArgs& a) {
  for (int s = 0; s < b->n; ++s)
    if (a.W[s] < 1 || a.W[s] > b->sys[s]->model.max_walkers) return FIRE_ERR_CAPACITY;
  return FIRE_OK;
}

static BatchGrad grad_args(const fire_batch* b, const std::vector<SysOff>& off, const StepArgs& a) {
  BatchGrad g{};
  g.n = b->n;
  g.P_shared = b->P_shared;
  for (int s = 0; s < b->n; ++s) {
    g.g[s] = (const double*)(a.ws + off[s].gtmp);
    g.priv_off[s] = b->priv_off[s];
  }
  g.priv_off[b->n] = b->P_total;
  return g;
}

static fire_status enqueue_combine(const fire_batch* b, const BatchGrad& g, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_grad, dim3((unsigned)((b->P_total + 255) / 256)), dim3(256), 0, st, g, b->P_total, grad);
  return hipGetLastError() == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

static fire_status enqueue_step(fire_batch* b, const StepArgs& a, hipStream_t origin) {
  fire_status r = check_sizes(b, a);
  if (r != FIRE_OK) return r;
  const std::vector<SysOff> off = batch_offsets(b, a.W, a.n_sweeps, nullptr, nullptr, nullptr);
  std::vector<int> order;
  const std::vector<int> br = schedule(b, a.W, &order);
  if (hipEventRecord(b->fork, origin) != hipSuccess) return FIRE_ERR_HIP;
  for (int k = 0; k < b->n_branch; ++k)
    if (hipStreamWaitEvent(b->streams[k], b->fork, 0) != hipSuccess) return FIRE_ERR_HIP;
  for (int s : order) {
    r = enqueue_system(b, s, off[s], a, b->streams[br[s]]);
    if (r != FIRE_OK) break;
  }
  // always join, so that the streams stay ordered after an error
  for (int k = 0; k < b->n_branch; ++k) {
    if (hipEventRecord(b->join[k], b->streams[k]) != hipSuccess) return FIRE_ERR_HIP;
    if (hipStreamWaitEvent(origin, b->join[k], 0) != hipSuccess) return FIRE_ERR_HIP;
  }
  if (r != FIRE_OK) return r;
  return enqueue_combine(b, grad_args(b, off, a), a.grad, origin);
}

static void graph_free(fire_graph* G) {
  for (hipGraphExec_t x : G->x)
    if (x) (void)hipGraphExecDestroy(x);
  for (hipGraph_t g : G->g)
    if (g) (void)hipGraphDestroy(g);
  delete G;
}

// Capture branch k's systems (in schedule order) on its own stream.
static fire_status capture_branch(fire_batch* b, int k, const std::vector<int>& order, const std::vector<int>& br,
                                  const std::vector<SysOff>& off, const StepArgs& a, fire_graph* G) {
  hipStream_t st = b->streams[k];
  if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) return FIRE_ERR_HIP;
  fire_status r = FIRE_OK;
  for (int s : order)
    if (br[s] == k && r == FIRE_OK) r = enqueue_system(b, s, off[s], a, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (r != FIRE_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return r != FIRE_OK ? r : FIRE_ERR_HIP;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return FIRE_ERR_HIP;
  }
  G->g.push_back(g);
  G->x.push_back(x);
  G->branch.push_back(k);
  return FIRE_OK;
}

}  // namespace fire

using namespace fire;

extern "C" {

fire_status fire_batch_create(const fire_system_desc* systems, int n_systems, const fire_model_desc* model,
                              fire_batch** out) {
  if (!systems || !model || !out || n_systems < 1) return FIRE_ERR_ARG;
  if (n_systems > kMaxSystems) return FIRE_ERR_CAPACITY;
  fire_batch* b = new fire_batch();
  b->n = n_systems;
  fire_status r = FIRE_OK;
  for (int s = 0; s < n_systems && r == FIRE_OK; ++s) {
    fire_model_desc md = *model;
    const int n = systems[s].n_up + systems[s].n_dn;
    md.cap_nbr = std::max(1, std::min(md.cap_nbr, n - 1));
    md.cap_upd = std::max(1, std::min(md.cap_upd, n));
    fire_handle* h = nullptr;
    r = fire_create(&systems[s], &md, &h);
    if (r != FIRE_OK) break;
    h->lap_budget = (size_t)12 << 30;   // per branch at most one system's Laplacian chunk is live
    b->sys.push_back(h);
    b->n_el.push_back(n);
  }
  if (r == FIRE_OK) {
    // every entry before the orbital block is shared and must agree in shape
    const fire_handle* h0 = b->sys[0];
    b->P_shared = theta_offset(h0, "orb_W_up");
    for (fire_handle* h : b->sys) {
      if (theta_offset(h, "orb_W_up") != b->P_shared) { r = FIRE_ERR_SHAPE; break; }
      for (size_t k = 0; k < h->theta.size() && r == FIRE_OK; ++k)
        if (h->theta[k].offset < b->P_shared && h->theta[k].shape != h0->theta[k].shape) r = FIRE_ERR_SHAPE;
    }
  }
  if (r == FIRE_OK) {
    int64_t o = b->P_shared;
    for (fire_handle* h : b->sys) {
      b->P_sys.push_back(h->P);
      b->priv_off.push_back(o);
      o += h->P - b->P_shared;
    }
    b->P_total = o;
    b->n_branch = std::min(n_systems, 4);
    for (int k = 0; k < b->n_branch && r == FIRE_OK; ++k) {
      hipStream_t st;
      hipEvent_t ev;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { r = FIRE_ERR_HIP; break; }
      b->streams.push_back(st);
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { r = FIRE_ERR_HIP; break; }
      b->join.push_back(ev);
    }
    if (r == FIRE_OK && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) r = FIRE_ERR_HIP;
  }
  if (r != FIRE_OK) {
    fire_batch_destroy(b);
    return r;
  }
  *out = b;
  return FIRE_OK;
}

fire_status fire_batch_destroy(fire_batch* b) {
  if (!b) return FIRE_ERR_ARG;
  for (fire_handle* h : b->sys) fire_destroy(h);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
  return FIRE_OK;
}

fire_status fire_batch_num_params(const fire_batch* b, int64_t* P_total, int64_t* P_shared) {
  if (!b || !P_total) return FIRE_ERR_ARG;
  *P_total = b->P_total;
  if (P_shared) *P_shared = b->P_shared;
  return FIRE_OK;
}

fire_status fire_batch_system(const fire_batch* b, int s, fire_handle** h, int64_t* priv_offset) {
  if (!b || s < 0 || s >= b->n) return FIRE_ERR_ARG;
  if (h) *h = b->sys[s];
  if (priv_offset) *priv_offset = b->priv_off[s];
  return FIRE_OK;
}

fire_status fire_batch_sizes(const fire_batch* b, const int* W, int n_sweeps, size_t* params_bytes,
                             size_t* state_bytes, size_t* workspace_bytes) {
  if (!b || !W || n_sweeps < 0) return FIRE_ERR_ARG;
  for (int s = 0; s < b->n; ++s)
    if (W[s] < 1) return FIRE_ERR_ARG;
  batch_offsets(b, W, n_sweeps, params_bytes, state_bytes, workspace_bytes);
  return FIRE_OK;
}

fire_status fire_batch_set_params(fire_batch* b, const double* theta, void* params_buf, hipStream_t stream) {
  if (!b || !theta || !params_buf) return FIRE_ERR_ARG;
  size_t pa = 0;
  for (int s = 0; s < b->n; ++s) {
    fire_status r = set_params_split(b->sys[s], theta, theta + b->priv_off[s], (char*)params_buf + pa, stream);
    if (r != FIRE_OK) return r;
    pa = align_up(pa + b->sys[s]->pl.total);
  }
  return FIRE_OK;
}

fire_status fire_batch_step(fire_batch* b, const int* W, double* R, void* state, void* ws, int n_sweeps,
                            double step, const double* noise, const double* unif, int32_t* n_accept,
                            double* e_loc, double* grad, int32_t* status, hipStream_t stream) {
  if (!b || !W || !R || !state || !ws || !e_loc || !grad || !status || n_sweeps < 0) return FIRE_ERR_ARG;
  if (n_sweeps > 0 && (!noise || !unif || !n_accept)) return FIRE_ERR_ARG;
  for (fire_handle* h : b->sys)
    if (!h->params) return FIRE_ERR_STATE;
  StepArgs a{W, R, (char*)state, (char*)ws, n_sweeps, step, noise, unif, n_accept, e_loc, grad, status};
  return enqueue_step(b, a, stream);
}

fire_status fire_batch_graph_create(fire_batch* b, const int* W, double* R, void* state, void* ws, int n_sweeps,
                                    double step, const double* noise, const double* unif, int32_t* n_accept,
                                    double* e_loc, double* grad, int32_t* status, fire_graph** out) {
  if (!out) return FIRE_ERR_ARG;
  if (!b || !W || !R || !state || !ws || !e_loc || !grad || !status || n_sweeps < 0) return FIRE_ERR_ARG;
  if (n_sweeps > 0 && (!noise || !unif || !n_accept)) return FIRE_ERR_ARG;
  for (fire_handle* h : b->sys)
    if (!h->params) return FIRE_ERR_STATE;
  StepArgs a{W, R, (char*)state, (char*)ws, n_sweeps, step, noise, unif, n_accept, e_loc, grad, status};
  fire_status r = check_sizes(b, a);
  if (r != FIRE_OK) return r;
  const std::vector<SysOff> off = batch_offsets(b, a.W, a.n_sweeps, nullptr, nullptr, nullptr);
  std::vector<int> order;
  const std::vector<int> br = schedule(b, a.W, &order);
  fire_graph* G = new fire_graph();
  G->b = b;
  for (int k = 0; k < b->n_branch && r == FIRE_OK; ++k) r = capture_branch(b, k, order, br, off, a, G);
  if (r != FIRE_OK) {
    graph_free(G);
    return r;
  }
  G->tail = grad_args(b, off, a);
  G->grad = grad;
  *out = G;
  return FIRE_OK;
}

fire_status fire_graph_launch(fire_graph* g, hipStream_t stream) {
  if (!g || !g->b || g->x.empty()) return FIRE_ERR_ARG;
  fire_batch* b = g->b;
  if (hipEventRecord(b->fork, stream) != hipSuccess) return FIRE_ERR_HIP;
  fire_status r = FIRE_OK;
  for (size_t k = 0; k < g->x.size(); ++k) {
    hipStream_t st = b->streams[g->branch[k]];
    if (hipStreamWaitEvent(st, b->fork, 0) != hipSuccess || hipGraphLaunch(g->x[k], st) != hipSuccess) r = FIRE_ERR_HIP;
    if (hipEventRecord(b->join[g->branch[k]], st) != hipSuccess ||
        hipStreamWaitEvent(stream, b->join[g->branch[k]], 0) != hipSuccess)
      return FIRE_ERR_HIP;
  }
  if (r != FIRE_OK) return r;
  return enqueue_combine(b, g->tail, g->grad, stream);
}

fire_status fire_graph_destroy(fire_graph* g) {
  if (!g) return FIRE_ERR_ARG;
  graph_free(g);
  return FIRE_OK;
}

fire_status fire_autotune(int on) { return autotune_set(on) == hipSuccess ? FIRE_OK : FIRE_ERR_HIP; }

fire_status fire_autotune_count(int* n) {
  if (!n) return FIRE_ERR_ARG;
  *n = autotune_count();
  return FIRE_OK;
}

fire_status fire_autotune_clear(void) {
  autotune_clear();
  return FIRE_OK;
}

fire_status fire_autotune_save(const char* path) {
  if (!path) return FIRE_ERR_ARG;
  return autotune_save(path) ? FIRE_OK : FIRE_ERR_ARG;
}

fire_status fire_autotune_load(const char* path) {
  if (!path) return FIRE_ERR_ARG;
  return autotune_load(path) ? FIRE_OK : FIRE_ERR_ARG;
}

}  // extern "C"
