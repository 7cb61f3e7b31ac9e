// C-ABI of libfire: handle, parameter layout, buffer sizes, parameter packing
// and the entry points.  All device work runs in the other translation units.
#include <string.h>

#include <mutex>

#include <string>
#include <vector>

#include "forward.hpp"
#include "paths.hpp"

using namespace fire;

// ---------------------------------------------------------------------------
// parameter packing: dst[i0*t0 + i1*t1 + i2*t2] = src[i0*s0 + i1*s1 + i2*s2]
// ---------------------------------------------------------------------------
template <typename TD, bool LO>
__global__ void k_strided(TD* dst, const double* __restrict__ src, int n0, int n1, int n2, int64_t s0, int64_t s1,
                          int64_t s2, int64_t t0, int64_t t1, int64_t t2) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t tot = (int64_t)n0 * n1 * n2;
  if (q >= tot) return;
  int i2 = (int)(q % n2);
  int64_t r = q / n2;
  int i1 = (int)(r % n1);
  int i0 = (int)(r / n1);
  double v = src[i0 * s0 + i1 * s1 + i2 * s2];
  TD* o = dst + i0 * t0 + i1 * t1 + i2 * t2;
  if constexpr (sizeof(TD) == 2) {
    const bf16_t hi = f2bf((float)v);
    *o = LO ? f2bf((float)(v - (double)bf2f(hi))) : hi;
  } else {
    *o = (TD)v;
  }
}

struct Copy {
  int n0, n1, n2;
  int64_t s0, s1, s2, t0, t1, t2;
};
static Copy plain(int64_t n) { return Copy{1, 1, (int)n, 0, 0, 1, 0, 0, 1}; }
// [nmat][rows][cols] -> [nmat][cols][rows]
static Copy transposed(int nmat, int rows, int cols) {
  return Copy{nmat, cols, rows, (int64_t)rows * cols, 1, cols, (int64_t)rows * cols, rows, 1};
}

static hipError_t do_copy(int tbytes, void* dst, const double* src, const Copy& c, hipStream_t s,
                          size_t lo_delta = 0) {
  int64_t tot = (int64_t)c.n0 * c.n1 * c.n2;
  if (tot <= 0) return hipSuccess;
  dim3 grid((unsigned)((tot + 255) / 256));
  if (tbytes == 8)
    hipLaunchKernelGGL((k_strided<double, false>), grid, dim3(256), 0, s, (double*)dst, src, c.n0, c.n1, c.n2, c.s0,
                       c.s1, c.s2, c.t0, c.t1, c.t2);
  else if (tbytes == 4)
    hipLaunchKernelGGL((k_strided<float, false>), grid, dim3(256), 0, s, (float*)dst, src, c.n0, c.n1, c.n2, c.s0,
                       c.s1, c.s2, c.t0, c.t1, c.t2);
  else {
    hipLaunchKernelGGL((k_strided<bf16_t, false>), grid, dim3(256), 0, s, (bf16_t*)dst, src, c.n0, c.n1, c.n2, c.s0,
                       c.s1, c.s2, c.t0, c.t1, c.t2);
    if (lo_delta)
      hipLaunchKernelGGL((k_strided<bf16_t, true>), grid, dim3(256), 0, s, (bf16_t*)((char*)dst + lo_delta), src,
                         c.n0, c.n1, c.n2, c.s0, c.s1, c.s2, c.t0, c.t1, c.t2);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// theta layout (order of the parameter vector)
// ---------------------------------------------------------------------------
static void build_theta(fire_handle* h) {
  const Dims& D = h->D;
  std::vector<std::pair<std::string, std::vector<int>>> e = {
      {"en_W1", {D.NT, 4, D.h1}}, {"en_b1", {D.NT, D.h1}}, {"en_W2", {D.h1, D.h2}}, {"en_b2", {D.h2}},
      {"en_W3", {D.h2, D.d}}, {"en_Wenv", {D.G, D.d}}, {"en_sig", {D.G}}, {"nuc_emb", {D.NT, D.d}},
      {"en_Wn", {4, D.d}}, {"ln_g", {D.d}}, {"ln_b", {D.d}}, {"glu_Wv", {D.d, D.d}}, {"glu_bv", {D.d}},
      {"glu_Wg", {D.d, D.d}}, {"glu_bg", {D.d}}, {"glu_Wo", {D.d, D.d}}, {"glu_bo", {D.d}},
      {"msg_Wa", {2, D.d, D.d}}, {"msg_Wb", {2, D.d, D.d}}, {"msg_We", {2, 4, D.d}}, {"msg_b", {2, D.d}},
      {"ee_W1", {2, 4, D.h1}}, {"ee_b1", {2, D.h1}}, {"ee_W2", {2, D.h1, D.h2}}, {"ee_b2", {2, D.h2}},
      {"ee_W3", {2, D.h2, D.d}}, {"ee_Wenv", {2, D.G, D.d}}, {"ee_sig", {2, D.G}},
      {"mlp_W", {D.L, D.d, D.d}}, {"mlp_b", {D.L, D.d}}, {"jas_cusp", {4}},
      {"orb_W_up", {D.K, D.d, D.nu}}, {"orb_W_dn", {D.K, D.d, D.nd}},
      {"env_pi_up", {D.K, D.nu, D.M, D.E}}, {"env_pi_dn", {D.K, D.nd, D.M, D.E}}, {"env_sigma", {D.M, D.E}},
  };
  if (D.Hj > 0) {
    // MLP Jastrow entries follow the cusp Jastrow (before the per-system
    // orbital block)
    size_t at = 0;
    while (at < e.size() && e[at].first != "jas_cusp") ++at;
    const int w = D.Hj;
    std::vector<std::pair<std::string, std::vector<int>>> jm = {
        {"jmlp_W1", {2, D.d, w}}, {"jmlp_b1", {2, w}}, {"jmlp_W2", {2, w, w}},
        {"jmlp_b2", {2, w}},      {"jmlp_w3", {2, w}}, {"jmlp_b3", {2}}};
    e.insert(e.begin() + (at + 1), jm.begin(), jm.end());
  }
  if (D.Ra > 0) {
    // attention Jastrow entries follow the MLP Jastrow's (or the cusp's)
    size_t at = 0;
    const char* after = D.Hj > 0 ? "jmlp_b3" : "jas_cusp";
    while (at < e.size() && e[at].first != after) ++at;
    const int w = D.Ha;
    std::vector<std::pair<std::string, std::vector<int>>> ja = {
        {"jatt_q", {D.Ra, D.d}},        {"jatt_Wv", {D.Ra, D.d, D.dr}}, {"jatt_W1", {2, D.NV(), w}},
        {"jatt_b1", {2, w}},             {"jatt_W2", {2, w, w}},         {"jatt_b2", {2, w}},
        {"jatt_w3", {2, w}},             {"jatt_b3", {2}}};
    e.insert(e.begin() + (at + 1), ja.begin(), ja.end());
  }
  int64_t off = 0;
  h->theta.clear();
  for (auto& x : e) {
    ThetaEntry t{x.first, off, x.second};
    off += t.size();
    h->theta.push_back(t);
  }
  h->P = off;
}

static const ThetaEntry& th(const fire_handle* h, const char* name) {
  for (auto& t : h->theta)
    if (t.name == name) return t;
  return h->theta[0];
}
namespace fire {
int64_t theta_offset(const fire_handle* h, const char* name) { return th(h, name).offset; }
}

static void build_layouts(fire_handle* h) {
  const Dims& D = h->D;
  size_t T = h->tsize, G = h->gsize, o = 0;
  ParamsLayout& L = h->pl;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  auto tn = [&](const char* name) { return take(th(h, name).size() * T); };
  L.en_W1 = tn("en_W1"); L.en_b1 = tn("en_b1"); L.en_W2 = tn("en_W2"); L.en_b2 = tn("en_b2");
  L.en_W3 = tn("en_W3"); L.en_Wenv = tn("en_Wenv"); L.en_sig = tn("en_sig"); L.nuc_emb = tn("nuc_emb");
  L.en_Wn = tn("en_Wn"); L.ln_g = tn("ln_g"); L.ln_b = tn("ln_b");
  L.msg_We = tn("msg_We"); L.msg_b = tn("msg_b"); L.ee_W1 = tn("ee_W1"); L.ee_b1 = tn("ee_b1");
  L.ee_W2 = tn("ee_W2"); L.ee_b2 = tn("ee_b2"); L.ee_W3 = tn("ee_W3"); L.ee_Wenv = tn("ee_Wenv");
  L.ee_sig = tn("ee_sig");
  L.b_vg = take(2 * D.d * T); L.b_o = take(D.d * T); L.mlp_b = take((size_t)D.L * D.d * T);
  L.env_sigma = tn("env_sigma");
  L.Wvg_t = take((size_t)2 * D.d * D.d * G); L.Wo_t = take((size_t)D.d * D.d * G);
  L.Wproj_t = take((size_t)4 * D.d * D.d * G); L.mlp_t = take((size_t)D.L * D.d * D.d * G);
  L.orb_t0 = take((size_t)D.K * D.nu * D.d * G); L.orb_t1 = take((size_t)D.K * D.nd * D.d * G);
  L.pi0 = take((size_t)D.K * D.nu * D.B * G); L.pi1 = take((size_t)D.K * D.nd * D.B * G);
  L.Wvg_n = take((size_t)2 * D.d * D.d * G); L.Wo_n = take((size_t)D.d * D.d * G);
  L.Wproj_n = take((size_t)4 * D.d * D.d * G); L.mlp_n = take((size_t)D.L * D.d * D.d * G);
  L.orb_n0 = take((size_t)D.K * D.nu * D.d * G); L.orb_n1 = take((size_t)D.K * D.nd * D.d * G);
  L.pi_n0 = take((size_t)D.K * D.nu * D.B * G); L.pi_n1 = take((size_t)D.K * D.nd * D.B * G);
  L.jm_W1t = take((size_t)2 * D.Hj * D.d * G); L.jm_W2t = take((size_t)2 * D.Hj * D.Hj * G);
  L.jm_W1n = take((size_t)2 * D.Hj * D.d * G); L.jm_W2n = take((size_t)2 * D.Hj * D.Hj * G);
  L.ja_Pt = take((size_t)D.NA() * D.d * G); L.ja_Pn = take((size_t)D.NA() * D.d * G);
  L.ja_W1t = take((size_t)2 * D.Ha * D.NV() * G); L.ja_W2t = take((size_t)2 * D.Ha * D.Ha * G);
  L.ja_W1n = take((size_t)2 * D.Ha * D.NV() * G); L.ja_W2n = take((size_t)2 * D.Ha * D.Ha * G);
  if (D.prec == FIRE_BF16_HYBRID) {
    const size_t region = o - L.Wvg_t;
    L.lo_delta = region;
    o += region;
    o = align_up(o);
  } else {
    L.lo_delta = 0;
  }
  L.Rn = take((size_t)D.M * 3 * 8); L.Zn = take((size_t)D.M * 8); L.ppw = take((size_t)D.M * 8);
  L.ntype = take((size_t)D.M * 4);
  L.species = take((size_t)D.M * 4);
  L.jas = take(4 * 8);
  L.jm_b1 = take((size_t)2 * D.Hj * T); L.jm_b2 = take((size_t)2 * D.Hj * T);
  L.jm_w3 = take((size_t)2 * D.Hj * T); L.jm_b3 = take(2 * T);
  L.ja_b1 = take((size_t)2 * D.Ha * T); L.ja_b2 = take((size_t)2 * D.Ha * T);
  L.ja_w3 = take((size_t)2 * D.Ha * T); L.ja_b3 = take(2 * T);
  L.total = o;

  StateRec& S = h->st;
  size_t I = h->isize;
  o = 0;
  S.h0 = take((size_t)D.n * D.d * T);
  S.proj = take((size_t)D.n * 4 * D.d * T);
  S.m = take((size_t)D.n * D.d * T);
  S.phi = take((size_t)phi_per_walker(D) * T);
  S.env = take((size_t)phi_per_walker(D) * T);
  S.inv = take((size_t)phi_per_walker(D) * I);
  S.dsign = take((size_t)2 * D.K * 8);
  S.dlog = take((size_t)2 * D.K * 8);
  S.lpsi = take(8);
  S.spsi = take(8);
  S.jas = take(8);
  S.jme = take(D.Hj > 0 ? (size_t)D.n * 2 * 8 : 0);
  S.jms = take(D.Hj > 0 ? 2 * 8 : 0);
  S.jae = take(D.Ra > 0 ? (size_t)D.n * D.NA() * T : 0);
  S.jat = take(D.Ra > 0 ? (size_t)(2 * D.Ra + D.NV() + 2) * 8 : 0);
  S.stride = o;
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* fire_status_string(fire_status s) {
  switch (s) {
    case FIRE_OK: return "ok";
    case FIRE_ERR_ARG: return "invalid argument";
    case FIRE_ERR_SHAPE: return "unsupported dimensions";
    case FIRE_ERR_PRECISION: return "unknown precision";
    case FIRE_ERR_CAPACITY: return "walker count or capacity out of range";
    case FIRE_ERR_HIP: return "HIP launch or copy failed";
    case FIRE_ERR_STATE: return "parameters not set";
  }
  return "unknown status";
}

// Largest number of pseudo-atoms whose r_max-balls share a point.  Atoms
// whose balls share a point are pairwise closer than 2 r_max, so the largest
// clique of the graph "closer than 2 r_max" bounds it (a branch-and-bound
// search; the graphs are sparse).
static int clique_max(const std::vector<std::vector<char>>& adj, const std::vector<int>& cand, int size, int best) {
  if (cand.empty()) return size > best ? size : best;
  for (size_t a = 0; a < cand.size(); ++a) {
    if (size + (int)(cand.size() - a) <= best) break;
    std::vector<int> next;
    for (size_t b = a + 1; b < cand.size(); ++b)
      if (adj[cand[a]][cand[b]]) next.push_back(cand[b]);
    best = clique_max(adj, next, size + 1, best);
  }
  return best;
}

static int ecp_atoms_bound(const fire_handle* h) {
  std::vector<int> at;
  for (int m = 0; m < h->D.M; ++m)
    for (const EcpChan& c : h->ecp)
      if (c.species == h->species[m]) { at.push_back(m); break; }
  const int na = (int)at.size();
  if (na == 0) return 0;
  const double lim = 4.0 * h->ecp_rmax * h->ecp_rmax;
  std::vector<std::vector<char>> adj(na, std::vector<char>(na, 0));
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < na; ++b) {
      const double* p = &h->Rn[3 * at[a]];
      const double* q = &h->Rn[3 * at[b]];
      const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
      adj[a][b] = a != b && dx * dx + dy * dy + dz * dz < lim;
    }
  int best = 1;
  for (int a = 0; a < na; ++a) {
    std::vector<int> nb;
    for (int b = a + 1; b < na; ++b)
      if (adj[a][b]) nb.push_back(b);
    best = clique_max(adj, nb, 1, best);
  }
  return best;
}

fire_status fire_create(const fire_system_desc* sys, const fire_model_desc* md, fire_handle** out) {
  if (!sys || !md || !out || !sys->R_nuc || !sys->Z || !sys->species || !sys->nuc_type || !sys->pp_width)
    return FIRE_ERR_ARG;
  if (md->precision < 0 || md->precision > 2) return FIRE_ERR_PRECISION;
  Dims D{};
  D.nu = sys->n_up; D.nd = sys->n_dn; D.n = D.nu + D.nd; D.M = sys->n_nuc;
  D.NT = md->n_nuc_types; D.d = md->width; D.L = md->mlp_layers; D.K = md->n_det; D.E = md->n_env;
  D.B = D.M * D.E;
  D.cut = md->cutoff; D.cutn = md->cutoff_nuc; D.cap_nbr = md->cap_nbr; D.cap_upd = md->cap_upd;
  D.prec = md->precision;
  D.split = md->precision == FIRE_BF16_HYBRID ? md->bf16_split : 0;
  D.Hj = md->jas_mlp_width;
  if (D.Hj < 0 || (D.Hj > 0 && (D.Hj % 8 != 0 || D.Hj > md->width))) return FIRE_ERR_SHAPE;
  D.Ra = md->jas_att_regs;
  D.dr = D.Ra > 0 ? md->jas_att_dim : 0;
  D.Ha = D.Ra > 0 ? md->jas_att_width : 0;
  if (D.Ra < 0 || D.Ra > 64) return FIRE_ERR_SHAPE;
  if (D.Ra > 0 && (D.dr < 1 || D.dr > 64 || D.NV() % 8 != 0 || D.NV() > 1024 || D.Ha < 8 || D.Ha > 256 ||
                   D.Ha % 8 != 0))
    return FIRE_ERR_SHAPE;
  if (D.nu < 0 || D.nd < 0 || D.n < 1 || D.nu > kMaxPerSpin || D.nd > kMaxPerSpin || D.M < 1 || D.M > 4096) return FIRE_ERR_SHAPE;
  if (D.d < 1 || D.d > 256 || D.L < 0 || D.L > 16 || D.K < 1 || D.K > 32 || D.E < 1) return FIRE_ERR_SHAPE;
  if (md->n_gauss != kMaxG || md->edge_h1 != kMaxH1 || md->edge_h2 != kMaxH2) return FIRE_ERR_SHAPE;
  if (D.NT < 1 || !(D.cut > 0) || !(D.cutn > 0)) return FIRE_ERR_SHAPE;
  if (md->max_walkers < 1 || D.cap_nbr < 1 || D.cap_nbr > 32767 || D.cap_upd < 1) return FIRE_ERR_CAPACITY;
  for (int m = 0; m < D.M; ++m)
    if (sys->nuc_type[m] < 0 || sys->nuc_type[m] >= D.NT) return FIRE_ERR_ARG;
  if (sys->n_ecp < 0 || (sys->n_ecp > 0 && !sys->ecp)) return FIRE_ERR_ARG;
  fire_handle* h = new fire_handle();
  h->D = D;
  h->model = *md;
  h->Rn.assign(sys->R_nuc, sys->R_nuc + 3 * D.M);
  h->Z.assign(sys->Z, sys->Z + D.M);
  h->ppw.assign(sys->pp_width, sys->pp_width + D.M);
  h->species.assign(sys->species, sys->species + D.M);
  h->ntype.assign(sys->nuc_type, sys->nuc_type + D.M);
  for (int k = 0; k < sys->n_ecp; ++k) {
    const fire_ecp_channel& c = sys->ecp[k];
    if (c.n_terms < 1 || c.n_terms > 4 || c.l < 0 || c.l > 1 || !c.a || !c.alpha) { delete h; return FIRE_ERR_ARG; }
    const int nq = c.n_quad == 0 ? 12 : c.n_quad;
    bool clash = nq != 4 && nq != 6 && nq != 12;
    for (const EcpChan& o : h->ecp) clash = clash || (o.species == c.species && o.nquad != nq);
    if (clash) { delete h; return FIRE_ERR_ARG; }
    EcpChan e{};
    e.species = c.species; e.l = c.l; e.nterms = c.n_terms; e.nquad = nq;
    for (int t = 0; t < c.n_terms; ++t) { e.a[t] = c.a[t]; e.alpha[t] = c.alpha[t]; }
    h->ecp.push_back(e);
  }
  h->ecp_rmax = sys->ecp_rmax;
  h->ecp_pmax = ecp_atoms_bound(h);
  h->tsize = D.prec == FIRE_FP64 ? 8 : 4;
  h->gsize = D.prec == FIRE_FP64 ? 8 : (D.prec == FIRE_FP32 ? 4 : 2);
  h->isize = D.prec == FIRE_FP32 ? 4 : 8;
  h->params = nullptr;
  h->theta_dev = nullptr;
  h->lap_budget = (size_t)48 << 30;
  build_theta(h);
  build_layouts(h);
  *out = h;
  return FIRE_OK;
}

fire_status fire_destroy(fire_handle* h) {
  if (h && h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  if (h && h->side_ecp) {
    (void)hipStreamSynchronize(h->side_ecp);
    (void)hipStreamDestroy(h->side_ecp);
  }
  if (h && h->side_ecp_join) (void)hipEventDestroy(h->side_ecp_join);
  if (h && h->side_ecp_fork) (void)hipEventDestroy(h->side_ecp_fork);
  if (h && h->side_fork) (void)hipEventDestroy(h->side_fork);
  if (h && h->side_join) (void)hipEventDestroy(h->side_join);
  delete h;
  return FIRE_OK;
}

fire_status fire_num_params(const fire_handle* h, int64_t* P) {
  if (!h || !P) return FIRE_ERR_ARG;
  *P = h->P;
  return FIRE_OK;
}

fire_status fire_param_layout(const fire_handle* h, fire_param_entry* out, int* n) {
  if (!h || !n) return FIRE_ERR_ARG;
  int cnt = (int)h->theta.size();
  if (out) {
    if (*n < cnt) return FIRE_ERR_ARG;
    for (int k = 0; k < cnt; ++k) {
      const ThetaEntry& t = h->theta[k];
      memset(&out[k], 0, sizeof(fire_param_entry));
      strncpy(out[k].name, t.name.c_str(), sizeof(out[k].name) - 1);
      out[k].offset = t.offset;
      out[k].ndim = (int)t.shape.size();
      for (size_t j = 0; j < t.shape.size() && j < 4; ++j) out[k].shape[j] = t.shape[j];
    }
  }
  *n = cnt;
  return FIRE_OK;
}

fire_status fire_sizes(const fire_handle* h, int W, size_t* params_bytes, size_t* state_bytes,
                       size_t* workspace_bytes) {
  if (!h || W < 1) return FIRE_ERR_ARG;
  if (W > h->model.max_walkers) return FIRE_ERR_CAPACITY;
  if (params_bytes) *params_bytes = h->pl.total;
  if (state_bytes) *state_bytes = h->st.stride * (size_t)W;
  if (workspace_bytes) *workspace_bytes = workspace_bytes_for(h, W);
  return FIRE_OK;
}

fire_status fire_state_layout(const fire_handle* h, size_t* offsets, size_t* stride) {
  if (!h || !offsets || !stride) return FIRE_ERR_ARG;
  const StateRec& S = h->st;
  size_t o[11] = {S.h0, S.proj, S.m, S.phi, S.env, S.inv, S.dsign, S.dlog, S.lpsi, S.spsi, S.jas};
  for (int k = 0; k < 11; ++k) offsets[k] = o[k];
  *stride = S.stride;
  return FIRE_OK;
}

}  // extern "C"

// Pack theta into params_buf.  Entries before the orbital block are read
// from `shared`, the orbital/envelope entries from `priv` (laid out as they
// follow the shared block in theta); fire_set_params passes theta and
// theta + (offset of the orbital block).
fire_status fire::set_params_split(fire_handle* h, const double* shared, const double* priv, void* params_buf,
                                   hipStream_t s) {
  if (!h || !shared || !priv || !params_buf) return FIRE_ERR_ARG;
  const Dims& D = h->D;
  char* b = (char*)params_buf;
  const ParamsLayout& L = h->pl;
  int T = (int)h->tsize, G = (int)h->gsize;
  const int64_t P0 = th(h, "orb_W_up").offset;
  auto src = [&](const char* name) {
    const int64_t o = th(h, name).offset;
    return o < P0 ? shared + o : priv + (o - P0);
  };
  auto cp = [&](size_t dst, const char* name) { return do_copy(T, b + dst, src(name), plain(th(h, name).size()), s); };
  hipError_t e = hipSuccess;
#define DO(x) do { e = (x); if (e != hipSuccess) return FIRE_ERR_HIP; } while (0)
  DO(cp(L.en_W1, "en_W1")); DO(cp(L.en_b1, "en_b1")); DO(cp(L.en_W2, "en_W2")); DO(cp(L.en_b2, "en_b2"));
  DO(cp(L.en_W3, "en_W3")); DO(cp(L.en_Wenv, "en_Wenv")); DO(cp(L.en_sig, "en_sig"));
  DO(cp(L.nuc_emb, "nuc_emb")); DO(cp(L.en_Wn, "en_Wn")); DO(cp(L.ln_g, "ln_g")); DO(cp(L.ln_b, "ln_b"));
  DO(cp(L.msg_We, "msg_We")); DO(cp(L.msg_b, "msg_b")); DO(cp(L.ee_W1, "ee_W1")); DO(cp(L.ee_b1, "ee_b1"));
  DO(cp(L.ee_W2, "ee_W2")); DO(cp(L.ee_b2, "ee_b2")); DO(cp(L.ee_W3, "ee_W3")); DO(cp(L.ee_Wenv, "ee_Wenv"));
  DO(cp(L.ee_sig, "ee_sig")); DO(cp(L.env_sigma, "env_sigma"));
  DO(do_copy(T, b + L.b_vg, src("glu_bv"), plain(D.d), s));
  DO(do_copy(T, b + L.b_vg + (size_t)D.d * T, src("glu_bg"), plain(D.d), s));
  DO(cp(L.b_o, "glu_bo")); DO(cp(L.mlp_b, "mlp_b"));
  DO(do_copy(8, b + L.jas, src("jas_cusp"), plain(4), s));
  if (D.Hj > 0) {
    const int w = D.Hj;
    const size_t LD0 = L.lo_delta;
    DO(cp(L.jm_b1, "jmlp_b1")); DO(cp(L.jm_b2, "jmlp_b2")); DO(cp(L.jm_w3, "jmlp_w3")); DO(cp(L.jm_b3, "jmlp_b3"));
    // W1t[k w + c][i] = W1[k][i][c]; W2t[k][c][i] = W2[k][i][c]
    DO(do_copy(G, b + L.jm_W1t, src("jmlp_W1"), transposed(2, D.d, w), s, LD0));
    DO(do_copy(G, b + L.jm_W2t, src("jmlp_W2"), transposed(2, w, w), s, LD0));
    // adjoint: W1n[k][i][c] = W1[k][i][c], W2n[k][i][c] = W2[k][i][c]
    DO(do_copy(G, b + L.jm_W1n, src("jmlp_W1"), plain((int64_t)2 * D.d * w), s, LD0));
    DO(do_copy(G, b + L.jm_W2n, src("jmlp_W2"), plain((int64_t)2 * w * w), s, LD0));
  }
  if (D.Ra > 0) {
    const int w = D.Ha, NA = D.NA(), NV = D.NV();
    const size_t LD0 = L.lo_delta;
    DO(cp(L.ja_b1, "jatt_b1")); DO(cp(L.ja_b2, "jatt_b2")); DO(cp(L.ja_w3, "jatt_w3")); DO(cp(L.ja_b3, "jatt_b3"));
    // Pt[r][c] = q[r][c];  Pt[Ra + r dr + e][c] = Wv[r][c][e]
    DO(do_copy(G, b + L.ja_Pt, src("jatt_q"), plain((int64_t)D.Ra * D.d), s, LD0));
    DO(do_copy(G, b + L.ja_Pt + (size_t)D.Ra * D.d * G, src("jatt_Wv"), transposed(D.Ra, D.d, D.dr), s, LD0));
    // Pn[c][r] = q[r][c];  Pn[c][Ra + r dr + e] = Wv[r][c][e]
    DO(do_copy(G, b + L.ja_Pn, src("jatt_q"), Copy{1, D.Ra, D.d, 0, D.d, 1, 0, 1, NA}, s, LD0));
    DO(do_copy(G, b + L.ja_Pn + (size_t)D.Ra * G, src("jatt_Wv"),
               Copy{D.Ra, D.d, D.dr, (int64_t)D.d * D.dr, D.dr, 1, D.dr, NA, 1}, s, LD0));
    DO(do_copy(G, b + L.ja_W1t, src("jatt_W1"), transposed(2, NV, w), s, LD0));
    DO(do_copy(G, b + L.ja_W2t, src("jatt_W2"), transposed(2, w, w), s, LD0));
    DO(do_copy(G, b + L.ja_W1n, src("jatt_W1"), plain((int64_t)2 * NV * w), s, LD0));
    DO(do_copy(G, b + L.ja_W2n, src("jatt_W2"), plain((int64_t)2 * w * w), s, LD0));
  }
  // GEMM operands Bt[N][K] (and their low bf16 parts under the hybrid precision)
  const int64_t dd = (int64_t)D.d * D.d;
  const size_t LD = L.lo_delta;
  DO(do_copy(G, b + L.Wvg_t, src("glu_Wv"), transposed(1, D.d, D.d), s, LD));
  DO(do_copy(G, b + L.Wvg_t + dd * G, src("glu_Wg"), transposed(1, D.d, D.d), s, LD));
  DO(do_copy(G, b + L.Wo_t, src("glu_Wo"), transposed(1, D.d, D.d), s, LD));
  DO(do_copy(G, b + L.Wproj_t, src("msg_Wa"), transposed(2, D.d, D.d), s, LD));
  DO(do_copy(G, b + L.Wproj_t + 2 * dd * G, src("msg_Wb"), transposed(2, D.d, D.d), s, LD));
  DO(do_copy(G, b + L.mlp_t, src("mlp_W"), transposed(D.L, D.d, D.d), s, LD));
  DO(do_copy(G, b + L.orb_t0, src("orb_W_up"), transposed(D.K, D.d, D.nu), s, LD));
  DO(do_copy(G, b + L.orb_t1, src("orb_W_dn"), transposed(D.K, D.d, D.nd), s, LD));
  DO(do_copy(G, b + L.pi0, src("env_pi_up"), plain((int64_t)D.K * D.nu * D.B), s, LD));
  DO(do_copy(G, b + L.pi1, src("env_pi_dn"), plain((int64_t)D.K * D.nd * D.B), s, LD));
  // adjoint orientation: Bt = W with the output columns of the forward GEMM as K
  // Wvg_n[k][c]: c < d -> Wv[k][c], c >= d -> Wg[k][c-d]
  DO(do_copy(G, b + L.Wvg_n, src("glu_Wv"), Copy{1, D.d, D.d, 0, D.d, 1, 0, 2 * D.d, 1}, s, LD));
  DO(do_copy(G, b + L.Wvg_n + (size_t)D.d * G, src("glu_Wg"), Copy{1, D.d, D.d, 0, D.d, 1, 0, 2 * D.d, 1}, s, LD));
  DO(do_copy(G, b + L.Wo_n, src("glu_Wo"), plain(dd), s, LD));
  // Wproj_n[k][q*d + c] = W_q[k][c] for q = (Wa0, Wa1, Wb0, Wb1)
  DO(do_copy(G, b + L.Wproj_n, src("msg_Wa"), Copy{2, D.d, D.d, dd, D.d, 1, D.d, 4 * D.d, 1}, s, LD));
  DO(do_copy(G, b + L.Wproj_n + 2 * (size_t)D.d * G, src("msg_Wb"), Copy{2, D.d, D.d, dd, D.d, 1, D.d, 4 * D.d, 1}, s, LD));
  DO(do_copy(G, b + L.mlp_n, src("mlp_W"), plain((int64_t)D.L * dd), s, LD));
  // orb_n[k][det*N + l] = orb_W[det][k][l]
  DO(do_copy(G, b + L.orb_n0, src("orb_W_up"),
             Copy{D.d, D.K, D.nu, D.nu, (int64_t)D.d * D.nu, 1, (int64_t)D.K * D.nu, D.nu, 1}, s));
  DO(do_copy(G, b + L.orb_n1, src("orb_W_dn"),
             Copy{D.d, D.K, D.nd, D.nd, (int64_t)D.d * D.nd, 1, (int64_t)D.K * D.nd, D.nd, 1}, s));
  // pi_n[b][(det,l)] = env_pi[(det,l)][b]
  DO(do_copy(G, b + L.pi_n0, src("env_pi_up"), transposed(1, D.K * D.nu, D.B), s, LD));
  DO(do_copy(G, b + L.pi_n1, src("env_pi_dn"), transposed(1, D.K * D.nd, D.B), s, LD));
  // molecule
  if (hipMemcpyAsync(b + L.Rn, h->Rn.data(), h->Rn.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b + L.Zn, h->Z.data(), h->Z.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b + L.ppw, h->ppw.data(), h->ppw.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b + L.ntype, h->ntype.data(), h->ntype.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b + L.species, h->species.data(), h->species.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return FIRE_ERR_HIP;
  // host vectors must outlive the async copies: wait for them
  if (hipStreamSynchronize(s) != hipSuccess) return FIRE_ERR_HIP;
#undef DO
  h->params = params_buf;
  h->theta_dev = shared;
  return FIRE_OK;
}

extern "C" {

fire_status fire_set_overlap(fire_handle* h, int on) {
  if (!h) return FIRE_ERR_ARG;
  if (on) {
    // the streams and events of the overlapped schedule, created once here
    // (default priority) so that compute calls never change the handle
    std::lock_guard<std::mutex> lock(fire::handle_mutex());
    bool ok = true;
    if (!h->side) ok = ok && hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) == hipSuccess;
    if (!h->side_ecp) ok = ok && hipStreamCreateWithFlags(&h->side_ecp, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t* ev : {&h->side_fork, &h->side_join, &h->side_ecp_fork, &h->side_ecp_join})
      if (!*ev) ok = ok && hipEventCreateWithFlags(ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) return FIRE_ERR_HIP;
  }
  h->overlap = on != 0;
  return FIRE_OK;
}

fire_status fire_set_ecp_chunk(fire_handle* h, int max_jobs) {
  if (!h || max_jobs < 0) return FIRE_ERR_ARG;
  h->ecp_chunk_cap = max_jobs;
  return FIRE_OK;
}

fire_status fire_set_params(fire_handle* h, const double* theta, void* params_buf, hipStream_t s) {
  if (!h || !theta || !params_buf) return FIRE_ERR_ARG;
  return fire::set_params_split(h, theta, theta + th(h, "orb_W_up").offset, params_buf, s);
}

static fire_status check_call(const fire_handle* h, int W, const void* R, const void* state, const void* ws,
                              const int32_t* status) {
  if (!h || !R || !state || !ws || !status || W < 1) return FIRE_ERR_ARG;
  if (W > h->model.max_walkers) return FIRE_ERR_CAPACITY;
  if (!h->params) return FIRE_ERR_STATE;
  return FIRE_OK;
}

fire_status fire_eval_logpsi(fire_handle* h, int W, const double* R, void* state, void* ws, double* sign,
                             double* logpsi, int32_t* status, hipStream_t s) {
  fire_status st = check_call(h, W, R, state, ws, status);
  if (st != FIRE_OK) return st;
  if (fill_i32(status, W, 0, s) != hipSuccess) return FIRE_ERR_HIP;
  hipError_t e = h->tsize == 8 ? forward<double>(h, W, R, (char*)state, (char*)ws, sign, logpsi, status, s)
                               : forward<float>(h, W, R, (char*)state, (char*)ws, sign, logpsi, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_mcmc_sweep(fire_handle* h, int W, double* R, void* state, void* ws, int n_sweeps, double step,
                            const double* noise, const double* unif, uint64_t seed, uint64_t counter,
                            int32_t* n_accept, double* logpsi, double* sign, int32_t* status, hipStream_t s) {
  fire_status st = check_call(h, W, R, state, ws, status);
  if (st != FIRE_OK) return st;
  if (n_sweeps < 0 || (!noise) != (!unif) || !n_accept || !(step >= 0)) return FIRE_ERR_ARG;
  hipError_t e = mcmc_sweep_path(h, W, R, (char*)state, (char*)ws, n_sweeps, step, 0.0, nullptr, noise, unif,
                                 nullptr, seed, counter, n_accept, logpsi, sign, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_adapt_step(double step, int64_t accepted, int64_t proposed, double target, double gain,
                            double* new_step) {
  if (!new_step || !(step > 0) || !isfinite(step) || proposed <= 0 || accepted < 0 || accepted > proposed ||
      !(target > 0 && target < 1) || !(gain >= 0) || !isfinite(gain))
    return FIRE_ERR_ARG;
  const double a = (double)accepted / (double)proposed;
  double f = exp(gain * (a - target));
  f = f < 0.5 ? 0.5 : (f > 2.0 ? 2.0 : f);
  *new_step = step * f;
  return FIRE_OK;
}

fire_status fire_mcmc_sweep_mixed(fire_handle* h, int W, double* R, void* state, void* ws, int n_sweeps,
                                  double step, double global_step, const int32_t* kinds, const double* noise,
                                  const double* unif, const double* pick, int32_t* n_accept, double* logpsi,
                                  double* sign, int32_t* status, hipStream_t s) {
  fire_status st = check_call(h, W, R, state, ws, status);
  if (st != FIRE_OK) return st;
  if (n_sweeps < 0 || !noise || !unif || !n_accept || !(step >= 0) || (n_sweeps > 0 && !kinds))
    return FIRE_ERR_ARG;
  bool any_global = false;
  for (int t = 0; t < n_sweeps; ++t) {
    if (kinds[t] != 0 && kinds[t] != 1) return FIRE_ERR_ARG;
    any_global = any_global || kinds[t] == 1;
  }
  if (any_global && (!pick || !(global_step > 0) || !isfinite(global_step))) return FIRE_ERR_ARG;
  hipError_t e = mcmc_sweep_path(h, W, R, (char*)state, (char*)ws, n_sweeps, step, global_step, kinds, noise,
                                 unif, pick, 0, 0, n_accept, logpsi, sign, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_local_energy(fire_handle* h, int W, const double* R, void* state, void* ws, const double* quad_rot,
                              double* e_loc, double* parts, double* grad_logpsi, int32_t* status, hipStream_t s) {
  fire_status st = check_call(h, W, R, state, ws, status);
  if (st != FIRE_OK) return st;
  if (!e_loc) return FIRE_ERR_ARG;
  hipError_t e = local_energy_path(h, W, R, (char*)state, (char*)ws, quad_rot, e_loc, parts, grad_logpsi, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_ecp_nonlocal(fire_handle* h, int W, const double* R, void* state, void* ws, const double* quad_rot,
                              double* v_nl, int32_t* status, hipStream_t s) {
  fire_status st = check_call(h, W, R, state, ws, status);
  if (st != FIRE_OK) return st;
  if (!v_nl) return FIRE_ERR_ARG;
  hipError_t e = ecp_path(h, W, R, (char*)state, (char*)ws, quad_rot, v_nl, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_grad_params(fire_handle* h, int W, const double* R, void* state, void* ws, const double* coeff,
                             double* grad, double* per_walker, int32_t* status, hipStream_t s) {
  fire_status st = check_call(h, W, R, state, ws, status);
  if (st != FIRE_OK) return st;
  if (!coeff || !grad) return FIRE_ERR_ARG;
  hipError_t e = grad_path(h, W, R, (char*)state, (char*)ws, coeff, grad, per_walker, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_splus_ratios(fire_handle* h, int W, const double* R, void* state, void* ws, int beta,
                              double* ratios, double* r_beta, int32_t* status, hipStream_t s) {
  fire_status st = check_call(h, W, R, state, ws, status);
  if (st != FIRE_OK) return st;
  if (!ratios || !r_beta || h->D.nu < 1 || beta < h->D.nu || beta >= h->D.n) return FIRE_ERR_ARG;
  hipError_t e = splus_path(h, W, R, (char*)state, (char*)ws, beta, ratios, r_beta, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_spring_step(fire_handle* h, int W, const double* O, const double* e_loc, double lambda, double eta,
                             const double* delta_prev, const double* delta_tilde, double lambda_pinv, double* delta,
                             void* ws, int32_t* info, hipStream_t s) {
  if (!h || !O || !e_loc || !delta || !ws || !info || W < 2) return FIRE_ERR_ARG;
  if (!(lambda > 0) || !isfinite(lambda) || !isfinite(eta)) return FIRE_ERR_ARG;
  if (delta_tilde && (!(lambda_pinv > 0) || !isfinite(lambda_pinv))) return FIRE_ERR_ARG;
  if (W > h->model.max_walkers || spring_ws_bytes(h->P, W) == 0) return FIRE_ERR_CAPACITY;
  hipError_t e = spring_step(h->P, W, O, e_loc, lambda, eta, delta_prev, delta_tilde, lambda_pinv, delta, (char*)ws,
                             info, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_profile_begin(fire_handle* h, hipStream_t stream, int32_t* counters, int capacity) {
  if (!h || !counters || capacity < 1) return FIRE_ERR_ARG;
  return profile_begin(counters, capacity, stream) == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_profile_end(fire_handle* h, hipStream_t s, int64_t* launches, double* ms, double* flops,
                             double* bytes) {
  if (!h || !launches || !ms || !flops || !bytes) return FIRE_ERR_ARG;
  return profile_end(s, launches, ms, flops, bytes) == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}

fire_status fire_sync_status(fire_handle* h, hipStream_t s, const int32_t* status, int W, int32_t* any_flags) {
  if (!h || !status || !any_flags || W < 1) return FIRE_ERR_ARG;
  std::vector<int32_t> host(W);
  if (hipMemcpyAsync(host.data(), status, (size_t)W * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return FIRE_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FIRE_ERR_HIP;
  int32_t a = 0;
  for (int k = 0; k < W; ++k) a |= host[k];
  *any_flags = a;
  return FIRE_OK;
}

}  // extern "C"
