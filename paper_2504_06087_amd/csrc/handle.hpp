// Internal handle, packed-parameter layout, state and workspace layouts.
#pragma once
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "gemm.hpp"

namespace fire {

struct ThetaEntry {
  std::string name;
  int64_t offset;
  std::vector<int> shape;
  int64_t size() const {
    int64_t s = 1;
    for (int v : shape) s *= v;
    return s;
  }
};

struct EcpChan {
  int species, l, nterms, nquad;
  double a[4], alpha[4];
};

// Byte offsets of every packed array inside params_buf.
struct ParamsLayout {
  // small arrays in the elementwise type T
  size_t en_W1, en_b1, en_W2, en_b2, en_W3, en_Wenv, en_sig, nuc_emb, en_Wn, ln_g, ln_b;
  size_t msg_We, msg_b, ee_W1, ee_b1, ee_W2, ee_b2, ee_W3, ee_Wenv, ee_sig;
  size_t b_vg, b_o, mlp_b, env_sigma;
  // GEMM operands Bt[N][K] in the GEMM type G
  size_t Wvg_t, Wo_t, Wproj_t, mlp_t, orb_t0, orb_t1, pi0, pi1;
  // GEMM operands in the adjoint orientation (B = W^T): Bt = W, type G
  size_t Wvg_n, Wo_n, Wproj_n, mlp_n, orb_n0, orb_n1, pi_n0, pi_n1;
  // MLP Jastrow: small arrays in T, GEMM operands in G (inside the region
  // that has low bf16 parts)
  size_t jm_b1, jm_b2, jm_w3, jm_b3, jm_W1t, jm_W2t, jm_W1n, jm_W2n;
  // attention Jastrow: small arrays in T, GEMM operands in G
  size_t ja_b1, ja_b2, ja_w3, ja_b3, ja_Pt, ja_Pn, ja_W1t, ja_W2t, ja_W1n, ja_W2n;
  // low bf16 parts of every GEMM operand above live at (offset + lo_delta)
  size_t lo_delta;
  // molecule
  size_t Rn, Zn, ppw, ntype, species;
  // cusp Jastrow (w_par, a_par, w_anti, a_anti), FP64
  size_t jas;
  size_t total;
};

// Per-walker record of cached intermediates (byte offsets within a record).
struct StateRec {
  // lpsi: log|sum_d det_d| (determinants only); jas: log of the Jastrow
  // magnitude, log J_cusp + log|J_MLP|, so that log|psi| = lpsi + jas.
  // With the MLP Jastrow: jme [n][2] per-electron readouts MLP_1(h_i),
  // MLP_2(h_i) and jms [2] their sums S_1, S_2 (FP64); sign(psi) =
  // spsi * sign(S_2).  With the attention Jastrow: jae [n][NA] per-electron
  // logits h_i . q_r and values h_i W^V_r (T), and jat (FP64): the logit
  // shifts m [N_reg], the softmax sums Z [N_reg] = sum_i e^{l_ri - m_r} and
  // N [NV] = sum_i e^{l_ri - m_r} u_ri, and the readouts o [2] = MLP_1(V),
  // MLP_2(V); sign(psi) also takes sign(o_2)
  size_t h0, proj, m, phi, env, inv, dsign, dlog, lpsi, spsi, jas, jme, jms, jae, jat;
  size_t stride;
};

}  // namespace fire

struct fire_handle {
  fire::Dims D;
  fire_model_desc model;
  std::vector<double> Rn, Z, ppw;
  std::vector<int> species, ntype;
  std::vector<fire::EcpChan> ecp;
  double ecp_rmax;
  std::vector<fire::ThetaEntry> theta;
  int64_t P;
  fire::ParamsLayout pl;
  fire::StateRec st;
  size_t tsize, gsize, isize;   // bytes of T, G and the stored-inverse type
  void* params;                 // device params buffer (set by fire_set_params)
  size_t lap_budget;            // workspace bytes the Laplacian's walker chunks may use
  const double* theta_dev;      // theta passed to fire_set_params
  // most pseudo-atoms within ecp_rmax of any one point (from the geometry)
  int ecp_pmax = 0;
  int ecp_chunk_cap = 0;   // fire_set_ecp_chunk: jobs per chunk cap (0: automatic)
  // second stream of the local energy: the kinetic energy runs on it beside
  // the pseudopotential on the caller's stream (default priority), with the
  // events that order it against the caller's stream; and a third stream
  // that takes every other electron's quadrature jobs, with its fork and join
  // events.  All are created by fire_set_overlap and live until
  // fire_destroy; compute calls never create or change them.
  bool overlap = false;         // fire_set_overlap
  hipStream_t side = nullptr;
  hipEvent_t side_fork = nullptr, side_join = nullptr;
  hipStream_t side_ecp = nullptr;
  hipEvent_t side_ecp_fork = nullptr, side_ecp_join = nullptr;
};

namespace fire {

// Workspace regions for a batch of W walkers (byte offsets).
struct WsLayout {
  size_t nbr_idx, nbr_cnt, y, ug, hA, hB, basis;
  size_t jrow, jscr;   // MLP Jastrow readouts [W n][2] (FP64) and their scratch
  size_t ascr;         // attention Jastrow: registers, readouts and their scratch
  size_t total;
};
WsLayout ws_forward(const fire_handle* h, int W);


// Forward evaluation (all walkers): fills state and (sign, logpsi).
template <typename T>
hipError_t forward(const fire_handle* h, int W, const double* R, char* state, char* ws,
                   double* sign, double* logpsi, int32_t* status, hipStream_t s);

// Full re-evaluation of Phi^-1 and determinant logs from the cached Phi.
template <typename T>
hipError_t refresh_dets(const fire_handle* h, int W, const double* R, char* state, double* sign, double* logpsi,
                        int32_t* status, hipStream_t s);

inline int gemm_kind(int prec) { return prec == FIRE_FP64 ? MMA_F64 : (prec == FIRE_FP32 ? MMA_F32 : MMA_BF16); }

// GEMM call sites (bits of Dims::split)
enum GemmSite { SITE_EMB = 1, SITE_ORB = 2, SITE_JET = 4, SITE_GRAD = 8 };

// Launch a GEMM whose Bt lies in the packed params buffer, choosing the MFMA
// kind of the handle's precision for this site.
inline hipError_t gemm_site(const fire_handle* h, int site, GemmArgs g, hipStream_t s) {
  int kind = gemm_kind(h->D.prec);
  if (kind == MMA_BF16 && (h->D.split & site)) {
    kind = MMA_BF16X3;
    g.Bt_lo = (const char*)g.Bt + h->pl.lo_delta;
  }
  return gemm(kind, g, s);
}

// Guards the lazy creation of the handles' side streams and the fork of
// the local energy onto them.
std::mutex& handle_mutex();

static inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

int64_t theta_offset(const fire_handle* h, const char* name);

// Pack parameters with the shared (embedding) entries read from `shared` and
// the orbital/envelope entries from `priv`.
fire_status set_params_split(fire_handle* h, const double* shared, const double* priv, void* params_buf,
                             hipStream_t s);

}  // namespace fire
