// Declarations shared by the kernel translation units.
#pragma once
#include "handle.hpp"

namespace fire {

hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

template <typename T>
hipError_t embed_and_orbitals(const fire_handle* h, const Net<T>& P, int W, const double* R, char* state,
                              char* ws, int32_t* status, hipStream_t s);

template <typename T> inline Net<T> make_net(const fire_handle* h) {
  Net<T> P;
  P.D = h->D;
  const char* b = (const char*)h->params;
  const ParamsLayout& L = h->pl;
  auto t = [&](size_t o) { return (const T*)(b + o); };
  P.en_W1 = t(L.en_W1); P.en_b1 = t(L.en_b1); P.en_W2 = t(L.en_W2); P.en_b2 = t(L.en_b2);
  P.en_W3 = t(L.en_W3); P.en_Wenv = t(L.en_Wenv); P.en_sig = t(L.en_sig); P.nuc_emb = t(L.nuc_emb);
  P.en_Wn = t(L.en_Wn); P.ln_g = t(L.ln_g); P.ln_b = t(L.ln_b);
  P.msg_We = t(L.msg_We); P.msg_b = t(L.msg_b); P.ee_W1 = t(L.ee_W1); P.ee_b1 = t(L.ee_b1);
  P.ee_W2 = t(L.ee_W2); P.ee_b2 = t(L.ee_b2); P.ee_W3 = t(L.ee_W3); P.ee_Wenv = t(L.ee_Wenv);
  P.ee_sig = t(L.ee_sig);
  P.b_vg = t(L.b_vg); P.b_o = t(L.b_o); P.mlp_b = t(L.mlp_b); P.env_sigma = t(L.env_sigma);
  P.Rn = (const double*)(b + L.Rn); P.Zn = (const double*)(b + L.Zn); P.ppw = (const double*)(b + L.ppw);
  P.ntype = (const int*)(b + L.ntype);
  P.jas = (const double*)(b + L.jas);
  P.Wvg_t = b + L.Wvg_t; P.Wo_t = b + L.Wo_t; P.Wproj_t = b + L.Wproj_t; P.mlp_t = b + L.mlp_t;
  P.orb_t0 = b + L.orb_t0; P.orb_t1 = b + L.orb_t1; P.pi0 = b + L.pi0; P.pi1 = b + L.pi1;
  P.Wvg_n = b + L.Wvg_n; P.Wo_n = b + L.Wo_n; P.Wproj_n = b + L.Wproj_n; P.mlp_n = b + L.mlp_n;
  P.orb_n0 = b + L.orb_n0; P.orb_n1 = b + L.orb_n1; P.pi_n0 = b + L.pi_n0; P.pi_n1 = b + L.pi_n1;
  P.jm_b1 = t(L.jm_b1); P.jm_b2 = t(L.jm_b2); P.jm_w3 = t(L.jm_w3); P.jm_b3 = t(L.jm_b3);
  P.jm_W1t = b + L.jm_W1t; P.jm_W2t = b + L.jm_W2t; P.jm_W1n = b + L.jm_W1n; P.jm_W2n = b + L.jm_W2n;
  P.ja_b1 = t(L.ja_b1); P.ja_b2 = t(L.ja_b2); P.ja_w3 = t(L.ja_w3); P.ja_b3 = t(L.ja_b3);
  P.ja_Pt = b + L.ja_Pt; P.ja_Pn = b + L.ja_Pn; P.ja_W1t = b + L.ja_W1t; P.ja_W2t = b + L.ja_W2t;
  P.ja_W1n = b + L.ja_W1n; P.ja_W2n = b + L.ja_W2n;
  return P;
}

}  // namespace fire
