// Per-electron MLP Jastrow factor (Methods, global electron correlation):
//   J_MLP = exp(S_1) S_2,  S_k = sum_i MLP_k(h_i),
//   MLP_k(h) = w3_k . SiLU(SiLU(h W1_k + b1_k) W2_k + b2_k) + b3_k,
// over the final embeddings h_i.  log|J_MLP| = S_1 + log|S_2| joins the
// Jastrow log magnitude cached in the state; sign(S_2) multiplies the sign
// of psi.  Because each readout depends on h_i alone, a single-electron
// update changes S_k by the readouts of the update-set rows only (Methods,
// low-rank wave-function updates: the Jastrow is updated like the orbitals).
#pragma once
#include "forward.hpp"

namespace fire {

// A pair of readout MLPs (index 0: log part, 1: node part) over rows of
// width `in`, hidden width H: operands as packed in the params buffer.
template <typename T> struct Readout {
  const void *W1t, *W2t, *W1n, *W2n;
  const T *b1, *b2, *w3, *b3;
  int in, H;
};
template <typename T> inline Readout<T> jm_readout(const fire_handle* h, const Net<T>& P) {
  return Readout<T>{P.jm_W1t, P.jm_W2t, P.jm_W1n, P.jm_W2n, P.jm_b1, P.jm_b2, P.jm_w3, P.jm_b3, h->D.d, h->D.Hj};
}
template <typename T> inline Readout<T> ja_readout(const fire_handle* h, const Net<T>& P) {
  return Readout<T>{P.ja_W1t, P.ja_W2t, P.ja_W1n, P.ja_W2n, P.ja_b1, P.ja_b2, P.ja_w3, P.ja_b3, h->D.NV(), h->D.Ha};
}

// Scratch bytes of readout_rows for M rows of hidden width H.
size_t readout_ws(const fire_handle* h, int64_t M, int H);
inline size_t jm_rows_ws(const fire_handle* h, int64_t M) { return h->D.Hj > 0 ? readout_ws(h, M, h->D.Hj) : 0; }

// out[r] = (MLP_1(X_r), MLP_2(X_r)) in FP64 for rows X [M][in] (dense);
// rows at or beyond *Mdev (when set) are skipped.
template <typename T>
hipError_t readout_rows(const fire_handle* h, const Readout<T>& Q, const T* X, int M, const int* Mdev,
                        char* scratch, double* out, hipStream_t s);
template <typename T>
inline hipError_t jm_rows(const fire_handle* h, const Net<T>& P, const T* X, int M, const int* Mdev, char* scratch,
                          double* out, hipStream_t s) {
  return readout_rows<T>(h, jm_readout<T>(h, P), X, M, Mdev, scratch, out, s);
}

// Evaluation: readouts rows [W n][2] into the state (jme) and their sums
// S_1, S_2 in electron order (jms).
hipError_t jm_store(const fire_handle* h, int W, const double* rows, char* state, hipStream_t s);

// After the cusp factor is in the state's Jastrow log: add S_1 + log|S_2|;
// S_2 = 0 (or non-finite) flags the walker FIRE_W_DETSUM_ZERO.
hipError_t jm_total(const fire_handle* h, int W, char* state, int32_t* status, hipStream_t s);

// Per job of a batch of single-electron updates (rows of job j in segment s:
// off[s (J+1) + j] .. + ucnt[2 j + s], electrons uidx[(2 j + s) capmax + t]):
// the new sums S_k' = S_k + sum over the rows (new - cached readout); adds
// S_1' - S_1 + log|S_2'| - log|S_2| to dj[j], writes the sign change
// sign(S_2' S_2) to jsg[j] and (S_1', S_2') to jsum[j].
hipError_t jm_delta(const fire_handle* h, int J, const int* jw, const int* uidx, int capmax, const int* ucnt,
                    const int* off, const double* jnew0, const double* jnew1, const char* state, double* dj,
                    double* jsg, double* jsum, hipStream_t s);

// Accepted Metropolis moves (acc[w] != 0): the update rows' readouts and the
// new sums into the state.
hipError_t jm_commit(const fire_handle* h, int W, const int* acc, const int* uidx, int capmax, const int* ucnt,
                     const int* off, const double* jnew0, const double* jnew1, const double* jsum, char* state,
                     hipStream_t s);

// Kinetic-energy terms of log|J_MLP| for walkers [w0, w0 + Wc) from the jets
// of the final embeddings (values hval [Wc n][d], jet rows jin[s] laid out by
// joff / ncnt as in the Laplacian): gJ [Wc][n][3] = grad log|J_MLP| and
// lapJ [Wc] = Lap log|J_MLP|.  S_2 comes from the state.  Scratch buffers:
// zv [2][Wc n][Hj] (T), jx[s], jy[s] [rowcap[s]][Hj] (T), jt[s]
// [rowcap[s]][2] (FP64).
struct JmJetArgs {
  int Wc, w0;
  int64_t rowcap[2];
  const int32_t* ncnt;
  const int* joff;
  const int* jtot;
  const int* memb;
  const int* mslot;
  const int* mcnt;
  int tcap;
  const void* hval;
  const void* jin[2];
  void* zv;
  void* jx[2];
  void* jy[2];
  double* jt[2];
  double* gJ;
  double* lapJ;
};
template <typename T>
hipError_t jm_kinetic(const fire_handle* h, const Net<T>& P, const JmJetArgs& a, const char* state,
                      hipStream_t s);

// ---------------------------------------------------------------------------
// attention-register Jastrow (Methods, global electron correlation):
//   l_ri = h_i . q_r,  u_ri = h_i W^V_r,  v_r = sum_i softmax_i(l_r) u_ri,
//   J_att = exp(MLP_1(V)) MLP_2(V),  V = Concat_r v_r.
// The state keeps per electron (l_i, u_i) and per walker the shifted sums
// Z_r = sum_i e^{l_ri - m_r}, N_r = sum_i e^{l_ri - m_r} u_ri with the shift
// m_r = max_i l_ri of the last full evaluation, so a single-electron update
// changes Z and N by the update rows only (O(|U|) per register, Methods,
// low-rank wave-function updates); V = N / Z and the readouts are O(1) in n.
// ---------------------------------------------------------------------------
// Evaluation: projections of the final embeddings X [W n][d] into the state,
// the sums, the register embeddings and the readouts.  ws: ja_eval_ws bytes.
size_t ja_eval_ws(const fire_handle* h, int W);
template <typename T>
hipError_t ja_eval(const fire_handle* h, const Net<T>& P, int W, const T* X, char* state, char* ws, hipStream_t s);

// After the cusp factor is in the state's Jastrow log: add o_1 + log|o_2|;
// o_2 = 0 flags FIRE_W_DETSUM_ZERO.
hipError_t ja_total(const fire_handle* h, int W, char* state, int32_t* status, hipStream_t s);

// Updates: anew[s] [rowcap[s]][NA] are the projections of the new update
// rows (computed by the caller's GEMM); per job the new sums, registers and
// readouts, the change of log|J_att| added to dj[j] and the sign change
// multiplied into jsg[j] (set when `first`).  ws: ja_update_ws bytes for J
// jobs: new sums [J][N_reg + NV] (FP64), registers [J][NV] (T), readouts
// [J][2] (FP64), scratch.
size_t ja_update_ws(const fire_handle* h, int J);
template <typename T>
hipError_t ja_delta(const fire_handle* h, const Net<T>& P, int J, const int* jw, const int* Jdev, const int* uidx,
                    int capmax, const int* ucnt, const int* off, const T* anew0, const T* anew1, const char* state,
                    char* ws, double* dj, double* jsg, bool first, hipStream_t s);
template <typename T>
hipError_t ja_commit(const fire_handle* h, int W, const int* acc, const int* uidx, int capmax, const int* ucnt,
                     const int* off, const T* anew0, const T* anew1, const char* ws, char* state, hipStream_t s);

// Kinetic-energy terms of log|J_att| added to gJ [Wc][n][3] and lapJ [Wc]
// (written when `first`): the jets of the projections (jet rows of h_i times
// Pt), dense tangents of Z and N per walker gathered over the member lists,
// the jets of V = N / Z, and the readout MLPs' jets over the 3n + 2 rows of
// each walker (value, tangents, Laplacian).  Scratch: ja_kin_ws bytes.
size_t ja_kin_ws(const fire_handle* h, int Wc, const int64_t rowcap[2]);
template <typename T>
hipError_t ja_kinetic(const fire_handle* h, const Net<T>& P, const JmJetArgs& a, const char* state, char* ws,
                      bool first, hipStream_t s);

}  // namespace fire
