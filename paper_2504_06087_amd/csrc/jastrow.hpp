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

// Scratch bytes of jm_rows for M rows.
size_t jm_rows_ws(const fire_handle* h, int64_t M);

// Readouts out[r] = (MLP_1(X_r), MLP_2(X_r)) in FP64 for rows X [M][d]
// (dense, row stride d) of the embedding; rows at or beyond *Mdev (when set)
// are skipped.  scratch: jm_rows_ws bytes.
template <typename T>
hipError_t jm_rows(const fire_handle* h, const Net<T>& P, const T* X, int M, const int* Mdev, char* scratch,
                   double* out, hipStream_t s);

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

}  // namespace fire
