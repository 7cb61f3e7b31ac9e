// Single-electron update machinery shared by Metropolis and the
// pseudopotential quadrature.
#pragma once
#include "paths.hpp"

namespace fire {

constexpr int WB_RB = 16;   // rows of G per workgroup in the Woodbury row update
constexpr int KS = 32;      // |U_s| up to which update-set rows are staged through LDS

// A batch of single-electron proposals ("jobs") for one electron index e.
// Job j moves electron e of walker jw[j] (identity when jw is null) to
// rexp[j] when rexp is set, else to r_e + step * xi[j].  Jobs at or beyond
// *Jdev (when set) are inactive.
struct Jobs {
  int J;
  int Jcap;            // workspace layout capacity (>= J); 0 means J
  const int* Jdev;
  const int* jw;
  const double* rexp;
  const double* xi;
  double step;
  bool woodbury;       // workspace laid out with the Woodbury buffers (Metropolis)
  int group;           // consecutive jobs sharing most of their update set (cache locality)
  // global single-electron jumps (Metropolis only): with pick set, r_e' is a
  // draw of the charge-weighted Gaussian mixture over the nuclei, R_m +
  // gstep * xi, and log rho(r_e) - log rho(r_e') goes to lqf[j]
  const double* pick;
  double gstep;
  const double* Rn;
  const double* Zn;
  int M;
  double* lqf;
};

struct UpdLayout {
  int capS[2], capmax;
  int64_t rowcap[2];
  size_t rnew, lqf, dj, uidx, ucnt, off, acc, detA, y, ug, h0new, projnew, basis, envnew;
  size_t rowinfo[2], hseg[2][2], mseg[2], oseg[2], dphi[2], bbuf[2];
  // MLP Jastrow (D.Hj > 0): new readouts of the update rows [rowcap[s]][2],
  // per-job new sums [J][2] and sign changes [J] (FP64), readout scratch
  size_t jnew[2], jsum, jsg, jscr;
  // attention Jastrow (D.Ra > 0): projections of the new update rows
  // [rowcap[s]][NA] (T) and the per-job sums, registers and readouts
  size_t anew[2], ja;
  size_t total;
};
// Workspace of J jobs.  Each spin segment holds J * min(capS, kRowsPerJob)
// rows; jobs whose rows would not fit are flagged FIRE_W_UPD_OVERFLOW and
// skipped.  with_woodbury adds the Metropolis-only Woodbury buffer.
constexpr int kRowsPerJob = 32;
UpdLayout upd_layout(const fire_handle* h, int J, bool with_woodbury = true);
bool update_fits(const fire_handle* h);

// Runs every step up to det A for each job: writes detA[j][det][spin] =
// (sign, log|det A|) into the workspace (UpdLayout::detA).
template <typename T>
hipError_t propose_ratio(const fire_handle* h, const Net<T>& P, const Jobs& jb, int e, const double* R,
                         char* state, char* ws, int32_t* status, hipStream_t st);

}  // namespace fire
