// Local-energy and pseudopotential drivers.
#pragma once
#include "paths.hpp"

namespace fire {

struct LapLayout {
  int Wc;
  int64_t rowcap[2];
  size_t nidx, ncnt, joff, jtot, yj, ugj, h0j, projj, hval, zval, basisj;
  size_t jetA[2], jetB[2], envj[2], oval[2], dphi[2], gd, hd;
  int tcap;                      // capacity of the T_n member lists per spin
  size_t memb, mslot, mcnt;
  // MLP Jastrow jets (D.Hj > 0): values [2][rows][Hj], jet rows [rowcap][Hj]
  // twice per spin, readout rows [rowcap][2] (FP64), grad [Wc][n][3], Lap [Wc]
  size_t jzv, jjx[2], jjy[2], jjt[2], jgJ, jlap;
  size_t jak;   // attention Jastrow jets (scratch of ja_kinetic)
  size_t total;
};
LapLayout lap_layout(const fire_handle* h, int W);
size_t lap_ws_bytes(const fire_handle* h, int W);
size_t lap_lds_needed(const fire_handle* h);

size_t ecp_ws_bytes(const fire_handle* h, int W);
// V_NL[w] for all walkers into vnl (overwritten); ws: scratch of ecp_ws_bytes
hipError_t ecp_into(const fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                    double* vnl, int32_t* status, hipStream_t st);

}  // namespace fire
