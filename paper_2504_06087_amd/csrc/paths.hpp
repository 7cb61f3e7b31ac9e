// Host-side drivers of the entry points beyond the forward evaluation.
#pragma once
#include "forward.hpp"

namespace fire {

size_t workspace_bytes_for(const fire_handle* h, int W);

// kinds (host [n_sweeps], NULL: all local): 1 marks a sweep of global jumps,
// which read pick [S][n][W] and the scale gstep
// noise == NULL: each sweep draws its numbers from the counter-based
// generator (key seed, counter base counter + sweep index)
hipError_t mcmc_sweep_path(fire_handle* h, int W, double* R, char* state, char* ws, int n_sweeps, double step,
                           double gstep, const int32_t* kinds, const double* noise, const double* unif,
                           const double* pick, uint64_t seed, uint64_t counter, int32_t* n_accept, double* logpsi,
                           double* sign, int32_t* status, hipStream_t s);
size_t rng_ws_offset(const fire_handle* h, int W);
// two-electron swap ratios of the S+ estimator (update.hip)
size_t swap_ws_bytes(const fire_handle* h, int W);
hipError_t splus_path(fire_handle* h, int W, const double* R, char* state, char* ws, int eb, double* ratios,
                      double* rb, int32_t* status, hipStream_t s);
// the natural-gradient step (spring.hip); 0 bytes when W exceeds its limit
size_t spring_ws_bytes(int64_t P, int W);
hipError_t spring_step(int64_t P, int W, const double* O, const double* e_loc, double lambda, double eta,
                       const double* dprev, const double* dtilde, double lambda0, double* delta, char* ws,
                       int32_t* info, hipStream_t st);
size_t rng_ws_bytes(const fire_handle* h, int W);
hipError_t local_energy_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                             double* e_loc, double* parts, double* grad_logpsi, int32_t* status, hipStream_t s);
hipError_t ecp_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                    double* v_nl, int32_t* status, hipStream_t s);
// per_walker (optional, [W][P]): d log|psi_w| / d theta per walker
hipError_t grad_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* coeff,
                     double* grad, double* per_walker, int32_t* status, hipStream_t s);

}  // namespace fire
