// Host-side drivers of the entry points beyond the forward evaluation.
#pragma once
#include "forward.hpp"

namespace fire {

size_t workspace_bytes_for(const fire_handle* h, int W);

hipError_t mcmc_sweep_path(fire_handle* h, int W, double* R, char* state, char* ws, int n_sweeps, double step,
                           const double* noise, const double* unif, int32_t* n_accept, double* logpsi,
                           double* sign, int32_t* status, hipStream_t s);
hipError_t local_energy_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                             double* e_loc, double* parts, double* grad_logpsi, int32_t* status, hipStream_t s);
hipError_t ecp_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* quad_rot,
                    double* v_nl, int32_t* status, hipStream_t s);
hipError_t grad_path(fire_handle* h, int W, const double* R, char* state, char* ws, const double* coeff,
                     double* grad, int32_t* status, hipStream_t s);

}  // namespace fire
