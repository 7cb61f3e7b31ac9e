/*
 * libfire -- the finite-range-embedding (FiRE) neural-network VMC hot path on
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Scherbela, Gao, Grohs, Guennemann, "Accurate Ab-initio Neural-network
 * Solutions to Large-Scale Electronic Structure Problems" (arXiv 2504.06087),
 * Methods section: wave-function ansatz (eq. wf), low-rank wave-function
 * updates, efficient Laplacian (eqs. forward_lap_jac, forward_lap_lap,
 * forward_lap_det_M, logdet_lowrank), variational Monte Carlo (Hamiltonian,
 * local energy, energy gradient) and the effective core potential.
 *
 * Conventions of every entry point
 *  - All tensor pointers are DEVICE pointers owned by the caller unless a
 *    comment says "host".  All work is enqueued on the caller's hipStream_t
 *    and no call allocates device memory.  No compute call synchronises the
 *    stream or reads a device value back to the host, so every compute call
 *    can be captured into a HIP graph.  (The pseudopotential quadrature sizes
 *    its launches from a bound on its job counts fixed by the geometry and
 *    reads the live counts on the device.)
 *  - Positions are FP64 [W][n][3], electrons 0..n_up-1 spin up, the rest down.
 *  - Errors the host can see (bad pointer, shape, precision, W > max_walkers)
 *    are returned immediately as a negative fire_status and nothing is
 *    enqueued.  Each call clears the caller's int32 status[W] and ORs into it
 *    the conditions it finds on the device (FIRE_W_*); a flagged walker's
 *    outputs are NaN and its sign 0.  Nothing is ever silently truncated.
 *  - state/workspace/params buffers are sized by fire_sizes and owned by the
 *    caller.  state must hold the result of fire_eval_logpsi (or of a sweep)
 *    for the same positions before local_energy, ecp_nonlocal or grad_params.
 *  - Calls on different streams with different state/workspace buffers may
 *    overlap; calls sharing a workspace must be ordered by the caller.
 */
#ifndef FIRE_H
#define FIRE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fire_status;
#define FIRE_OK 0
#define FIRE_ERR_ARG -1         /* null pointer or bad size */
#define FIRE_ERR_SHAPE -2       /* dimensions outside what the kernels support */
#define FIRE_ERR_PRECISION -3   /* unknown precision mode */
#define FIRE_ERR_CAPACITY -4    /* W > max_walkers or a capacity below its minimum */
#define FIRE_ERR_HIP -5         /* a HIP launch or copy failed */
#define FIRE_ERR_STATE -6       /* parameters not set */

/* per-walker device status bits */
#define FIRE_W_NBR_OVERFLOW 1   /* more neighbours within c than cap_nbr */
#define FIRE_W_UPD_OVERFLOW 2   /* update set larger than cap_upd */
#define FIRE_W_SINGULAR 4       /* zero pivot in an orbital matrix or in A */
#define FIRE_W_NONFINITE 8      /* a non-finite position or result */
#define FIRE_W_DETSUM_ZERO 16   /* the determinants cancel exactly: psi = 0 */

typedef enum {
  FIRE_FP64 = 0,        /* every stage in FP64 */
  FIRE_FP32 = 1,        /* FP32 everywhere (FP32 MFMA GEMMs, FP32 LU and inverse) */
  FIRE_BF16_HYBRID = 2  /* BF16 GEMM operands with FP32 accumulation, FP32
                           elementwise, FP64 LU / log-det / running inverse */
} fire_precision;

/* One semilocal pseudopotential channel v_l(r) = sum_k a_k exp(-alpha_k r^2)
 * (Methods, effective core potential).  Host arrays. */
typedef struct {
  int species;
  int l;               /* 0 or 1 */
  int n_terms;         /* <= 4 */
  const double* a;     /* host [n_terms] */
  const double* alpha; /* host [n_terms] */
  int n_quad;          /* angular quadrature points of this species (SI,
                          effective core potential, N_quad per species):
                          4 tetrahedron, 6 octahedron, 12 icosahedron, 0 = 12;
                          every channel of one species gives the same value */
} fire_ecp_channel;

/* The molecule (Methods, Hamiltonian eq. hamiltonian).  Host arrays, copied. */
typedef struct {
  int n_nuc;
  const double* R_nuc;     /* host [n_nuc][3] bohr */
  const double* Z;         /* host [n_nuc]; effective charge for pseudo-atoms */
  const int* species;      /* host [n_nuc] element id (selects ECP channels) */
  const int* nuc_type;     /* host [n_nuc] row of per-nucleus parameter tables */
  const double* pp_width;  /* host [n_nuc]; 0: -Z/r, w > 0: -Z erf(r/w)/r */
  int n_up, n_dn;
  int n_ecp;               /* number of channels (0: all-electron) */
  const fire_ecp_channel* ecp;
  double ecp_rmax;         /* quadrature applied iff |r_i - R_I| < ecp_rmax */
} fire_system_desc;

/* The ansatz (Methods, wave-function ansatz) and run limits. */
typedef struct {
  int width;          /* embedding width d */
  int mlp_layers;     /* L */
  int n_det;          /* K */
  int n_env;          /* envelopes per nucleus */
  int n_gauss;        /* radial Gaussians in the filters (32) */
  int edge_h1, edge_h2; /* filter MLP widths (16, 8) */
  int n_nuc_types;    /* rows of the per-nucleus tables */
  double cutoff;      /* c, electron-electron */
  double cutoff_nuc;  /* c_n, electron-nucleus */
  int precision;      /* fire_precision */
  int max_walkers;    /* W limit of every call on this handle */
  int cap_nbr;        /* max |N_i| per electron (both spin classes) */
  int cap_upd;        /* max |U| of a single-electron update */
  int refresh_every;  /* sweeps between full FP64 re-evaluations */
  int bf16_split;     /* FIRE_BF16_HYBRID only: GEMM sites whose operands are
                         split into bf16 high + low parts (three MFMA products,
                         FP32 accumulation): bit 0 embedding/MLP rows, bit 1
                         orbital/envelope rows, bit 2 Laplacian tangent rows */
  int jas_mlp_width;  /* per-electron MLP Jastrow (Methods, global electron
                         correlation): J_MLP = exp(sum_i MLP_1(h_i)) *
                         sum_i MLP_2(h_i) over the final embeddings h_i, each
                         MLP two SiLU hidden layers of this width and a scalar
                         linear readout; the factor multiplies the cusp factor.
                         0: off; else a multiple of 8, at most width.  Adds the
                         theta entries jmlp_W1 [2][d][w], jmlp_b1 [2][w],
                         jmlp_W2 [2][w][w], jmlp_b2 [2][w], jmlp_w3 [2][w],
                         jmlp_b3 [2] after jas_cusp (index 0: MLP_1, 1: MLP_2).
                         sum_i MLP_2(h_i) = 0 makes psi = 0 (FIRE_W_DETSUM_ZERO). */
  int jas_att_regs;   /* attention-register Jastrow (Methods, global electron
                         correlation): N_reg registers; for register r the
                         softmax over the electrons of h_i . q_r weights the
                         values h_i W^V_r (d_reg wide), V = Concat_r v_r, and
                         J_att = exp(MLP_1(V)) MLP_2(V), each readout MLP two
                         SiLU hidden layers of jas_att_width and a scalar
                         linear readout.  0: off; else <= 64.  Adds theta
                         entries jatt_q [N_reg][d], jatt_Wv [N_reg][d][d_reg],
                         jatt_W1 [2][N_reg d_reg][w], jatt_b1 [2][w],
                         jatt_W2 [2][w][w], jatt_b2 [2][w], jatt_w3 [2][w],
                         jatt_b3 [2] after the MLP Jastrow's.  MLP_2(V) = 0
                         makes psi = 0 (FIRE_W_DETSUM_ZERO). */
  int jas_att_dim;    /* d_reg (<= 64; N_reg d_reg a multiple of 8, <= 1024) */
  int jas_att_width;  /* readout width w: a multiple of 8, 8..256 */
} fire_model_desc;

typedef struct fire_handle fire_handle;

typedef struct {
  char name[32];
  int64_t offset;     /* element offset into theta */
  int32_t ndim;
  int32_t shape[4];
} fire_param_entry;

/* Create/destroy a handle.  Copies the host arrays.  Returns FIRE_ERR_SHAPE
 * outside the dimensions the kernels support (width <= 256, n_up, n_dn <=
 * 192, n_gauss == 32, edge MLP widths exactly 16 and 8, K <= 32, L <= 16). */
fire_status fire_create(const fire_system_desc* sys, const fire_model_desc* model, fire_handle** out);
fire_status fire_destroy(fire_handle* h);

/* The FP64 parameter vector theta: names, offsets and shapes, in order.  *n
 * holds the capacity of out on entry and the entry count on return (out may
 * be NULL to query the count). */
fire_status fire_param_layout(const fire_handle* h, fire_param_entry* out, int* n);
fire_status fire_num_params(const fire_handle* h, int64_t* P);

/* Bytes of the caller-owned buffers for W walkers. */
fire_status fire_sizes(const fire_handle* h, int W, size_t* params_bytes, size_t* state_bytes,
                       size_t* workspace_bytes);

/* Byte offsets, within one walker's record of the state buffer, of the
 * cached intermediates: offsets[0..10] = h0 [n][d], projections [n][4][d]
 * (a_par, a_anti, b_par, b_anti), messages m [n][d], Phi [K][(n_up^2 +
 * n_dn^2)] (per determinant the up block then the down block, row i =
 * electron, column l = orbital), envelopes (same shape as Phi), G = Phi^-T
 * (same shape: G[k][l] = (Phi^-1)[l][k], the derivative of log|det| by
 * Phi[k][l]), determinant signs [K][2] and log|det| [K][2] (FP64),
 * log|sum_d det_d| and its sign (FP64), and the log of the cusp Jastrow
 * factor (FP64; log|psi| is the sum of the last two logs).  Arrays
 * other than the FP64 ones use the precision's elementwise type (FP64 for
 * FIRE_FP64, FP32 otherwise; Phi^-1 is FP64 except under FIRE_FP32).
 * *stride is the record size; walker w's record starts at w * stride. */
fire_status fire_state_layout(const fire_handle* h, size_t* offsets, size_t* stride);

/* Pack theta (device FP64 [P]) and the molecule into params_buf in the
 * layouts and precisions the kernels use.  params_buf must stay alive and
 * unchanged for every later call on this handle. */
fire_status fire_set_params(fire_handle* h, const double* theta, void* params_buf, hipStream_t stream);

/* Stream overlap inside fire_local_energy (off by default).  With on != 0 the
 * kinetic energy (Methods, forward Laplacian) runs on a second stream of the
 * handle beside the nonlocal pseudopotential, whose electrons alternate
 * between the caller's stream and a third one; both fork from and join the
 * caller's stream within the call.  Results equal the serial schedule up to
 * the order in which the two pseudopotential lane sums are added.  The first
 * call with on != 0 creates the streams (default priority) and their events,
 * which live until fire_destroy; compute calls never create or change them.
 * Overlapped kernels share the chip, so per-kernel timings under it are not
 * standalone rates, and the GEMM autotuner does not time shapes inside an
 * overlapped call.  Errors: FIRE_ERR_ARG for a null handle, FIRE_ERR_HIP when
 * a stream or event cannot be created. */
fire_status fire_set_overlap(fire_handle* h, int on);

/* Upper bound on the quadrature jobs per chunk of the nonlocal
 * pseudopotential (Methods, pseudopotentials: each electron's quadrature
 * points go through the low-rank ratio in chunks).  0 (the default) lets
 * the library choose: equal chunks covering an electron's job bound, at most
 * 24 GiB of update segments per chunk.  A positive max_jobs lowers that cap
 * (rounded down to a multiple of 12, at least 12), which shrinks the
 * workspace fire_sizes reports; call fire_sizes after this.  Results do not
 * depend on the chunking (each walker's quadrature terms are summed in one
 * fixed order).  Errors: FIRE_ERR_ARG for a null handle or max_jobs < 0. */
fire_status fire_set_ecp_chunk(fire_handle* h, int max_jobs);

/* log|psi| and its sign for W walkers (Methods, eq. wf with the cusp
 * Jastrow factor as J: psi = exp(J_cusp) sum_d det Phi_d^up det Phi_d^down,
 * J_cusp = sum_{i<j} w a^2/(a + r_ij) with theta entry jas_cusp = (w_par,
 * a_par, w_anti, a_anti); J_cusp = 0 for zero weights), and the cached
 * intermediates the update, Laplacian and adjoint paths reuse (embeddings
 * h0, projections, messages, Phi, Phi^-1, per-determinant sign and log|det|,
 * log J_cusp) written to state.  R: [W][n][3]; sign, logpsi: [W];
 * status: [W]. */
fire_status fire_eval_logpsi(fire_handle* h, int W, const double* R, void* state, void* ws,
                             double* sign, double* logpsi, int32_t* status, hipStream_t stream);

/* fire_eval_logpsi without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same computation, kernels and outputs as
 * fire_eval_logpsi, with its workspace taken from a file-scope device array
 * of FIRE_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The caller still owns R, state, sign, logpsi and
 * status.  The call allocates nothing.  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (different streams, or
 * threads) race and must be ordered by the caller.  Errors: as
 * fire_eval_logpsi; FIRE_ERR_CAPACITY when the evaluation of W walkers needs
 * more than FIRE_NOALLOC_SCRATCH_BYTES of workspace (about 1.25 MB per walker
 * at 180 electrons, width 256 and 432 envelope functions in the BF16 hybrid:
 * up to 53 walkers; 4 electrons at width 32: over 10 000); FIRE_ERR_HIP when
 * the array's device address cannot be looked up. */
#define FIRE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fire_status fire_eval_logpsi_noalloc(fire_handle* h, int W, const double* R, void* state, double* sign,
                                     double* logpsi, int32_t* status, hipStream_t stream);

/* n_sweeps systematic-scan Metropolis sweeps with Gaussian single-electron
 * moves r_e' = r_e + step*xi (Methods, improved Monte Carlo sampling), each
 * proposal evaluated by neighbour recompute and the matrix-determinant lemma
 * (Methods, low-rank wave-function updates), accepted iff u < (psi'/psi)^2;
 * accepted moves update Phi^-1 by the Woodbury identity.  State is refreshed
 * by a full evaluation every refresh_every sweeps.  Random numbers: explicit
 * noise [S][n][W][3] (xi) and unif [S][n][W] (u), or both NULL: then sweep t
 * draws them on the device from the counter-based generator Philox4x32-10
 * (Salmon et al., SC'11) with key seed and counter (w, e + 2^16 b, lo32(c),
 * hi32(c)), c = counter + t, b = 0, 1, 2 (three blocks per proposal; 53-bit
 * uniforms from pairs of words, xi by Box-Muller from blocks 0 and 1, u from
 * block 2); a caller advances counter by n_sweeps between calls.  seed and
 * counter are ignored with explicit numbers.  R is updated in place;
 * n_accept [W] is incremented; logpsi/sign [W] receive the final values.
 * FIRE_ERR_ARG when exactly one of noise and unif is NULL. */
fire_status fire_mcmc_sweep(fire_handle* h, int W, double* R, void* state, void* ws, int n_sweeps,
                            double step, const double* noise, const double* unif, uint64_t seed,
                            uint64_t counter, int32_t* n_accept, double* logpsi, double* sign,
                            int32_t* status, hipStream_t stream);

/* Sweeps that mix the local moves of fire_mcmc_sweep with global
 * single-electron jumps (SI, improved Monte Carlo sampling: the
 * charge-weighted Gaussian-mixture proposal over the nuclei and its
 * acceptance factor).  kinds: host int32 [n_sweeps], 0 = a sweep of local
 * moves r_e' = r_e + step*xi, 1 = a sweep of global jumps: component m is the
 * first nucleus whose cumulative charge fraction sum_{m'<=m} Z_m'/sum Z
 * exceeds pick[t][e][w], r_e' = R_m + global_step*xi, accepted iff
 * u < (psi'/psi)^2 rho(r_e)/rho(r_e') with rho(r) = sum_m Z_m
 * N(r | R_m, global_step^2 I)/sum Z (Z: the effective charges of the system
 * description).  pick: device FP64 [S][n][W] uniforms in [0,1), may be NULL
 * when no sweep is global; global_step > 0 then.  Every other argument,
 * the update machinery and the refresh are those of fire_mcmc_sweep.
 * FIRE_ERR_ARG for a kind other than 0/1 or a missing pick/scale. */
/* Step-size adaptation of the local moves (Methods, improved Monte Carlo
 * sampling: the proposal scale is adjusted on the fly towards a target
 * acceptance ratio; 50 % in the paper's hyperparameters).  With the
 * acceptance ratio a = accepted / proposed of the last sweeps,
 * *new_step = step * exp(gain * (a - target)), limited to [step/2, 2 step]:
 * a fixed point at a = target, larger steps when too many moves are
 * accepted.  Host arithmetic only (no device work); FIRE_ERR_ARG for a
 * non-positive step, proposed <= 0, accepted outside [0, proposed], a
 * target outside (0, 1) or a negative gain. */
fire_status fire_adapt_step(double step, int64_t accepted, int64_t proposed, double target, double gain,
                            double* new_step);

fire_status fire_mcmc_sweep_mixed(fire_handle* h, int W, double* R, void* state, void* ws, int n_sweeps,
                                  double step, double global_step, const int32_t* kinds,
                                  const double* noise, const double* unif, const double* pick,
                                  int32_t* n_accept, double* logpsi, double* sign, int32_t* status,
                                  hipStream_t stream);

/* Local energy E_L = -1/2 (Lap log|psi| + |grad log|psi||^2) + V_ee + V_en +
 * V_nn + V_NL (Methods, local energy and Hamiltonian) by the sparse forward
 * Laplacian (Methods, efficient Laplacian).  quad_rot [W][3][3] rotates the
 * pseudopotential quadrature (NULL: identity).  parts [W][5] (kinetic, V_ee,
 * V_en, V_nn, V_NL) and grad_logpsi [W][n][3] are optional (NULL). */
fire_status fire_local_energy(fire_handle* h, int W, const double* R, void* state, void* ws,
                              const double* quad_rot, double* e_loc, double* parts,
                              double* grad_logpsi, int32_t* status, hipStream_t stream);

/* Nonlocal pseudopotential energy per walker (Methods, effective core
 * potential): for every electron within ecp_rmax of a pseudo-atom, an
 * equal-weight angular quadrature of psi ratios from single-electron low-rank
 * updates, with the pseudo-atom species' n_quad points (4 tetrahedron, 6
 * octahedron, 12 icosahedron), rotated by quad_rot[w] ([W][3][3], NULL:
 * identity). */
fire_status fire_ecp_nonlocal(fire_handle* h, int W, const double* R, void* state, void* ws,
                              const double* quad_rot, double* v_nl, int32_t* status,
                              hipStream_t stream);

/* grad[P] = sum_w coeff[w] d log|psi_w| / d theta (Methods, energy gradient
 * with coeff_w = (E_L,w - mean E_L)/W), by a hand-written adjoint with
 * per-layer recomputation.  grad is overwritten.  per_walker (optional,
 * device FP64 [W][P], NULL to skip): row w receives d log|psi_w| / d theta,
 * the per-walker gradients the natural-gradient step needs (Methods,
 * variational Monte Carlo, eq. spring); grad is then the coeff-weighted sum of
 * the rows.  The per-walker mode runs the adjoint one walker at a time. */
fire_status fire_grad_params(fire_handle* h, int W, const double* R, void* state, void* ws,
                             const double* coeff, double* grad, double* per_walker, int32_t* status,
                             hipStream_t stream);

/* Two-electron swap ratios of the S+ spin penalty (SI, low-rank updates in
 * S+ operator): for the spin-down electron beta (n_up <= beta < n) and every
 * spin-up electron a, ratios[w][a] = psi(pi_{a,beta} r_w) / psi(r_w), the
 * wave function with the positions of a and beta exchanged over the cached
 * one, and r_beta[w] = 1 - sum_a ratios[w][a], the per-walker estimator R_beta
 * whose square gives <S+ psi|S+ psi> = n_down/(n_up + 1) E[R_beta^2].  Each
 * ratio is one low-rank update: the embeddings of the two positions keep
 * their nuclear part, the pairs of a third electron with either position
 * change class, and the determinants change in the rows of {a, beta} and the
 * electrons within c of either position (a rank-|U| update per spin block
 * through the matrix-determinant lemma).  ratios: device [W][n_up]; r_beta:
 * [W].  state must hold the evaluation at R.  Errors: FIRE_ERR_ARG for null
 * pointers, no spin-up electron or beta outside the spin-down range. */
fire_status fire_splus_ratios(fire_handle* h, int W, const double* R, void* state, void* ws, int beta,
                              double* ratios, double* r_beta, int32_t* status, hipStream_t stream);

/* One natural-gradient parameter update (Methods, variational Monte Carlo,
 * eq. spring, with momentum; SI, non-hermitian operator gradients in
 * Spring, eq. aux_spring):
 *   delta = Obar^T (Obar Obar^T + lambda I)^-1 (eps + eps~ - eta Obar delta_prev)
 *           + eta delta_prev + (delta_tilde - Obar^T eps~)
 * with Obar the per-walker gradients O (device FP64 [W][P], row w =
 * d log|psi_w| / d theta, e.g. from fire_grad_params' per_walker) centred over
 * the walkers, eps = e_loc (device [W]) centred, and, when delta_tilde
 * (device [P], a gradient not of the form Obar^T v) is given, eps~ = (Obar
 * Obar^T + lambda_pinv I)^-1 Obar delta_tilde, the damped pseudo-inverse that
 * splits delta_tilde into its part in the span of the rows of Obar (added to
 * eps) and the rest (added to delta).  delta_prev (device [P]) may be NULL
 * (zero).  The W x W Gram matrix is one FP64 MFMA GEMM over the parameters;
 * the damped systems are solved by a blocked FP64 Cholesky factorisation.
 * ws: the handle's workspace (fire_sizes covers it).  info (device int32):
 * 0, or 1 when a damped Gram matrix was not positive definite.  Errors:
 * FIRE_ERR_ARG for null pointers, W < 2, lambda <= 0 or (with delta_tilde)
 * lambda_pinv <= 0; FIRE_ERR_CAPACITY for W above max_walkers or 8192. */
fire_status fire_spring_step(fire_handle* h, int W, const double* O, const double* e_loc, double lambda,
                             double eta, const double* delta_prev, const double* delta_tilde,
                             double lambda_pinv, double* delta, void* ws, int32_t* info, hipStream_t stream);

/* Kernel timing for roofline reports.  Between fire_profile_begin and
 * fire_profile_end every MFMA GEMM launched on `stream` by this handle is
 * bracketed by HIP events, and its actual row count is written (by the
 * kernel) into counters (device, int32 [capacity]).  fire_profile_end
 * synchronises the stream and returns, per GEMM kind (0 f64, 1 f32, 2 bf16,
 * 3 split bf16), the launch count, summed kernel time (ms), algorithmic
 * flops 2*M*N*K and algorithmic HBM bytes (M rows of A read and of C written,
 * C also read when accumulating, the multiplier rows read, Bt read once;
 * host arrays of 4).  Launches beyond capacity are not timed.
 * Both calls also enqueue one empty kernel (k_profile_mark) on the stream, so
 * that a kernel trace or counter run can cut out exactly the profiled work. */
fire_status fire_profile_begin(fire_handle* h, hipStream_t stream, int32_t* counters, int capacity);
fire_status fire_profile_end(fire_handle* h, hipStream_t stream, int64_t* launches, double* ms, double* flops,
                             double* bytes);

/* ---------------------------------------------------------------------------
 * Uneven multi-system batches.  n_systems molecules with different electron
 * counts share one model: every theta entry before the orbital block
 * (filters, per-species nuclear tables -- nuc_type must index species --,
 * LayerNorm/GLU, messages, MLP) is shared, the orbital weights and envelope
 * parameters (orb_W_up .. env_sigma) are per system (Methods, wave function
 * ansatz: the embedding network does not depend on the molecule).  The batch
 * theta is [shared | private of system 0 | private of system 1 | ...];
 * system s's private block starts at the offset fire_batch_system returns.
 * Per-system caps are min(cap_nbr, n_s - 1) and min(cap_upd, n_s); the
 * model's max_walkers bounds every W[s].  At most 32 systems.
 *
 * Buffers are concatenations in system order: R [sum_s W_s n_s 3], noise
 * [sum_s S n_s W_s 3] (system s's block is its [S][n_s][W_s][3] array),
 * unif [sum_s S n_s W_s], n_accept / e_loc / status [sum_s W_s].
 */
typedef struct fire_batch fire_batch;
typedef struct fire_graph fire_graph;

fire_status fire_batch_create(const fire_system_desc* systems, int n_systems, const fire_model_desc* model,
                              fire_batch** out);
fire_status fire_batch_destroy(fire_batch* b);
/* *P_total: batch theta length; *P_shared (may be NULL): shared entries. */
fire_status fire_batch_num_params(const fire_batch* b, int64_t* P_total, int64_t* P_shared);
/* System s's handle (owned by the batch; usable with every single-system
 * call once fire_batch_set_params has run) and its private-block offset. */
fire_status fire_batch_system(const fire_batch* b, int s, fire_handle** h, int64_t* priv_offset);
/* Bytes of the caller-owned batch buffers; W: host [n_systems]. */
fire_status fire_batch_sizes(const fire_batch* b, const int* W, int n_sweeps, size_t* params_bytes,
                             size_t* state_bytes, size_t* workspace_bytes);
/* Pack the batch theta (device FP64 [P_total]) into params_buf. */
fire_status fire_batch_set_params(fire_batch* b, const double* theta, void* params_buf, hipStream_t stream);
/* One step for every system: full evaluation; n_sweeps Metropolis sweeps
 * (noise/unif as fire_mcmc_sweep; n_accept incremented); local energy;
 * c_w = (E_L,w - mean_s E_L)/W_s over the finite E_L of each system (Methods,
 * energy gradient; flagged walkers get c_w = 0); grad [P_total] = the
 * per-system sums of c_w d log|psi_w|/d theta, the shared entries summed over
 * systems.  status collects every condition of the step.  The systems run on
 * up to four internal streams forked from and joined back to `stream`. */
fire_status fire_batch_step(fire_batch* b, const int* W, double* R, void* state, void* ws, int n_sweeps,
                            double step, const double* noise, const double* unif, int32_t* n_accept,
                            double* e_loc, double* grad, int32_t* status, hipStream_t stream);
/* Capture fire_batch_step with these exact arguments into HIP graphs, one
 * per internal stream branch (the buffers are bound into them: a replay reads
 * their contents at launch time).  The graph object refers to the batch's
 * streams and is valid while the batch lives. */
fire_status fire_batch_graph_create(fire_batch* b, const int* W, double* R, void* state, void* ws, int n_sweeps,
                                    double step, const double* noise, const double* unif, int32_t* n_accept,
                                    double* e_loc, double* grad, int32_t* status, fire_graph** out);
/* Replay the whole captured step with one call: the branch graphs run on the
 * batch's streams, forked from and joined back to `stream`, then the gradient
 * combine runs on `stream`.  Replays of one batch must not overlap. */
fire_status fire_graph_launch(fire_graph* g, hipStream_t stream);
fire_status fire_graph_destroy(fire_graph* g);

/* GEMM tile autotuner (process-wide).  While on, the first launch of every
 * new GEMM shape (kind, ceil log2 of the row capacity, N, K, K-split) on a
 * stream that is not capturing times each tile shape (128x128, 128x64,
 * 64x128, 64x64; one warm-up and one timed launch each, synchronising the
 * stream) and keeps the fastest; later launches of that shape use it, also
 * inside captured graphs.  Every tile shape sums K in the same order, so the
 * choice never changes results.  GEMMs that accumulate into their output,
 * and GEMMs whose live row count is a device value (the row capacity says
 * little about the rows live at the first launch), are not timed and use
 * 128x128.  A shape also records whether its rows are device-counted and
 * whether its output rows are dense.  save/load write/read the choices as
 * text, one line per shape: kind log2M N K split form variant. */
fire_status fire_autotune(int on);
fire_status fire_autotune_count(int* n_shapes);
fire_status fire_autotune_clear(void);
fire_status fire_autotune_save(const char* path);
fire_status fire_autotune_load(const char* path);

/* OR of status[0..W-1] into *any_flags (host); synchronises the stream. */
fire_status fire_sync_status(fire_handle* h, hipStream_t stream, const int32_t* status, int W,
                             int32_t* any_flags);

const char* fire_status_string(fire_status s);

#ifdef __cplusplus
}
#endif
#endif /* FIRE_H */
