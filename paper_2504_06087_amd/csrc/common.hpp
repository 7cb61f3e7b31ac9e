// Shared device helpers and the internal data layout of libfire.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "../../include/fire.h"

#define FIRE_HOST_DEVICE __host__ __device__ __forceinline__
#define FIRE_DEV __device__ __forceinline__

typedef uint16_t bf16_t;   // storage of bfloat16 values

namespace fire {

constexpr int kFcutP = 6;          // exponent p of the polynomial cutoff
constexpr double kLnEps = 1e-5;    // LayerNorm epsilon
constexpr int kMaxG = 32;          // radial Gaussians per filter
constexpr int kMaxPerSpin = 192;   // electrons per spin block (register inversion, Woodbury LDS)
constexpr int kMaxH1 = 16;         // filter hidden widths
constexpr int kMaxH2 = 8;

// ---------------------------------------------------------------------------
// Dimensions of one handle
// ---------------------------------------------------------------------------
struct Dims {
  int n, nu, nd;      // electrons
  int M;              // nuclei
  int NT;             // rows of per-nucleus tables
  int d, L, K, E;     // width, MLP layers, determinants, envelopes per nucleus
  // filter radial Gaussians and hidden widths: fixed at the widths the
  // method uses (32 Gaussians, edge MLP 16 -> 8), so every filter loop has
  // compile-time bounds
  static constexpr int G = kMaxG, h1 = kMaxH1, h2 = kMaxH2;
  int B;              // M * E envelope basis size
  double cut, cutn;   // c, c_n
  int cap_nbr, cap_upd;
  int prec;
  int split;          // GEMM sites using split bf16 operands (hybrid precision)
  int Hj;             // hidden width of the MLP Jastrow (0: off)
  int Ra, dr, Ha;     // attention Jastrow: registers (0: off), register width, readout width
  FIRE_HOST_DEVICE int NV() const { return Ra * dr; }          // register embedding width
  FIRE_HOST_DEVICE int NA() const { return Ra * (1 + dr); }    // logits + values per electron
  FIRE_HOST_DEVICE int nsig(int s) const { return s == 0 ? nu : nd; }
};

// Workgroups are dealt to the eight XCDs round-robin by index.  For a grid
// that is a multiple of 8, logical block (b % 8) * (grid / 8) + b / 8 gives
// each XCD one contiguous run of logical blocks, so consecutive blocks that
// read the same rows share that XCD's L2.
FIRE_DEV int64_t xcd_run(int64_t b, int64_t grid) { return (b & 7) * (grid >> 3) + (b >> 3); }
// The same dealing in runs of T logical blocks: XCD b % 8 takes every
// eighth run, in order, so each run (blocks that share rows) stays in one
// L2 while a live prefix of the grid (the rest exiting at once) still
// spreads over all eight XCDs.  The grid is a multiple of 8 T.
FIRE_DEV int64_t xcd_runs(unsigned b, unsigned T) {
  const unsigned i = b >> 3, q = i / T;
  return ((int64_t)(q << 3) + (b & 7)) * T + (i - q * T);
}
FIRE_HOST_DEVICE int64_t round8(int64_t n) { return (n + 7) / 8 * 8; }

// Per-walker size in elements of Phi / Phi^-1 for all determinants.
FIRE_HOST_DEVICE int64_t phi_per_det(const Dims& D) { return (int64_t)D.nu * D.nu + (int64_t)D.nd * D.nd; }
FIRE_HOST_DEVICE int64_t phi_per_walker(const Dims& D) { return (int64_t)D.K * phi_per_det(D); }
FIRE_HOST_DEVICE int64_t phi_block_off(const Dims& D, int s) { return s == 0 ? 0 : (int64_t)D.nu * D.nu; }

// ---------------------------------------------------------------------------
// Scalar functions and derivatives
// ---------------------------------------------------------------------------
template <typename T> FIRE_DEV T sigmoid_(T x) { return T(1) / (T(1) + exp(-x)); }
template <typename T> FIRE_DEV T silu_(T x) { return x * sigmoid_(x); }
// SiLU and its first two derivatives
template <typename T> FIRE_DEV void silu3(T x, T& f, T& f1, T& f2) {
  T s = sigmoid_(x);
  f = x * s;
  f1 = s * (T(1) + x * (T(1) - s));
  f2 = s * (T(1) - s) * (T(2) + x * (T(1) - T(2) * s));
}

// Cusp Jastrow pair term (Methods, global electron correlation):
// u(r) = w a^2 / (a + r) with (w, a) = q[0..1] for equal spins, q[2..3] for
// opposite spins, and its first two derivatives in r.
FIRE_DEV double jas_u(const double* q, bool same, double r) {
  const double w = same ? q[0] : q[2], a = same ? q[1] : q[3];
  return w * a * a / (a + r);
}
FIRE_DEV void jas_u3(const double* q, bool same, double r, double& u, double& u1, double& u2) {
  const double w = same ? q[0] : q[2], a = same ? q[1] : q[3];
  const double t = 1.0 / (a + r), c = w * a * a;
  u = c * t;
  u1 = -c * t * t;
  u2 = 2.0 * c * t * t * t;
}

// u(x) = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2) for x < 1, else 0
template <typename T> FIRE_DEV T fcut_(T x) {
  if (!(x < T(1))) return T(0);
  const T p = T(kFcutP);
  T xp = x * x * x;
  xp = xp * xp;                    // x^6
  return T(1) - (p + 1) * (p + 2) / 2 * xp + p * (p + 2) * xp * x - p * (p + 1) / 2 * xp * x * x;
}
// u, du/dx, d2u/dx2
template <typename T> FIRE_DEV void fcut3(T x, T& f, T& f1, T& f2) {
  if (!(x < T(1))) { f = f1 = f2 = T(0); return; }
  const T p = T(kFcutP);
  T x2 = x * x, x4 = x2 * x2, x5 = x4 * x, x6 = x4 * x2;
  f = T(1) - (p + 1) * (p + 2) / 2 * x6 + p * (p + 2) * x6 * x - p * (p + 1) / 2 * x6 * x2;
  // u' = -p(p+1)(p+2)/2 x^(p-1) (1-x)^2
  T om = T(1) - x;
  T c = p * (p + 1) * (p + 2) / 2;
  f1 = -c * x5 * om * om;
  // u'' = -c [ (p-1) x^(p-2) (1-x)^2 - 2 x^(p-1) (1-x) ]
  f2 = -c * (x4 * om * ((p - 1) * om - T(2) * x));
}

// log(1+r)/r and its derivatives w.r.t. r (limit 1, -1/2, 2/3 at r = 0)
template <typename T> FIRE_DEV void log1p_over3(T r, T& f, T& f1, T& f2) {
  if (r < T(1e-4)) {
    // series: 1 - r/2 + r^2/3 - r^3/4 + r^4/5
    f = T(1) + r * (T(-0.5) + r * (T(1) / 3 + r * (T(-0.25) + r * T(0.2))));
    f1 = T(-0.5) + r * (T(2) / 3 + r * (T(-0.75) + r * T(0.8)));
    f2 = T(2) / 3 + r * (T(-1.5) + r * T(2.4));
    return;
  }
  T L = log1p(r);
  T ir = T(1) / r;
  f = L * ir;
  T a = T(1) / (T(1) + r);
  f1 = (a - f) * ir;                         // (1/(1+r) - L/r)/r
  f2 = (-a * a - T(2) * f1) * ir;            // d/dr of f1
}
template <typename T> FIRE_DEV T log1p_over(T r) {
  if (r < T(1e-4)) return T(1) + r * (T(-0.5) + r * (T(1) / 3 + r * (T(-0.25) + r * T(0.2))));
  return log1p(r) / r;
}

// ---------------------------------------------------------------------------
// bf16 conversion (round to nearest even)
// ---------------------------------------------------------------------------
FIRE_HOST_DEVICE bf16_t f2bf(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  uint32_t u = v.u;
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  uint32_t r = 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)((u + r) >> 16);
}
FIRE_HOST_DEVICE float bf2f(bf16_t b) {
  union { float f; uint32_t u; } v;
  v.u = ((uint32_t)b) << 16;
  return v.f;
}

// ---------------------------------------------------------------------------
// Block reductions (blockDim.x a multiple of 64, <= 1024)
// ---------------------------------------------------------------------------
// two consecutive elements, read or written as one aligned access
template <typename X> struct alignas(2 * sizeof(X)) Two {
  X a, b;
};

template <typename T> FIRE_DEV T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T> FIRE_DEV T block_sum(T v, T* red) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  T t = 0;
  int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

// ---------------------------------------------------------------------------
// Network parameters on the device (pointers into the packed params buffer)
// ---------------------------------------------------------------------------
template <typename T> struct Net {
  Dims D;
  // electron-nucleus filter and embeddings
  const T *en_W1, *en_b1, *en_W2, *en_b2, *en_W3, *en_Wenv, *en_sig, *nuc_emb, *en_Wn;
  const T *ln_g, *ln_b;
  // message passing (two spin classes)
  const T *msg_We, *msg_b, *ee_W1, *ee_b1, *ee_W2, *ee_b2, *ee_W3, *ee_Wenv, *ee_sig;
  // GEMM biases
  const T *b_vg, *b_o, *mlp_b;
  // envelopes
  const T* env_sigma;
  // molecule
  const double *Rn, *Zn, *ppw;
  // cusp Jastrow (w_par, a_par, w_anti, a_anti), FP64
  const double* jas;
  const int* ntype;
  // packed GEMM weights (element type set by the precision)
  const void *Wvg_t, *Wo_t, *Wproj_t, *mlp_t, *orb_t0, *orb_t1, *pi0, *pi1;
  // the same GEMM weights in the adjoint orientation (Bt = W)
  const void *Wvg_n, *Wo_n, *Wproj_n, *mlp_n, *orb_n0, *orb_n1, *pi_n0, *pi_n1;
  // MLP Jastrow (D.Hj > 0): biases b1 [2 Hj], b2 [2 Hj], readouts w3 [2][Hj]
  // and b3 [2] in T; GEMM operands W1t [2 Hj][d] (both first layers),
  // W2t [2][Hj][Hj], and W1n [2][d][Hj], W2n [2][Hj][Hj] for the adjoint
  const T *jm_b1, *jm_b2, *jm_w3, *jm_b3;
  const void *jm_W1t, *jm_W2t, *jm_W1n, *jm_W2n;
  // attention Jastrow (D.Ra > 0): projection Pt [NA][d] (queries, then the
  // value maps r-major) and Pn [d][NA] for the adjoint; readout MLPs over V
  // as for the MLP Jastrow (input width NV, hidden Ha)
  const T *ja_b1, *ja_b2, *ja_w3, *ja_b3;
  const void *ja_Pt, *ja_Pn, *ja_W1t, *ja_W2t, *ja_W1n, *ja_W2n;
};

// ---------------------------------------------------------------------------
// Internal state and workspace layout (byte offsets)
// ---------------------------------------------------------------------------
struct StateLayout {
  // per-walker strides (bytes) and base offsets; arrays are walker-major
  size_t h0, proj, m, phi, inv, dsign, dlog, lpsi, spsi;
  size_t total;
};

}  // namespace fire
