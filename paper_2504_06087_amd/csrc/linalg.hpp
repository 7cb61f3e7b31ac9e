// Small dense FP64 linear algebra executed by one workgroup on LDS.
#pragma once
#include "common.hpp"

namespace fire {

// In-place Gauss-Jordan elimination with partial (row) pivoting of the N x N
// matrix A (leading dimension LD) held in LDS, run by every thread of the
// block.  Multipliers are formed by division by the pivot (as in LU), so two
// identical rows leave an exact zero pivot.  On return A holds A^-1 (when
// invert is set and the matrix is non-singular), sc[0] the sign and sc[1]
// log|det A|, and fl[1] = 1 when a zero or non-finite pivot was met.
// f: LDS scratch [N]; perm: LDS scratch [N]; sc: LDS [2]; fl: LDS [2].
// The block size is a multiple of 128 (all callers launch 256 threads).
FIRE_DEV void gj_block(double* A, int N, int LD, double* f, int* perm, double* sc, int* fl, bool invert) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) { sc[0] = 1.0; sc[1] = 0.0; fl[1] = 0; }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < N; i += 64) {
        double v = fabs(A[i * LD + k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        double ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) fl[0] = bi;
    }
    __syncthreads();
    const int p = fl[0];
    if (p != k)
      for (int j = tid; j < N; j += nt) {
        double t = A[k * LD + j];
        A[k * LD + j] = A[p * LD + j];
        A[p * LD + j] = t;
      }
    __syncthreads();
    const double piv = A[k * LD + k];
    if (piv == 0.0 || !isfinite(piv)) {
      if (tid == 0) fl[1] = 1;
      break;
    }
    if (tid == 0) {
      perm[k] = p;
      sc[1] += log(fabs(piv));
      sc[0] *= (piv < 0 ? -1.0 : 1.0) * (p != k ? -1.0 : 1.0);
    }
    for (int i = tid; i < N; i += nt) f[i] = (i == k) ? 0.0 : A[i * LD + k] / piv;
    __syncthreads();
    // thread t updates column c0 + t % 128 for c0 = 0, 128, ... and the
    // rows t / 128, t / 128 + nt / 128, ...: the pivot-row element stays in a
    // register and no index is divided (same update per element as a flat
    // loop, so the same result)
    const int tc = tid & 127, tr = tid >> 7, rs = nt >> 7;
    if (invert) {
      for (int j = tc; j < N; j += 128) {
        const double akj = A[k * LD + j];
        for (int i = tr; i < N; i += rs) {
          if (i == k) continue;
          if (j == k) A[i * LD + j] = -f[i];
          else A[i * LD + j] -= f[i] * akj;
        }
      }
    } else {
      // determinant only: eliminate below the pivot
      for (int j = k + 1 + tc; j < N; j += 128) {
        const double akj = A[k * LD + j];
        for (int i = k + 1 + tr; i < N; i += rs) A[i * LD + j] -= f[i] * akj;
      }
    }
    __syncthreads();
    if (invert)
      for (int j = tid; j < N; j += nt) A[k * LD + j] = (j == k) ? 1.0 / piv : A[k * LD + j] / piv;
    __syncthreads();
  }
  __syncthreads();
  if (!invert || fl[1]) return;
  for (int k = N - 1; k >= 0; --k) {
    int p = perm[k];
    if (p != k)
      for (int i = tid; i < N; i += nt) {
        double t = A[i * LD + k];
        A[i * LD + k] = A[i * LD + p];
        A[i * LD + p] = t;
      }
    __syncthreads();
  }
}

}  // namespace fire
