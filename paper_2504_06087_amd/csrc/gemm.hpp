// Row-mapped GEMM with fused epilogue on MFMA (gfx950).
#pragma once
#include "common.hpp"

namespace fire {

// off(r) = (r / rpg) * gstride + (r % rpg) * rstride     (elements)
struct RowMap {
  int64_t rpg, gstride, rstride;
};
// off(c) = (c / cpg) * cgstride + (c % cpg)               (elements)
struct ColMap {
  int64_t cpg, cgstride;
};
inline RowMap rows_dense(int64_t ld) { return RowMap{1, ld, 0}; }
inline ColMap cols_dense() { return ColMap{1ll << 40, 0}; }

enum GemmAct { ACT_NONE = 0, ACT_SILU = 1 };
enum GemmKind { MMA_F64 = 0, MMA_F32 = 1, MMA_BF16 = 2, MMA_BF16X3 = 3 };

// C[r][c] = epi( sum_k A[r][k] * Bt[c][k] )
//   epi: v (+ bias[c]) -> act -> (* aux[r][c]) -> (+= C[r][c] if accumulate) -> store
// A is of element type TA (double or float), Bt of TB (double, float or bf16
// storage), C/aux/bias of TC.
struct GemmArgs {
  const void* A;
  RowMap amap;
  const void* Bt;
  int64_t ldb;        // row stride of Bt (>= K)
  const void* bias;   // [N] or nullptr
  const void* aux;    // nullptr or multiplier
  RowMap xmap;
  ColMap xcol;
  void* C;
  RowMap cmap;
  ColMap ccol;
  int M, N, K;        // M: row capacity (grid size)
  int act;
  int accumulate;
  const int* Mdev;    // optional device row count (<= M); rows beyond it are skipped
  int bias_period;    // > 0: bias only on rows r with r % bias_period == 0
  const void* Bt_lo;  // MMA_BF16X3: low bf16 part of Bt (Bt holds the high part)
  int* prof_rows;     // when set, block 0 writes the row count actually processed
  int ksplit;         // > 1: K is split into ksplit ranges; range z writes C + z * c_split_stride
  int64_t c_split_stride;
};

// Optional timing of GEMM launches (one profiler per process, host side).
struct GemmProfiler {
  bool on;
  int* counters;
  int capacity, used;
  hipStream_t stream;
  void* ev;           // std::vector of event pairs (opaque)
  int* kinds;
  int* nk;            // N*K per launch (host)
  double* bpr;        // algorithmic HBM bytes per processed row (A row, C row(s))
  double* bfix;       // algorithmic HBM bytes independent of the rows (Bt)
  int* shape;         // per launch: row capacity, N, K, tile variant (host)
};
GemmProfiler& gemm_profiler();
hipError_t profile_begin(int* counters, int capacity, hipStream_t s);
// profile_end: per-kind totals; with FIRE_GEMM_LOG set to a file path, one
// line per launch (kind, rows processed, row capacity, N, K, variant, ms,
// algorithmic bytes) is appended to that file.
hipError_t profile_end(hipStream_t s, int64_t* launches, double* ms, double* flops, double* bytes);

// Launch on stream; kind fixes the element types:
//   MMA_F64: A double, Bt double, C double
//   MMA_F32: A float,  Bt float,  C float
//   MMA_BF16: A float, Bt bf16,   C float   (A rounded to bf16 when staged)
//   MMA_BF16X3: A float, Bt bf16 hi + lo, C float: A and B are split into
//     bf16 high and low parts and C = Ah Bh + Ah Bl + Al Bh (FP32 accumulate)
hipError_t gemm(int kind, const GemmArgs& g, hipStream_t s);

// Tile autotuner (process-wide): on/off, number of tuned shapes, clear,
// save/load of the choices as text.  autotune_hold(+1 / -1) brackets work
// whose GEMMs share the chip with other streams (overlapped calls): no shape
// is timed while a hold is active, so no contended timing is kept.
void autotune_hold(int delta);
struct AutotuneHold {
  bool on;
  explicit AutotuneHold(bool o) : on(o) { if (on) autotune_hold(1); }
  ~AutotuneHold() { if (on) autotune_hold(-1); }
};
hipError_t autotune_set(int on);
int autotune_count();
void autotune_clear();
bool autotune_save(const char* path);
bool autotune_load(const char* path);

}  // namespace fire
