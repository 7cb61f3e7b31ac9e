// Tiled MFMA GEMM for gfx950 with row-mapped operands and a fused epilogue.
//
// One 256-thread workgroup (4 wave64s in a 2x2 arrangement) computes a BM x BN
// tile of C, staging BK = 32 wide K-slices of A and Bt through LDS.  Every
// lane reads eight consecutive K elements of its A row and Bt row; bf16 uses
// one v_mfma_f32_16x16x32_bf16 per 16x16 sub-tile, f32/f64 split the eight
// elements over eight 16x16x4 MFMAs (lane group g feeds k = 8g + t to the t-th
// instruction, so the eight instructions together cover the 32-wide slice).
#include "gemm.hpp"

#include <cstdio>
#include <map>
#include <mutex>

namespace fire {

typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int BK = 32;

template <int KIND> struct MK;
template <> struct MK<MMA_F64> {
  using TA = double; using TB = double; using TC = double; using TL = double; using Acc = d4v;
  static constexpr int PAD = 2;
};
template <> struct MK<MMA_F32> {
  using TA = float; using TB = float; using TC = float; using TL = float; using Acc = f4v;
  static constexpr int PAD = 4;
};
template <> struct MK<MMA_BF16> {
  using TA = float; using TB = bf16_t; using TC = float; using TL = bf16_t; using Acc = f4v;
  static constexpr int PAD = 8;
};
template <> struct MK<MMA_BF16X3> {
  using TA = float; using TB = bf16_t; using TC = float; using TL = bf16_t; using Acc = f4v;
  static constexpr int PAD = 8;
};

// rows and columns are < 2^31: 32-bit quotients, 64-bit offsets
FIRE_DEV int64_t roff(const RowMap& m, int64_t r) {
  if (m.rpg == 1) return r * m.gstride;
  const uint32_t rr = (uint32_t)r, p = (uint32_t)m.rpg;
  const uint32_t q = rr / p;
  return (int64_t)q * m.gstride + (int64_t)(rr - q * p) * m.rstride;
}
FIRE_DEV int64_t coff(const ColMap& m, int64_t c) {
  if (m.cpg >= (int64_t)1 << 31) return c;
  const uint32_t cc = (uint32_t)c, p = (uint32_t)m.cpg;
  const uint32_t q = cc / p;
  return (int64_t)q * m.cgstride + (cc - q * p);
}

template <typename TL, typename TS> FIRE_DEV TL to_lds(TS v) { return (TL)v; }
template <> FIRE_DEV bf16_t to_lds<bf16_t, float>(float v) { return f2bf(v); }
template <> FIRE_DEV bf16_t to_lds<bf16_t, bf16_t>(bf16_t v) { return v; }

// Load 4 consecutive elements (k..k+3) of a row; zero outside [0,K) or when !valid.
template <typename TS> FIRE_DEV void load4(const TS* p, int k, int K, bool valid, bool vec, TS out[4]) {
  if (valid && vec && k + 3 < K) {
    if constexpr (sizeof(TS) == 4) {
      float4 v = *reinterpret_cast<const float4*>(p + k);
      out[0] = __builtin_bit_cast(TS, v.x); out[1] = __builtin_bit_cast(TS, v.y);
      out[2] = __builtin_bit_cast(TS, v.z); out[3] = __builtin_bit_cast(TS, v.w);
    } else if constexpr (sizeof(TS) == 8) {
      double2 a = *reinterpret_cast<const double2*>(p + k);
      double2 b = *reinterpret_cast<const double2*>(p + k + 2);
      out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
    } else {
      uint2 v = *reinterpret_cast<const uint2*>(p + k);
      out[0] = (TS)(v.x & 0xffff); out[1] = (TS)(v.x >> 16);
      out[2] = (TS)(v.y & 0xffff); out[3] = (TS)(v.y >> 16);
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) out[t] = (valid && k + t < K) ? p[k + t] : (TS)0;
  }
}

template <int KIND, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g, int vecA, int vecB) {
  using P = MK<KIND>;
  using TA = typename P::TA; using TB = typename P::TB; using TC = typename P::TC;
  using TL = typename P::TL; using Acc = typename P::Acc;
  constexpr int LDK = BK + P::PAD;
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int CA = BM * BK / 4 / 256;   // 4-element chunks per thread (A)
  constexpr int CB = BN * BK / 4 / 256;
  constexpr bool SPLIT = KIND == MMA_BF16X3;
  __shared__ __attribute__((aligned(16))) TL As[BM * LDK];
  __shared__ __attribute__((aligned(16))) TL Bs[BN * LDK];
  __shared__ __attribute__((aligned(16))) TL Asl[SPLIT ? BM * LDK : 8];
  __shared__ __attribute__((aligned(16))) TL Bsl[SPLIT ? BN * LDK : 8];

  const int tid = threadIdx.x;
  const int nct = (g.N + BN - 1) / BN;
  // split-K: blockIdx.y selects a K range and a C slice
  int kbeg = 0, kend = g.K;
  if (g.ksplit > 1) {
    const int kc = ((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK;
    kbeg = blockIdx.y * kc;
    kend = kbeg + kc < g.K ? kbeg + kc : g.K;
    g.C = (char*)g.C + (int64_t)blockIdx.y * g.c_split_stride * (int64_t)sizeof(typename P::TC);
  }
  const int Kl = kend - kbeg;
  // XCD-aware remap: consecutive logical tiles on the same XCD share A rows in L2
  const int nb = gridDim.x, per = nb / 8;
  const int bid = blockIdx.x;
  const int lid = (bid < per * 8) ? (bid % 8) * per + bid / 8 : bid;
  const int rt = lid / nct, ct = lid % nct;
  const int64_t row0 = (int64_t)rt * BM, col0 = (int64_t)ct * BN;
  if (g.Mdev) {
    int m = *g.Mdev;
    if (m < g.M) g.M = m;
  }
  if (g.prof_rows && blockIdx.x == 0 && threadIdx.x == 0) *g.prof_rows = g.M;
  if (row0 >= g.M) return;

  const TA* A = (const TA*)g.A;
  const TB* Bt = (const TB*)g.Bt;
  const TA* arow[CA];
  bool aval[CA];
  int ak[CA], ar[CA];
#pragma unroll
  for (int t = 0; t < CA; ++t) {
    int q = tid + 256 * t;
    ar[t] = q / (BK / 4);
    ak[t] = (q % (BK / 4)) * 4;
    int64_t r = row0 + ar[t];
    aval[t] = r < g.M;
    arow[t] = A + (aval[t] ? roff(g.amap, r) : 0);
  }
  const TB* brow[CB];
  const TB* browl[CB];
  bool bval[CB];
  int bk[CB], br[CB];
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    int q = tid + 256 * t;
    br[t] = q / (BK / 4);
    bk[t] = (q % (BK / 4)) * 4;
    int64_t c = col0 + br[t];
    bval[t] = c < g.N;
    brow[t] = Bt + (bval[t] ? c * g.ldb : 0);
    browl[t] = SPLIT ? (const TB*)g.Bt_lo + (bval[t] ? c * g.ldb : 0) : brow[t];
  }

  Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

  TA ra[CA][4];
  TB rb[CB][4];
  TB rbl[SPLIT ? CB : 1][4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < CA; ++t) load4<TA>(arow[t], k0 + ak[t], Kl, aval[t], vecA, ra[t]);
#pragma unroll
    for (int t = 0; t < CB; ++t) load4<TB>(brow[t], k0 + bk[t], Kl, bval[t], vecB, rb[t]);
    if constexpr (SPLIT) {
#pragma unroll
      for (int t = 0; t < CB; ++t) load4<TB>(browl[t], k0 + bk[t], Kl, bval[t], vecB, rbl[t]);
    }
  };

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lg = lane >> 4, l16 = lane & 15;

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  // loads clamp to [0, kend): shift the row pointers to kbeg
#pragma unroll
  for (int t = 0; t < CA; ++t) arow[t] += kbeg;
#pragma unroll
  for (int t = 0; t < CB; ++t) { brow[t] += kbeg; browl[t] += kbeg; }
  if (nk > 0) gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    if constexpr (sizeof(TL) == 2) {
      // 4 bf16 per 8-byte LDS store
#pragma unroll
      for (int t = 0; t < CA; ++t) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float a = (float)ra[t][e];
          const bf16_t hi = f2bf(a);
          h[e] = hi;
          if constexpr (SPLIT) l[e] = f2bf(a - bf2f(hi));
        }
        *reinterpret_cast<uint2*>(&As[ar[t] * LDK + ak[t]]) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
        if constexpr (SPLIT)
          *reinterpret_cast<uint2*>(&Asl[ar[t] * LDK + ak[t]]) = make_uint2(l[0] | (l[1] << 16), l[2] | (l[3] << 16));
      }
#pragma unroll
      for (int t = 0; t < CB; ++t) {
        *reinterpret_cast<uint2*>(&Bs[br[t] * LDK + bk[t]]) =
            make_uint2((uint32_t)rb[t][0] | ((uint32_t)rb[t][1] << 16), (uint32_t)rb[t][2] | ((uint32_t)rb[t][3] << 16));
        if constexpr (SPLIT)
          *reinterpret_cast<uint2*>(&Bsl[br[t] * LDK + bk[t]]) = make_uint2(
              (uint32_t)rbl[t][0] | ((uint32_t)rbl[t][1] << 16), (uint32_t)rbl[t][2] | ((uint32_t)rbl[t][3] << 16));
      }
    } else if constexpr (sizeof(TL) == 4) {
#pragma unroll
      for (int t = 0; t < CA; ++t)
        *reinterpret_cast<float4*>(&As[ar[t] * LDK + ak[t]]) = make_float4(ra[t][0], ra[t][1], ra[t][2], ra[t][3]);
#pragma unroll
      for (int t = 0; t < CB; ++t)
        *reinterpret_cast<float4*>(&Bs[br[t] * LDK + bk[t]]) = make_float4(rb[t][0], rb[t][1], rb[t][2], rb[t][3]);
    } else {
#pragma unroll
      for (int t = 0; t < CA; ++t) {
        *reinterpret_cast<double2*>(&As[ar[t] * LDK + ak[t]]) = make_double2(ra[t][0], ra[t][1]);
        *reinterpret_cast<double2*>(&As[ar[t] * LDK + ak[t] + 2]) = make_double2(ra[t][2], ra[t][3]);
      }
#pragma unroll
      for (int t = 0; t < CB; ++t) {
        *reinterpret_cast<double2*>(&Bs[br[t] * LDK + bk[t]]) = make_double2(rb[t][0], rb[t][1]);
        *reinterpret_cast<double2*>(&Bs[br[t] * LDK + bk[t] + 2]) = make_double2(rb[t][2], rb[t][3]);
      }
    }
    __syncthreads();
    if (kt + 1 < nk) gload((kt + 1) * BK);

    if constexpr (KIND == MMA_BF16 || KIND == MMA_BF16X3) {
      bf16x8v af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        af[i] = *reinterpret_cast<const bf16x8v*>(&As[(wm * (BM / 2) + i * 16 + l16) * LDK + 8 * lg]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bfr[j] = *reinterpret_cast<const bf16x8v*>(&Bs[(wn * (BN / 2) + j * 16 + l16) * LDK + 8 * lg]);
      if constexpr (SPLIT) {
        bf16x8v afl[TM], bfl[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          afl[i] = *reinterpret_cast<const bf16x8v*>(&Asl[(wm * (BM / 2) + i * 16 + l16) * LDK + 8 * lg]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bfl[j] = *reinterpret_cast<const bf16x8v*>(&Bsl[(wn * (BN / 2) + j * 16 + l16) * LDK + 8 * lg]);
        // small cross terms first, then the leading product
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afl[i], bfr[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfl[j], acc[i][j], 0, 0, 0);
          }
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    } else {
      TL af[TM][8], bfr[TN][8];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const TL* src = &As[(wm * (BM / 2) + i * 16 + l16) * LDK + 8 * lg];
#pragma unroll
        for (int e = 0; e < 8; ++e) af[i][e] = src[e];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const TL* src = &Bs[(wn * (BN / 2) + j * 16 + l16) * LDK + 8 * lg];
#pragma unroll
        for (int e = 0; e < 8; ++e) bfr[j][e] = src[e];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            if constexpr (KIND == MMA_F64)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][e], bfr[j][e], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][e], bfr[j][e], acc[i][j], 0, 0, 0);
          }
    }
    __syncthreads();
  }

  // epilogue: each lane holds column l16 of a 16x16 sub-tile; register e is
  // row 4*lg + e for the f32-accumulating MFMAs and row 4*e + lg for the f64 one
  // (measured lane layouts of v_mfma_f32_16x16x{4f32,32_bf16} and
  // v_mfma_f64_16x16x4f64 on gfx950)
  const TC* bias = (const TC*)g.bias;
  const TC* aux = (const TC*)g.aux;
  TC* C = (TC*)g.C;
  int64_t rco[TM][4], rxo[TM][4];
  bool rok[TM][4], rbias[TM][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t r = row0 + wm * (BM / 2) + i * 16 + (KIND == MMA_F64 ? 4 * e + lg : 4 * lg + e);
      rok[i][e] = r < g.M;
      rco[i][e] = rok[i][e] ? roff(g.cmap, r) : 0;
      rxo[i][e] = (rok[i][e] && aux) ? roff(g.xmap, r) : 0;
      rbias[i][e] = !(g.bias_period > 0 && (uint32_t)r % (uint32_t)g.bias_period);
    }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    int64_t c = col0 + wn * (BN / 2) + j * 16 + l16;
    if (c >= g.N) continue;
    TC bc = bias ? bias[c] : TC(0);
    int64_t cco = coff(g.ccol, c);
    int64_t xco = aux ? coff(g.xcol, c) : 0;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (!rok[i][e]) continue;
        TC v = (TC)acc[i][j][e] + (rbias[i][e] ? bc : TC(0));
        if (g.act == ACT_SILU) v = silu_(v);
        if (aux) v *= aux[rxo[i][e] + xco];
        TC* dst = C + rco[i][e] + cco;
        if (g.accumulate) v += *dst;
        *dst = v;
      }
  }
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

GemmProfiler& gemm_profiler() {
  static GemmProfiler p{};
  return p;
}

// ---------------------------------------------------------------------------
// Tile shapes and the autotuner.  Variant v of the f32/bf16 kinds is a BM x BN
// tile with (BM, BN) = (128,128), (128,64), (64,128), (64,64); f64 has one
// 64 x 64 variant.  Every variant sums K in the same order (32-wide slices,
// one MFMA chain per 16 x 16 sub-tile), so all produce bit-identical C.
// While tuning is on, the first launch of each new shape (kind, log2 M, N, K,
// split) on a stream that is not capturing times every variant on the real
// operands and keeps the fastest; GEMMs that accumulate into C are not timed
// (running them twice would add twice) and keep variant 0.
constexpr int kVariants = 4;
static const int kTileM[kVariants] = {128, 128, 64, 64};
static const int kTileN[kVariants] = {128, 64, 128, 64};

struct TuneKey {
  int kind, lgm, n, k, split;
  bool operator<(const TuneKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (lgm != o.lgm) return lgm < o.lgm;
    if (n != o.n) return n < o.n;
    if (k != o.k) return k < o.k;
    return split < o.split;
  }
};
struct Tuner {
  std::mutex mu;
  std::map<TuneKey, int> choice;
  bool on = false;
};
static Tuner& tuner() {
  static Tuner t;
  return t;
}
static TuneKey key_of(int kind, const GemmArgs& g) {
  int lg = 0;
  while ((1ll << lg) < (int64_t)g.M) ++lg;
  return TuneKey{kind, lg, g.N, g.K, g.ksplit > 1 ? g.ksplit : 1};
}

template <int KIND, int BM, int BN> static hipError_t launch_tile(const GemmArgs& g, hipStream_t s, int vecA,
                                                                  int vecB) {
  const int64_t tiles = (int64_t)((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<KIND, BM, BN>), dim3((unsigned)tiles, g.ksplit > 1 ? g.ksplit : 1), dim3(256), 0, s,
                     g, vecA, vecB);
  return hipGetLastError();
}

template <int KIND> static hipError_t launch_variant(int v, const GemmArgs& g, hipStream_t s, int vecA, int vecB) {
  if constexpr (KIND == MMA_F64) {
    return launch_tile<KIND, 64, 64>(g, s, vecA, vecB);
  } else {
    switch (v) {
      case 1: return launch_tile<KIND, 128, 64>(g, s, vecA, vecB);
      case 2: return launch_tile<KIND, 64, 128>(g, s, vecA, vecB);
      case 3: return launch_tile<KIND, 64, 64>(g, s, vecA, vecB);
      default: return launch_tile<KIND, 128, 128>(g, s, vecA, vecB);
    }
  }
}

// time every variant of this shape once (after one warm-up launch each)
template <int KIND> static int tune_shape(const GemmArgs& g, hipStream_t s, int vecA, int vecB) {
  const int nv = KIND == MMA_F64 ? 1 : kVariants;
  if (nv == 1) return 0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 0;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return 0; }
  int best = 0;
  float best_ms = 0.f;
  for (int v = 0; v < nv; ++v) {
    if (launch_variant<KIND>(v, g, s, vecA, vecB) != hipSuccess) continue;
    (void)hipEventRecord(e0, s);
    if (launch_variant<KIND>(v, g, s, vecA, vecB) != hipSuccess) continue;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (v == 0 || ms < best_ms) { best = v; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

template <int KIND> static int pick_variant(const GemmArgs& g, hipStream_t s, int vecA, int vecB) {
  if (KIND == MMA_F64) return 0;
  Tuner& t = tuner();
  const TuneKey key = key_of(KIND, g);
  {
    std::lock_guard<std::mutex> lk(t.mu);
    auto it = t.choice.find(key);
    if (it != t.choice.end()) return it->second;
    if (!t.on || g.accumulate || g.prof_rows) return 0;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return 0;
  const int v = tune_shape<KIND>(g, s, vecA, vecB);
  std::lock_guard<std::mutex> lk(t.mu);
  t.choice[key] = v;
  return v;
}

template <int KIND> static hipError_t launch(GemmArgs g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  int vecA = aligned16(g.A) && g.K % 4 == 0 && g.amap.gstride % 4 == 0 && (g.amap.rpg == 1 || g.amap.rstride % 4 == 0);
  int vecB = aligned16(g.Bt) && g.K % 4 == 0 && g.ldb % 4 == 0 &&
             (KIND != MMA_BF16X3 || aligned16(g.Bt_lo));
  if (g.ksplit > 1) vecA = vecA && ((((g.K + g.ksplit - 1) / g.ksplit + BK - 1) / BK * BK) % 4 == 0);
  GemmProfiler& pr = gemm_profiler();
  const bool prof = pr.on && s == pr.stream && pr.used < pr.capacity;
  const int v = pick_variant<KIND>(g, s, vecA, vecB);
  hipEvent_t* evs = prof ? (hipEvent_t*)pr.ev : nullptr;
  int slot = 0;
  if (prof) {
    slot = pr.used++;
    g.prof_rows = pr.counters + slot;
    pr.kinds[slot] = KIND;
    pr.nk[slot] = g.N * g.K;
    (void)hipEventRecord(evs[2 * slot], s);
  }
  hipError_t e = launch_variant<KIND>(v, g, s, vecA, vecB);
  if (prof) (void)hipEventRecord(evs[2 * slot + 1], s);
  return e;
}

hipError_t autotune_set(int on) {
  Tuner& t = tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  t.on = on != 0;
  return hipSuccess;
}

int autotune_count() {
  Tuner& t = tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  return (int)t.choice.size();
}

void autotune_clear() {
  Tuner& t = tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  t.choice.clear();
}

// one line per shape: kind log2M N K split variant
bool autotune_save(const char* path) {
  Tuner& t = tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  FILE* f = fopen(path, "w");
  if (!f) return false;
  fprintf(f, "# kind log2M N K split variant(0:128x128 1:128x64 2:64x128 3:64x64)\n");
  for (auto& kv : t.choice)
    fprintf(f, "%d %d %d %d %d %d\n", kv.first.kind, kv.first.lgm, kv.first.n, kv.first.k, kv.first.split,
            kv.second);
  return fclose(f) == 0;
}

bool autotune_load(const char* path) {
  Tuner& t = tuner();
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[256];
  std::map<TuneKey, int> m;
  bool ok = true;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    TuneKey k{};
    int v = 0;
    if (sscanf(line, "%d %d %d %d %d %d", &k.kind, &k.lgm, &k.n, &k.k, &k.split, &v) != 6 || v < 0 ||
        v >= kVariants || k.kind < 0 || k.kind > 3) {
      ok = false;
      break;
    }
    m[k] = k.kind == MMA_F64 ? 0 : v;
  }
  fclose(f);
  if (!ok) return false;
  std::lock_guard<std::mutex> lk(t.mu);
  for (auto& kv : m) t.choice[kv.first] = kv.second;
  return true;
}

hipError_t profile_begin(int* counters, int capacity, hipStream_t s) {
  GemmProfiler& pr = gemm_profiler();
  if (pr.ev) {
    hipEvent_t* e = (hipEvent_t*)pr.ev;
    for (int k = 0; k < 2 * pr.capacity; ++k) (void)hipEventDestroy(e[k]);
    delete[] e;
    delete[] pr.kinds;
    delete[] pr.nk;
  }
  pr.ev = nullptr;
  pr.capacity = capacity;
  pr.counters = counters;
  pr.used = 0;
  pr.stream = s;
  hipEvent_t* e = new hipEvent_t[2 * (size_t)capacity];
  for (int k = 0; k < 2 * capacity; ++k)
    if (hipEventCreate(&e[k]) != hipSuccess) return hipErrorOutOfMemory;
  pr.ev = e;
  pr.kinds = new int[capacity];
  pr.nk = new int[capacity];
  pr.on = true;
  return hipSuccess;
}

hipError_t profile_end(hipStream_t s, int64_t* launches, double* ms, double* flops) {
  GemmProfiler& pr = gemm_profiler();
  pr.on = false;
  for (int k = 0; k < 4; ++k) { launches[k] = 0; ms[k] = 0; flops[k] = 0; }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  int* rows = new int[pr.used > 0 ? pr.used : 1];
  if (pr.used > 0) e = hipMemcpy(rows, pr.counters, (size_t)pr.used * 4, hipMemcpyDeviceToHost);
  hipEvent_t* ev = (hipEvent_t*)pr.ev;
  for (int k = 0; k < pr.used && e == hipSuccess; ++k) {
    float t = 0;
    (void)hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]);
    const int kd = pr.kinds[k];
    launches[kd] += 1;
    ms[kd] += t;
    flops[kd] += 2.0 * (double)rows[k] * (double)pr.nk[k];
  }
  delete[] rows;
  return e;
}

hipError_t gemm(int kind, const GemmArgs& g, hipStream_t s) {
  switch (kind) {
    case MMA_F64: return launch<MMA_F64>(g, s);
    case MMA_F32: return launch<MMA_F32>(g, s);
    case MMA_BF16: return launch<MMA_BF16>(g, s);
    case MMA_BF16X3: return launch<MMA_BF16X3>(g, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace fire
