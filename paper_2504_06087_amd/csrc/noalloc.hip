// The allocation-free variant of the evaluation entry point.  Its workspace
// is a file-scope device array (`scratch`) instead of a caller buffer, for
// callers that cannot allocate device memory (code under graph capture,
// tight serving loops).  Each GPU holds its own copy of the array, at its own
// address, from the first use of the library on it until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns
// on that device (the array's name is a host-side stand-in there).
#include <mutex>

#include "forward.hpp"

namespace fire {

constexpr size_t kScratchBytes = FIRE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace fire

extern "C" fire_status fire_eval_logpsi_noalloc(fire_handle* h, int W, const double* R, void* state, double* sign,
                                                double* logpsi, int32_t* status, hipStream_t s) {
  if (!h || !R || !state || !status || W < 1) return FIRE_ERR_ARG;
  if (W > h->model.max_walkers) return FIRE_ERR_CAPACITY;
  if (!h->params) return FIRE_ERR_STATE;
  if (fire::ws_forward(h, W).total > fire::kScratchBytes) return FIRE_ERR_CAPACITY;
  void* ws = nullptr;
  if (fire::noalloc_scratch(&ws) != hipSuccess) return FIRE_ERR_HIP;
  if (fire::fill_i32(status, W, 0, s) != hipSuccess) return FIRE_ERR_HIP;
  hipError_t e = h->tsize == 8 ? fire::forward<double>(h, W, R, (char*)state, (char*)ws, sign, logpsi, status, s)
                               : fire::forward<float>(h, W, R, (char*)state, (char*)ws, sign, logpsi, status, s);
  return e == hipSuccess ? FIRE_OK : FIRE_ERR_HIP;
}
