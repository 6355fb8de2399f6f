// A search that allocates nothing: ffa_search with its workspace in a fixed
// device array of the library instead of a caller's buffer, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops).  Each GPU holds its own copy of the array for the life of the
// process; every call on a GPU shares it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ffa_internal.h"

using namespace ffa;

namespace {

constexpr size_t kScratchMax = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// The workspace array.  In host code this name is not a device address: the
// kernels get scratch_ptr()'s address of the current GPU's copy.
static __device__ __align__(256) unsigned char scratch[kScratchMax];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of the array, looked up once per
// GPU (hipGetSymbolAddress allocates nothing).
ffa_status scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(FFA_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return FFA_OK;
}

}  // namespace

extern "C" ffa_status ffa_search_noalloc(ffa_plan p, const void* d_series, float* d_snr, int32_t* d_width,
                                         void* stream) {
  if (!p || !d_series || !d_snr || !d_width) return fail(FFA_ERR_INVALID, "null argument");
  if (p->ws_bytes > kScratchMax)
    return fail(FFA_ERR_UNSUPPORTED, "the plan's workspace (" + std::to_string(p->ws_bytes) +
                                         " B) exceeds the library's 64 MiB scratch; use ffa_search with a "
                                         "workspace, or a plan with a smaller ring_mb");
  const DeviceTables* dt = nullptr;
  ffa_status s = find_device_tables(p, &dt);
  if (s != FFA_OK) return s;
  void* ws = nullptr;
  s = scratch_ptr(&ws);
  if (s != FFA_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // nothing in the workspace needs to start at zero: every element a search
  // reads (centring sums, octave series, ring) is written by it first
  s = build_octaves(p, d_series, ws, p->n_octaves - 1, 1, st, dt);
  if (s != FFA_OK) return s;
  return run_launches(p, dt, d_snr, d_width, ws, st);
}
