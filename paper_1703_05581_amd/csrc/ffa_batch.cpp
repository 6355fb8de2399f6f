// Batched search: the periodograms of many series, each with its own plan.
// The series are spread over a few library-owned HIP streams, joined to the
// caller's stream with events, so the launches of one series fill the GPU
// while another's drain.
#include <algorithm>
#include <deque>
#include <mutex>
#include <vector>

#include "ffa_internal.h"

using namespace ffa;

namespace {

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Streams and events of one device (default priority; never destroyed).
struct StreamPool {
  int device = -1;
  hipStream_t streams[kBatchStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kBatchStreams] = {};
  std::mutex mu;  // one batch enqueues on the pool at a time
};

ffa_status stream_pool(StreamPool** out) {
  static std::mutex mu;
  static std::deque<StreamPool> pools;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  for (auto& p : pools)
    if (p.device == dev) {
      *out = &p;
      return FFA_OK;
    }
  pools.emplace_back();
  StreamPool& p = pools.back();
  bool ok = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) == hipSuccess;
  for (int j = 0; ok && j < kBatchStreams; ++j)
    ok = hipStreamCreateWithFlags(&p.streams[j], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&p.join[j], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    pools.pop_back();
    return fail(FFA_ERR_DEVICE, "cannot create the batch streams");
  }
  p.device = dev;
  *out = &p;
  return FFA_OK;
}

// Batch workspace: one region per stream used, each large enough for the
// largest plan's workspace.
ffa_status batch_layout(int32_t n, const ffa_plan* plans, int32_t* regions, size_t* region_bytes) {
  if (n < 1 || !plans) return fail(FFA_ERR_INVALID, "need at least one plan");
  size_t r = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!plans[i]) return fail(FFA_ERR_INVALID, "null plan");
    r = std::max(r, plans[i]->ws_bytes);
  }
  *regions = std::min<int32_t>(n, kBatchStreams);
  *region_bytes = (size_t)round_up((int64_t)r, (int64_t)kWsAlign);
  return FFA_OK;
}

}  // namespace

extern "C" ffa_status ffa_batch_workspace(int32_t n, const ffa_plan* plans, size_t* ws_bytes) {
  if (!ws_bytes) return fail(FFA_ERR_INVALID, "null argument");
  int32_t regions = 0;
  size_t rb = 0;
  ffa_status s = batch_layout(n, plans, &regions, &rb);
  if (s != FFA_OK) return s;
  *ws_bytes = (size_t)regions * rb;
  return FFA_OK;
}

extern "C" ffa_status ffa_search_batch(int32_t n, const ffa_plan* plans, const void* const* d_series,
                                       float* const* d_snr, int32_t* const* d_width, void* d_ws,
                                       size_t ws_bytes, void* stream) {
  if (!d_series || !d_snr || !d_width || !d_ws) return fail(FFA_ERR_INVALID, "null argument");
  int32_t regions = 0;
  size_t rb = 0;
  ffa_status s = batch_layout(n, plans, &regions, &rb);
  if (s != FFA_OK) return s;
  if (ws_bytes < (size_t)regions * rb) return fail(FFA_ERR_INVALID, "workspace smaller than ffa_batch_workspace");
  if (reinterpret_cast<uintptr_t>(d_ws) % kWsAlign) return fail(FFA_ERR_INVALID, "workspace not 256-byte aligned");
  std::vector<const DeviceTables*> dts((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    if (!d_series[i] || !d_snr[i] || !d_width[i]) return fail(FFA_ERR_INVALID, "null series or output");
    s = device_tables(plans[i], &dts[(size_t)i]);
    if (s != FFA_OK) return s;
  }
  StreamPool* pool = nullptr;
  s = stream_pool(&pool);
  if (s != FFA_OK) return s;
  hipStream_t caller = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(pool->mu);
  s = check_hip(hipEventRecord(pool->fork, caller), "record fork event");
  if (s != FFA_OK) return s;
  for (int32_t j = 0; j < regions; ++j) {
    s = check_hip(hipStreamWaitEvent(pool->streams[j], pool->fork, 0), "fork wait");
    if (s != FFA_OK) return s;
  }
  // Series i runs on stream i mod regions, in region i mod regions; the
  // series of one stream run one after another, so they can share its region.
  ffa_status first_error = FFA_OK;
  for (int32_t i = 0; i < n && first_error == FFA_OK; ++i) {
    const int32_t j = i % regions;
    void* region = reinterpret_cast<char*>(d_ws) + (size_t)j * rb;
    ffa_plan p = plans[i];
    first_error = build_octaves(p, d_series[i], region, p->n_octaves - 1, 1, pool->streams[j]);
    if (first_error == FFA_OK)
      first_error = run_launches(p, dts[(size_t)i], d_snr[i], d_width[i], region, pool->streams[j]);
  }
  // join every stream, also after an error, so the caller's stream never
  // runs ahead of work already enqueued
  for (int32_t j = 0; j < regions; ++j) {
    ffa_status e = check_hip(hipEventRecord(pool->join[j], pool->streams[j]), "record join event");
    if (e == FFA_OK) e = check_hip(hipStreamWaitEvent(caller, pool->join[j], 0), "join wait");
    if (first_error == FFA_OK) first_error = e;
  }
  return first_error;
}
