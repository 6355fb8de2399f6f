// Search server: continuous batching of requests that arrive over time.
//
// One device arena of the HBM budget holds every admitted request's series
// copy, workspace and periodogram.  A scheduler thread admits pending
// requests in arrival order while their footprint fits what is free; when the
// head does not fit, later requests that do may pass it (backfill), up to a
// bound on how often the head is passed, after which admission waits for the
// head.  Each admitted request is enqueued on the least-loaded of the
// server's streams, where it runs next to requests admitted earlier; a device
// input is read only after the caller's stream has passed the point of
// submission.  A host callback on the stream stamps the completion.  A
// request keeps its memory until it is waited on, so clients that stop
// collecting results stop new admissions rather than exhaust memory.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ffa_internal.h"

using namespace ffa;
using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxPending = 1 << 16;
constexpr int32_t kMaxStreams = 16;
// Pending requests looked at behind a head that does not fit (bounds the
// scheduler's work per wake-up).
constexpr size_t kBackfillScan = 64;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n;
      const size_t start = it->first + n;
      free_.erase(it);
      if (rest) free_[start] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }

 private:
  std::map<size_t, size_t> free_;
};

enum class State { kPending, kRunning, kDone, kFailed, kCollecting };

struct Request {
  int64_t ticket = 0;
  ffa_plan plan = nullptr;
  std::vector<unsigned char> host;  // copy of a host series
  const void* dev_series = nullptr; // caller's device series
  hipEvent_t ready = nullptr;       // recorded on the producer stream at submit
  size_t series_bytes = 0, ws_bytes = 0, out_bytes = 0, footprint = 0;
  size_t off = 0;                   // arena offset of its block
  int stream = -1;
  int32_t passed = 0;               // later requests admitted while it was the head
  bool inject_fail = false;         // test hook: fail before enqueueing anything
  State state = State::kPending;
  ffa_status err = FFA_OK;
  Clock::time_point t_submit, t_done;
  Request() = default;
  Request(const Request&) = delete;
  Request& operator=(const Request&) = delete;
  ~Request() {
    if (ready) (void)hipEventDestroy(ready);
  }
};

}  // namespace

struct ffa_server_s {
  int device = -1;
  int32_t max_bypass = 0;
  char* base = nullptr;
  size_t budget = 0;
  std::unique_ptr<Arena> arena;
  std::vector<hipStream_t> streams;
  std::vector<int> inflight;
  hipStream_t copy_stream = nullptr;  // result copies in ffa_server_wait
  std::mutex copy_mu;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_ticket = 1;
  std::set<int64_t> fail_tickets;  // test hook (ffa_debug_server_fail)
  bool stop = false;
  std::thread sched;
};

namespace {

struct DoneCtx {
  ffa_server_s* s;
  Request* r;
};

// Runs on a HIP runtime thread once everything before it on the stream is
// done; makes no HIP call.
void on_done(void* p) {
  std::unique_ptr<DoneCtx> c(static_cast<DoneCtx*>(p));
  std::lock_guard<std::mutex> lk(c->s->mu);
  c->r->t_done = Clock::now();
  c->r->state = State::kDone;
  c->s->inflight[(size_t)c->r->stream]--;
  c->s->cv.notify_all();
}

// Enqueues one admitted request on its stream (called without the lock).
ffa_status enqueue(ffa_server_s* s, Request* r) {
  if (r->inject_fail) return fail(FFA_ERR_DEVICE, "launch failure injected by ffa_debug_server_fail");
  hipStream_t st = s->streams[(size_t)r->stream];
  char* blk = s->base + r->off;
  const void* series = r->dev_series;
  size_t o = 0;
  if (r->ready) {
    ffa_status e = check_hip(hipStreamWaitEvent(st, r->ready, 0), "wait for the producer stream");
    if (e != FFA_OK) return e;
  }
  if (!series) {
    ffa_status e = check_hip(hipMemcpyAsync(blk, r->host.data(), r->series_bytes, hipMemcpyHostToDevice, st),
                             "series upload");
    if (e != FFA_OK) return e;
    series = blk;
    o = align_up(r->series_bytes);
  }
  void* ws = blk + o;
  float* snr = reinterpret_cast<float*>(blk + o + align_up(r->ws_bytes));
  int32_t* width = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(snr) + align_up((size_t)r->plan->n_trials * 4));
  ffa_status e = ffa_search(r->plan, series, snr, width, ws, r->ws_bytes, st);
  if (e != FFA_OK) return e;
  DoneCtx* c = new (std::nothrow) DoneCtx{s, r};
  if (!c) return fail(FFA_ERR_NOMEM, "completion record");
  e = check_hip(hipLaunchHostFunc(st, on_done, c), "completion callback");
  if (e != FFA_OK) delete c;
  return e;
}

void scheduler(ffa_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    // Admit in arrival order while the head fits.  Behind a head that does
    // not, a later request that fits is admitted too (backfill) until the
    // head has been passed max_bypass times; then admission waits for it.
    std::vector<Request*> admitted;
    size_t i = 0;
    while (i < s->pending.size() && i <= kBackfillScan) {
      Request* head = s->pending.front();
      if (i > 0 && head->passed >= s->max_bypass) break;
      Request* r = s->pending[i];
      size_t off = 0;
      if (!s->arena->alloc(r->footprint, &off)) {
        ++i;
        continue;
      }
      if (i > 0) head->passed++;
      s->pending.erase(s->pending.begin() + (std::ptrdiff_t)i);
      r->inject_fail = s->fail_tickets.erase(r->ticket) > 0;
      r->off = off;
      r->stream = (int)(std::min_element(s->inflight.begin(), s->inflight.end()) - s->inflight.begin());
      s->inflight[(size_t)r->stream]++;
      r->state = State::kRunning;
      admitted.push_back(r);
    }
    if (!admitted.empty()) {
      lk.unlock();
      std::vector<ffa_status> errs;
      for (Request* r : admitted) errs.push_back(enqueue(s, r));
      lk.lock();
      for (size_t i = 0; i < admitted.size(); ++i) {
        if (errs[i] == FFA_OK) continue;
        // The work enqueued before the failing call may still run; keep the
        // block until the stream has drained past it, then report.
        Request* r = admitted[i];
        lk.unlock();
        (void)hipStreamSynchronize(s->streams[(size_t)r->stream]);
        lk.lock();
        r->err = errs[i];
        r->state = State::kFailed;
        r->t_done = Clock::now();
        s->inflight[(size_t)r->stream]--;
        s->arena->release(r->off, r->footprint);
      }
      s->cv.notify_all();
      continue;
    }
    s->cv.wait(lk);
  }
}

Request* find(ffa_server_s* s, int64_t ticket) {
  auto it = s->reqs.find(ticket);
  return it == s->reqs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" ffa_status ffa_server_create(size_t budget, int32_t n_streams, int32_t max_bypass, ffa_server* out) {
  if (!out) return fail(FFA_ERR_INVALID, "null argument");
  *out = nullptr;
  if (budget < kAlign) return fail(FFA_ERR_INVALID, "hbm_budget_bytes too small");
  if (n_streams < 1 || n_streams > kMaxStreams) return fail(FFA_ERR_INVALID, "n_streams must be in [1, 16]");
  if (max_bypass < 0) return fail(FFA_ERR_INVALID, "max_bypass must be >= 0");
  std::unique_ptr<ffa_server_s> s(new (std::nothrow) ffa_server_s());
  if (!s) return fail(FFA_ERR_NOMEM, "server allocation");
  s->max_bypass = max_bypass;
  if (hipGetDevice(&s->device) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDevice failed");
  s->budget = budget / kAlign * kAlign;
  if (hipMalloc(reinterpret_cast<void**>(&s->base), s->budget) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FFA_ERR_NOMEM, "cannot allocate the server's HBM pool");
  }
  s->arena.reset(new Arena(s->budget));
  for (int32_t j = 0; j < n_streams; ++j) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
      (void)hipFree(s->base);
      return fail(FFA_ERR_DEVICE, "cannot create the server streams");
    }
    s->streams.push_back(st);
    s->inflight.push_back(0);
  }
  if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
    (void)hipFree(s->base);
    return fail(FFA_ERR_DEVICE, "cannot create the server streams");
  }
  ffa_server_s* raw = s.get();
  try {
    s->sched = std::thread(scheduler, raw);
  } catch (...) {
    for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
    (void)hipStreamDestroy(s->copy_stream);
    (void)hipFree(s->base);
    return fail(FFA_ERR_NOMEM, "cannot start the scheduler thread");
  }
  *out = s.release();
  return FFA_OK;
}

extern "C" ffa_status ffa_server_submit(ffa_server s, ffa_plan p, const void* series, int is_device,
                                        void* producer_stream, int64_t* ticket) {
  if (!s || !p || !series || !ticket) return fail(FFA_ERR_INVALID, "null argument");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return fail(FFA_ERR_NOMEM, "request allocation");
  r->plan = p;
  const size_t elem = p->desc.dtype == FFA_IN_U8 ? 1 : 4;
  r->series_bytes = (size_t)p->desc.N * elem;
  r->ws_bytes = p->ws_bytes;
  r->out_bytes = align_up((size_t)p->n_trials * 4) * 2;
  r->footprint = (is_device ? 0 : align_up(r->series_bytes)) + align_up(r->ws_bytes) + r->out_bytes;
  if (r->footprint > s->budget) return fail(FFA_ERR_UNSUPPORTED, "request footprint exceeds the server's HBM budget");
  if (is_device) {
    r->dev_series = series;
    // The request's stream waits for this event, so the series is read only
    // after the work the caller queued before submitting has written it.
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDevice failed");
    if (cur != s->device) return fail(FFA_ERR_INVALID, "submit a device series with the server's device current");
    if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess) {
      r->ready = nullptr;
      (void)hipGetLastError();
      return fail(FFA_ERR_DEVICE, "cannot create the producer event");
    }
    ffa_status e = check_hip(hipEventRecord(r->ready, static_cast<hipStream_t>(producer_stream)),
                             "record on the producer stream");
    if (e != FFA_OK) return e;
  } else {
    try {
      r->host.resize(r->series_bytes);
    } catch (...) {
      return fail(FFA_ERR_NOMEM, "host copy of the series");
    }
    std::memcpy(r->host.data(), series, r->series_bytes);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->pending.size() >= kMaxPending) return fail(FFA_ERR_BUSY, "admission queue full");
  r->ticket = s->next_ticket++;
  r->t_submit = Clock::now();
  *ticket = r->ticket;
  s->pending.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  s->cv.notify_all();
  return FFA_OK;
}

extern "C" ffa_status ffa_server_wait(ffa_server s, int64_t ticket, int64_t timeout_us, float* host_snr,
                                      int32_t* host_width, double* latency_s) {
  if (!s) return fail(FFA_ERR_INVALID, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  Request* r = find(s, ticket);
  if (!r || r->state == State::kCollecting) return fail(FFA_ERR_INVALID, "unknown ticket");
  auto ready = [&] { return r->state == State::kDone || r->state == State::kFailed; };
  if (timeout_us < 0) {
    s->cv.wait(lk, ready);
  } else if (!s->cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return fail(FFA_ERR_TIMEOUT, "request not finished");
  }
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  if (r->state == State::kFailed) {
    const ffa_status e = r->err;
    s->reqs.erase(ticket);
    return fail(e, "the request's launch failed");
  }
  r->state = State::kCollecting;
  lk.unlock();
  // copy the periodogram out (the request's stream has passed it)
  const size_t o = (r->dev_series ? 0 : align_up(r->series_bytes)) + align_up(r->ws_bytes);
  const size_t nt = (size_t)r->plan->n_trials;
  ffa_status e = FFA_OK;
  {
    std::lock_guard<std::mutex> ck(s->copy_mu);
    if (host_snr)
      e = check_hip(hipMemcpyAsync(host_snr, s->base + r->off + o, nt * 4, hipMemcpyDeviceToHost, s->copy_stream),
                    "copy scores");
    if (e == FFA_OK && host_width)
      e = check_hip(hipMemcpyAsync(host_width, s->base + r->off + o + align_up(nt * 4), nt * 4,
                                   hipMemcpyDeviceToHost, s->copy_stream),
                    "copy widths");
    const ffa_status e2 = check_hip(hipStreamSynchronize(s->copy_stream), "result copy");
    if (e == FFA_OK) e = e2;
  }
  lk.lock();
  s->arena->release(r->off, r->footprint);
  s->reqs.erase(ticket);
  s->cv.notify_all();
  return e;
}

// Test hook: the request with this ticket (issued or still to be issued)
// fails when admitted, before anything of it is enqueued, as a launch that
// the runtime refused would; the server keeps serving the others.
extern "C" ffa_status ffa_debug_server_fail(ffa_server s, int64_t ticket) {
  if (!s || ticket <= 0) return fail(FFA_ERR_INVALID, "null server or bad ticket");
  std::lock_guard<std::mutex> lk(s->mu);
  s->fail_tickets.insert(ticket);
  return FFA_OK;
}

extern "C" ffa_status ffa_server_destroy(ffa_server s) {
  if (!s) return fail(FFA_ERR_INVALID, "null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  s->sched.join();
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  (void)hipStreamDestroy(s->copy_stream);
  (void)hipFree(s->base);
  delete s;
  return FFA_OK;
}
