// Batched search: the periodograms of many series, each with its own plan,
// as one work queue.
//
// Every step of every series goes into one step list (series by series, each
// in its plan's step order).  The list is cut into window groups like one
// plan's (about window_tiles tiles each, within one shared intermediate
// ring), so a launch holds the tiles of many series at once: small series no
// longer run launches of a few thousand tiles, and the launch tails of one
// series fill with another's tiles.  Plans that fold in different arithmetic
// (exact integers or float) or score with different algorithms form separate
// classes, each its own queue, since their tiles run different kernel
// variants.  Each series keeps its plan's octave series in a region of its
// own in the batch workspace; outputs go through a per-series table the
// kernels index by Phase::series.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "ffa_internal.h"

using namespace ffa;

namespace {

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Device copies of one class's tables.
struct ClassDev {
  Phase* phases = nullptr;
  int32_t* tile_phase = nullptr;
  int32_t* widths = nullptr;
  double* sqrtw = nullptr;
};

struct BatchDev {
  int device = -1;
  std::vector<ClassDev> cls;
  DeredSeg* dered_segs = nullptr;  // the dereddening plan of all the batch's float series
  int32_t* dered_block_seg = nullptr;
  hipEvent_t done = nullptr;  // recorded after each search (cached batches only)
};

struct BatchClass {
  int32_t is_int = 0, alg = 1, select_iters = 64, select_cand = 64;
  std::vector<Step> steps;
  std::vector<Phase> nat;
  Queue q;
  int64_t ring_off = 0;
  std::vector<int32_t> wtab;
  std::vector<double> sqrtw;  // sqrt(width) of every entry, then 1/sqrt(width)
};

void free_class(ClassDev& c) {
  if (c.phases) (void)hipFree(c.phases);
  if (c.tile_phase) (void)hipFree(c.tile_phase);
  if (c.widths) (void)hipFree(c.widths);
  if (c.sqrtw) (void)hipFree(c.sqrtw);
  c = ClassDev();
}

}  // namespace

struct ffa_batch_s {
  std::vector<ffa_plan> plans;  // not owned
  std::vector<uint64_t> uids;
  std::vector<int64_t> series_base;  // element offset of each series' region
  int64_t outs_off = 0;              // element offset of the SeriesOut table
  std::vector<BatchClass> classes;
  DeredPlan dered;                   // exact dereddening of every float series, all at once
  std::vector<uint8_t> dered_by_batch;  // series whose dereddening is in `dered`
  int64_t n_tiles = 0;
  int32_t n_launches = 0;
  size_t ws_bytes = 0;
  bool track_use = false;  // record an event after each search (cached batches)
  std::mutex dev_mu;
  std::deque<BatchDev> dev;
};

namespace {

void free_batch_device(ffa_batch_s* b) {
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (auto& d : b->dev) {
    if (d.device != cur) (void)hipSetDevice(d.device);
    if (d.done) {
      (void)hipEventSynchronize(d.done);
      (void)hipEventDestroy(d.done);
    }
    for (auto& c : d.cls) free_class(c);
    if (d.dered_segs) (void)hipFree(d.dered_segs);
    if (d.dered_block_seg) (void)hipFree(d.dered_block_seg);
    if (d.device != cur && cur >= 0) (void)hipSetDevice(cur);
  }
  b->dev.clear();
}

// Host planning of a batch: classes, steps, queues, workspace layout.
ffa_status plan_batch(int32_t n, const ffa_plan* plans, ffa_batch_s** out) {
  if (n < 1 || !plans) return fail(FFA_ERR_INVALID, "need at least one plan");
  for (int32_t i = 0; i < n; ++i)
    if (!plans[i]) return fail(FFA_ERR_INVALID, "null plan");
  std::unique_ptr<ffa_batch_s> b(new (std::nothrow) ffa_batch_s());
  if (!b) return fail(FFA_ERR_NOMEM, "batch allocation");
  b->plans.assign(plans, plans + n);
  for (int32_t i = 0; i < n; ++i) b->uids.push_back(plans[i]->uid);
  // workspace: output table, then one series region per series
  int64_t cur = 0;
  b->outs_off = cur;
  cur = round_up(cur + 4 * (int64_t)n, 64);  // SeriesOut is 16 B = 4 elements
  for (int32_t i = 0; i < n; ++i) {
    b->series_base.push_back(cur);
    cur = round_up(cur + plans[i]->series_elems, 64);
  }
  // the exact dereddening of every float series as one plan of launches
  b->dered_by_batch.assign((size_t)n, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (plans[i]->dered.segs.empty()) continue;
    b->dered_by_batch[(size_t)i] = 1;
    for (DeredSeg sg : plans[i]->dered.segs) {
      sg.x_off += b->series_base[(size_t)i];
      sg.out_off += b->series_base[(size_t)i];
      b->dered.segs.push_back(sg);
    }
  }
  plan_dered(b->dered);
  // classes: (exact integer folds, algorithm, selection exits)
  std::vector<int32_t> cls_of((size_t)n, -1);
  for (int32_t i = 0; i < n; ++i) {
    const ffa_plan p = plans[i];
    const int32_t alg = p->desc.snr == FFA_SNR_ALG2_OFFPULSE ? 2 : 1;
    for (size_t c = 0; c < b->classes.size(); ++c) {
      const BatchClass& k = b->classes[c];
      if (k.is_int == p->acc_int && k.alg == alg && k.select_iters == p->select_iters &&
          k.select_cand == p->select_cand)
        cls_of[(size_t)i] = (int32_t)c;
    }
    if (cls_of[(size_t)i] < 0) {
      BatchClass k;
      k.is_int = p->acc_int;
      k.alg = alg;
      k.select_iters = p->select_iters;
      k.select_cand = p->select_cand;
      cls_of[(size_t)i] = (int32_t)b->classes.size();
      b->classes.push_back(std::move(k));
    }
  }
  for (size_t c = 0; c < b->classes.size(); ++c) {
    BatchClass& k = b->classes[c];
    // width tables of the class: each plan's widths at an offset
    std::vector<int32_t> wbase((size_t)n, 0);
    for (int32_t i = 0; i < n; ++i) {
      if (cls_of[(size_t)i] != (int32_t)c) continue;
      wbase[(size_t)i] = (int32_t)k.wtab.size();
      k.wtab.insert(k.wtab.end(), plans[i]->wtab.begin(), plans[i]->wtab.end());
    }
    const int32_t nsq = (int32_t)k.wtab.size();
    for (int32_t w : k.wtab) k.sqrtw.push_back(std::sqrt((double)w));
    for (int32_t j = 0; j < nsq; ++j) k.sqrtw.push_back(1.0 / k.sqrtw[(size_t)j]);
    // the launch knobs of the class: the largest windows and ring any of its
    // plans asks for
    QueueKnobs kn;
    bool first = true;
    for (int32_t i = 0; i < n; ++i) {
      if (cls_of[(size_t)i] != (int32_t)c) continue;
      const QueueKnobs& pk = plans[i]->knobs;
      if (first) {
        kn = pk;
        first = false;
      } else {
        kn.window_tiles = std::max(kn.window_tiles, pk.window_tiles);
        kn.ring_bytes = std::max(kn.ring_bytes, pk.ring_bytes);
        if (kn.fixed_steps != pk.fixed_steps) kn.fixed_steps = 0;
        kn.split_occupancy = kn.split_occupancy && pk.split_occupancy;
      }
    }
    // A class with many windows' worth of tiles runs window groups 8x larger
    // than one plan's, with a ring 4x larger (fewer launches and launch
    // tails; the batch is one job with one workspace on a 288 GB part).
    {
      int64_t class_tiles = 0;
      for (int32_t i = 0; i < n; ++i)
        if (cls_of[(size_t)i] == (int32_t)c)
          for (const Step& ps : plans[i]->steps) class_tiles += ps.total_tiles;
      if (kn.fixed_steps == 0 && class_tiles >= 64 * (int64_t)kn.window_tiles && kn.window_tiles <= (1 << 21)) {
        kn.window_tiles *= 8;
        kn.ring_bytes *= 4;
      }
    }
    // steps and their natural-order phases, series by series
    for (int32_t i = 0; i < n; ++i) {
      if (cls_of[(size_t)i] != (int32_t)c) continue;
      const ffa_plan p = plans[i];
      for (const Step& ps : p->steps) {
        Step s = ps;
        s.series = i;
        s.oct_off = b->series_base[(size_t)i] + p->oct_off[(size_t)s.octave];
        s.in_end = s.oct_off + p->oct_len[(size_t)s.octave];
        s.wofs = ps.wofs + wbase[(size_t)i];
        s.fold_phase0 = (int32_t)k.nat.size();
        const int32_t si = (int32_t)k.steps.size();
        for (int32_t pass = 0; pass < s.n_passes; ++pass) {
          Phase ph = p->nat_phases[(size_t)(ps.fold_phase0 + pass)];
          ph.step = si;
          ph.series = i;
          ph.oct_off = s.oct_off;
          ph.wofs = s.wofs;
          ph.isqrt_ofs = nsq + s.wofs;
          k.nat.push_back(ph);
        }
        k.steps.push_back(s);
      }
    }
    ffa_status st = build_queue(k.steps, k.nat, kn, &k.q);
    if (st != FFA_OK) return st;
    if (!queue_valid(k.steps, k.q, k.is_int))
      return fail(FFA_ERR_INVALID, "internal planning error: a batch tile reaches outside its buffers");
    k.ring_off = round_up(cur, 64);
    cur = k.ring_off + k.q.ring_elems;
    b->n_tiles += k.q.n_tiles;
    b->n_launches += (int32_t)k.q.launches.size();
  }
  b->ws_bytes = (size_t)round_up(cur * 4, (int64_t)kWsAlign);
  *out = b.release();
  return FFA_OK;
}

// Device tables of batch b on the current device (made on first use).
ffa_status batch_device(ffa_batch_s* b, BatchDev** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(b->dev_mu);
  for (auto& d : b->dev)
    if (d.device == dev) {
      *out = &d;
      return FFA_OK;
    }
  BatchDev d;
  d.device = dev;
  auto release = [&] {
    for (auto& c : d.cls) free_class(c);
    if (d.dered_segs) (void)hipFree(d.dered_segs);
    if (d.dered_block_seg) (void)hipFree(d.dered_block_seg);
    if (d.done) (void)hipEventDestroy(d.done);
  };
  ffa_status st = FFA_OK;
  if (b->track_use) st = check_hip(hipEventCreateWithFlags(&d.done, hipEventDisableTiming), "batch event");
  if (st == FFA_OK) st = upload_dered(b->dered, &d.dered_segs, &d.dered_block_seg);
  for (const BatchClass& k : b->classes) {
    if (st != FFA_OK) break;
    ClassDev c;
    const size_t pb = k.q.phases.size() * sizeof(Phase);
    const size_t tb = k.q.tile_phase.size() * sizeof(int32_t);
    const size_t wb = std::max<size_t>(k.wtab.size(), 1) * sizeof(int32_t);
    const size_t sb = std::max<size_t>(k.sqrtw.size(), 1) * sizeof(double);
    if (hipMalloc(&c.phases, pb) != hipSuccess || hipMalloc(&c.tile_phase, tb) != hipSuccess ||
        hipMalloc(&c.widths, wb) != hipSuccess || hipMalloc(&c.sqrtw, sb) != hipSuccess) {
      free_class(c);
      st = fail(FFA_ERR_NOMEM, "batch tables: hipMalloc failed");
      break;
    }
    d.cls.push_back(c);
    st = check_hip(hipMemcpy(c.phases, k.q.phases.data(), pb, hipMemcpyHostToDevice), "upload batch phases");
    if (st == FFA_OK)
      st = check_hip(hipMemcpy(c.tile_phase, k.q.tile_phase.data(), tb, hipMemcpyHostToDevice),
                     "upload batch tile map");
    if (st == FFA_OK && !k.wtab.empty())
      st = check_hip(hipMemcpy(c.widths, k.wtab.data(), k.wtab.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                     "upload batch widths");
    if (st == FFA_OK && !k.sqrtw.empty())
      st = check_hip(hipMemcpy(c.sqrtw, k.sqrtw.data(), k.sqrtw.size() * sizeof(double), hipMemcpyHostToDevice),
                     "upload batch sqrt widths");
  }
  if (st != FFA_OK) {
    release();
    return st;
  }
  b->dev.push_back(std::move(d));
  *out = &b->dev.back();
  return FFA_OK;
}

ffa_status check_batch_ws(const ffa_batch_s* b, const void* d_ws, size_t ws_bytes) {
  if (!d_ws) return fail(FFA_ERR_INVALID, "null workspace");
  if (ws_bytes < b->ws_bytes) return fail(FFA_ERR_INVALID, "workspace smaller than the batch's ws_bytes");
  if (reinterpret_cast<uintptr_t>(d_ws) % kWsAlign) return fail(FFA_ERR_INVALID, "workspace not 256-byte aligned");
  return FFA_OK;
}

// Every series' octave series (centred float, or exact integer sums), each
// in its region of the workspace.
ffa_status prepare_batch(ffa_batch_s* b, const void* const* d_series, void* d_ws, size_t ws_bytes, hipStream_t st) {
  if (!d_series) return fail(FFA_ERR_INVALID, "null argument");
  ffa_status s = check_batch_ws(b, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const size_t n = b->plans.size();
  for (size_t i = 0; i < n; ++i)
    if (!d_series[i]) return fail(FFA_ERR_INVALID, "null series");
  BatchDev* dev = nullptr;
  s = batch_device(b, &dev);
  if (s != FFA_OK) return s;
  char* ws = reinterpret_cast<char*>(d_ws);
  for (size_t i = 0; i < n && s == FFA_OK; ++i) {
    const ffa_plan p = b->plans[i];
    s = build_octaves(p, d_series[i], ws + (size_t)b->series_base[i] * 4, p->n_octaves - 1, 1, st, nullptr,
                      !b->dered_by_batch[i]);
  }
  // every float series' octaves dereddened together
  if (s == FFA_OK && dev->dered_segs) s = run_dered(b->dered, dev->dered_segs, dev->dered_block_seg, d_ws, st);
  return s;
}

// The queues, window by window, on the octave series already in the workspace.
ffa_status search_prepared_batch(ffa_batch_s* b, float* const* d_snr, int32_t* const* d_width, void* d_ws,
                                 size_t ws_bytes, hipStream_t st) {
  if (!d_snr || !d_width) return fail(FFA_ERR_INVALID, "null argument");
  ffa_status s = check_batch_ws(b, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const size_t n = b->plans.size();
  std::vector<SeriesOut> outs(n);
  for (size_t i = 0; i < n; ++i) {
    if (!d_snr[i] || !d_width[i]) return fail(FFA_ERR_INVALID, "null output");
    outs[i] = SeriesOut{d_snr[i], d_width[i]};
  }
  BatchDev* dev = nullptr;
  s = batch_device(b, &dev);
  if (s != FFA_OK) return s;
  char* ws = reinterpret_cast<char*>(d_ws);
  SeriesOut* outs_dev = reinterpret_cast<SeriesOut*>(ws + (size_t)b->outs_off * 4);
  s = check_hip(launch_set_outs(outs_dev, outs.data(), (int32_t)n, st), "output table kernel");
  for (size_t c = 0; c < b->classes.size() && s == FFA_OK; ++c) {
    const BatchClass& k = b->classes[c];
    const ClassDev& cd = dev->cls[c];
    TileArgs a{};
    a.phases = cd.phases;
    a.tile_phase = cd.tile_phase;
    a.widths = cd.widths;
    a.sqrtw = cd.sqrtw;
    a.outs = outs_dev;
    a.oct_base = 0;
    a.ring_off = k.ring_off;
    a.mode = kModeScore;
    a.alg = k.alg;
    a.select_iters = k.select_iters;
    a.select_cand = k.select_cand;
    for (const Launch& w : k.q.launches) {
      if (w.ntiles == 0) continue;
      a.tile0 = w.tile0;
      s = check_hip(launch_tiles(a, w.ntiles, w.lds_bytes, w.max_P0, k.is_int, d_ws, st), "FFA kernel");
      if (s != FFA_OK) break;
    }
  }
  if (b->track_use && dev->done) {
    const ffa_status e = check_hip(hipEventRecord(dev->done, st), "batch event record");
    if (s == FFA_OK) s = e;
  }
  return s;
}

ffa_status run_batch(ffa_batch_s* b, const void* const* d_series, float* const* d_snr, int32_t* const* d_width,
                     void* d_ws, size_t ws_bytes, hipStream_t st) {
  if (!d_series || !d_snr || !d_width) return fail(FFA_ERR_INVALID, "null argument");
  const size_t n = b->plans.size();
  for (size_t i = 0; i < n; ++i)
    if (!d_series[i] || !d_snr[i] || !d_width[i]) return fail(FFA_ERR_INVALID, "null series or output");
  ffa_status s = prepare_batch(b, d_series, d_ws, ws_bytes, st);
  if (s != FFA_OK) return s;
  return search_prepared_batch(b, d_snr, d_width, d_ws, ws_bytes, st);
}

// Batches made by ffa_search_batch / ffa_batch_workspace, kept for reuse:
// the most recently used few, keyed by their plans (plan uids are never
// reused, so a destroyed plan never matches).  An evicted batch waits for its
// last search before its tables are freed.
constexpr size_t kCacheSize = 4;
std::mutex g_cache_mu;
std::list<std::shared_ptr<ffa_batch_s>> g_cache;

ffa_status cached_batch(int32_t n, const ffa_plan* plans, std::shared_ptr<ffa_batch_s>* out) {
  if (n < 1 || !plans) return fail(FFA_ERR_INVALID, "need at least one plan");
  for (int32_t i = 0; i < n; ++i)
    if (!plans[i]) return fail(FFA_ERR_INVALID, "null plan");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
    const ffa_batch_s& b = **it;
    if (b.plans.size() != (size_t)n) continue;
    bool same = true;
    for (int32_t i = 0; i < n && same; ++i) same = b.plans[(size_t)i] == plans[i] && b.uids[(size_t)i] == plans[i]->uid;
    if (same) {
      g_cache.splice(g_cache.begin(), g_cache, it);
      *out = g_cache.front();
      return FFA_OK;
    }
  }
  ffa_batch_s* raw = nullptr;
  ffa_status s = plan_batch(n, plans, &raw);
  if (s != FFA_OK) return s;
  raw->track_use = true;
  std::shared_ptr<ffa_batch_s> sp(raw, [](ffa_batch_s* b) {
    free_batch_device(b);
    delete b;
  });
  g_cache.push_front(sp);
  while (g_cache.size() > kCacheSize) g_cache.pop_back();
  *out = sp;
  return FFA_OK;
}

}  // namespace

extern "C" ffa_status ffa_batch_create(int32_t n, const ffa_plan* plans, ffa_batch* out) {
  if (!out) return fail(FFA_ERR_INVALID, "null argument");
  *out = nullptr;
  ffa_batch_s* b = nullptr;
  ffa_status s = plan_batch(n, plans, &b);
  if (s != FFA_OK) return s;
  *out = b;
  return FFA_OK;
}

extern "C" ffa_status ffa_batch_destroy(ffa_batch b) {
  if (!b) return fail(FFA_ERR_INVALID, "null batch");
  free_batch_device(b);
  delete b;
  return FFA_OK;
}

extern "C" ffa_status ffa_batch_query(ffa_batch b, size_t* ws_bytes, int64_t* n_tiles, int32_t* n_launches) {
  if (!b) return fail(FFA_ERR_INVALID, "null batch");
  if (ws_bytes) *ws_bytes = b->ws_bytes;
  if (n_tiles) *n_tiles = b->n_tiles;
  if (n_launches) *n_launches = b->n_launches;
  return FFA_OK;
}

extern "C" ffa_status ffa_batch_search(ffa_batch b, const void* const* d_series, float* const* d_snr,
                                       int32_t* const* d_width, void* d_ws, size_t ws_bytes, void* stream) {
  if (!b) return fail(FFA_ERR_INVALID, "null batch");
  return run_batch(b, d_series, d_snr, d_width, d_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

extern "C" ffa_status ffa_batch_prepare(ffa_batch b, const void* const* d_series, void* d_ws, size_t ws_bytes,
                                        void* stream) {
  if (!b) return fail(FFA_ERR_INVALID, "null batch");
  return prepare_batch(b, d_series, d_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

extern "C" ffa_status ffa_batch_search_prepared(ffa_batch b, float* const* d_snr, int32_t* const* d_width, void* d_ws,
                                                size_t ws_bytes, void* stream) {
  if (!b) return fail(FFA_ERR_INVALID, "null batch");
  return search_prepared_batch(b, d_snr, d_width, d_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

extern "C" ffa_status ffa_batch_workspace(int32_t n, const ffa_plan* plans, size_t* ws_bytes) {
  if (!ws_bytes) return fail(FFA_ERR_INVALID, "null argument");
  std::shared_ptr<ffa_batch_s> b;
  ffa_status s = cached_batch(n, plans, &b);
  if (s != FFA_OK) return s;
  *ws_bytes = b->ws_bytes;
  return FFA_OK;
}

extern "C" ffa_status ffa_search_batch(int32_t n, const ffa_plan* plans, const void* const* d_series,
                                       float* const* d_snr, int32_t* const* d_width, void* d_ws,
                                       size_t ws_bytes, void* stream) {
  std::shared_ptr<ffa_batch_s> b;
  ffa_status s = cached_batch(n, plans, &b);
  if (s != FFA_OK) return s;
  return run_batch(b.get(), d_series, d_snr, d_width, d_ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

// Test hook (not in the public header): the queue of class c of a batch
// (phases and launches), so host tests can walk it like a plan's.
extern "C" int64_t ffa_debug_batch(ffa_batch b, int32_t c, void* phases, int64_t cap, int64_t* layout,
                                   int64_t lcap) {
  if (!b || c < 0 || c >= (int32_t)b->classes.size()) return -1;
  const BatchClass& k = b->classes[(size_t)c];
  const int64_t n = (int64_t)k.q.phases.size();
  if (phases && cap >= n) std::memcpy(phases, k.q.phases.data(), (size_t)n * sizeof(Phase));
  const int64_t nw = (int64_t)k.q.launches.size();
  if (layout && lcap >= 8 + 4 * nw) {
    layout[0] = k.ring_off;
    layout[1] = k.q.ring_elems;
    layout[2] = (int64_t)b->classes.size();
    layout[3] = k.q.n_tiles;
    layout[4] = k.q.lds_bytes;
    layout[5] = k.q.max_P0;
    layout[6] = (int64_t)b->ws_bytes;
    layout[7] = k.q.lookahead;
    for (int64_t i = 0; i < nw; ++i) {
      const Launch& w = k.q.launches[(size_t)i];
      layout[8 + 4 * i] = w.tile0;
      layout[9 + 4 * i] = w.ntiles;
      layout[10 + 4 * i] = w.lds_bytes;
      layout[11 + 4 * i] = w.max_P0;
    }
  }
  return n;
}

extern "C" int64_t ffa_debug_batch_series_base(ffa_batch b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->series_base.size()) return -1;
  return b->series_base[(size_t)i];
}
