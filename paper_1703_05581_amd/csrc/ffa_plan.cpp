// Search planning: steps, pass split, work-queue phases, workspace layout.
//
// A plan is built on the host only; its device tables are uploaded on first
// use on a GPU (device_tables), so plans can be made and inspected without a
// GPU.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "ffa_internal.h"

namespace ffa {
namespace {

thread_local std::string g_last_error;

int32_t next_pow2(int64_t m) {
  int32_t M = 1;
  while (M < m) M <<= 1;
  return M;
}

int32_t ilog2(int64_t v) {
  int32_t l = 0;
  while ((int64_t(1) << (l + 1)) <= v) ++l;
  return l;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Widths of a step: the given list in order, without widths above P0; or the
// paper's rule (Sec. 2.2.1): powers of two up to and including the first one
// above 20% of P0.
void step_widths(const std::vector<int32_t>& user, int32_t P0,
                 std::vector<int32_t>* out) {
  out->clear();
  if (!user.empty()) {
    for (int32_t w : user)
      if (w <= P0) out->push_back(w);
    return;
  }
  for (int32_t v = 1; (int)out->size() < kMaxWidths; v *= 2) {
    if (v <= P0) out->push_back(v);
    if (5 * v > P0) break;
  }
}

// Pass split of an L-level step: as few passes as the LDS allows.  The last
// pass keeps its rows with room for the boxcar prefix sums (stride
// P0 + wmax + 1); earlier passes use stride P0.
// LDS row stride of a pass of depth d: P0 bins plus a halo of
// min(2^(d-1), P0) bins for the shifted butterfly reads; the last pass also
// needs P0 + wmax + 1 entries for the boxcar prefix sums.
// Where the LDS budget still allows it at the same depth, the row keeps
// 3*2^(d-2) spare bins instead, so the kernel can run the top two levels as
// one radix-4 pass (it reads the spare room from the stride).
int32_t halo_of(int32_t P0, int32_t d) { return std::min<int32_t>(int32_t(1) << (d - 1), P0); }
// esz: bytes per LDS element (4, or 2 for a 16-bit first pass).
int32_t stride_of(const Step& s, int32_t d, bool last, int32_t esz = 4) {
  const int32_t extra = last ? s.wmax + 1 : 0;
  const int32_t base = s.P0 + std::max<int32_t>(halo_of(s.P0, d), extra);
  if (d >= 2) {
    const int32_t wide = s.P0 + std::max<int32_t>(std::min<int32_t>(3 << (d - 2), s.P0), extra);
    const int64_t lds = (int64_t(1) << d) * wide * esz + (last ? (int64_t)kScratchBytes : 0);
    if (wide > base && lds <= s.lds_budget) return wide;
  }
  return base;
}
int64_t lds_of(const Step& s, int32_t d, bool last, int32_t esz = 4) {
  return (int64_t(1) << d) * stride_of(s, d, last, esz) * esz + (last ? (int64_t)kScratchBytes : 0);
}
int32_t esz_of(const Phase& ph) { return ph.u16 ? 2 : 4; }

void split_passes(Step* s, int64_t lds_budget) {
  s->lds_budget = lds_budget;
  int32_t dfin = 1, dmid = 1;
  auto fits = [&](int32_t d, bool last) { return lds_of(*s, d, last) <= lds_budget; };
  while (dfin < 24 && fits(dfin + 1, true)) ++dfin;
  while (dmid < 24 && fits(dmid + 1, false)) ++dmid;
  if (s->L <= dfin) {
    s->n_passes = 1;
    s->depth[0] = s->L;
    return;
  }
  // fewest passes, depths as equal as the LDS allows, deeper passes first
  int32_t np = 2;
  for (;; ++np) {
    int32_t left = s->L, ok = 1;
    for (int32_t i = np - 1; i >= 0; --i) {
      const int32_t cap = i == np - 1 ? dfin : dmid;
      const int32_t d = std::min(cap, left - i);  // leave >= 1 level per earlier pass
      if (d < 1) ok = 0;
      left -= d;
    }
    if (ok && left <= 0) break;
  }
  int32_t dep[kMaxPasses + 8];
  for (int32_t i = 0; i < np; ++i) dep[i] = s->L / np + (i < s->L % np ? 1 : 0);
  // respect the caps: move levels from a pass above its cap to others
  for (int iter = 0; iter < 64; ++iter) {
    bool moved = false;
    for (int32_t i = 0; i < np; ++i) {
      const int32_t cap = i == np - 1 ? dfin : dmid;
      if (dep[i] <= cap) continue;
      for (int32_t j = 0; j < np; ++j) {
        const int32_t cj = j == np - 1 ? dfin : dmid;
        if (j != i && dep[j] < cj) {
          --dep[i];
          ++dep[j];
          moved = true;
          break;
        }
      }
    }
    if (!moved) break;
  }
  for (int32_t i = 0; i < np; ++i) s->depth[i] = dep[i];
  s->n_passes = np;
}

// Ring space a multi-pass step's intermediates take: one M*P0 buffer, two
// when a middle pass reads one and writes the other; 64-element aligned.
int64_t ring_region(const Step& s) {
  return s.n_passes > 1 ? round_up((int64_t)(s.n_passes > 2 ? 2 : 1) * s.M * s.P0, 64) : 0;
}

// The ring as an arena.  Steps are cut into groups of consecutive steps;
// pass p of a step in group g runs in window g + p, so a group's
// intermediates are live in windows g .. g + max_passes - 1.  The groups'
// multi-pass steps are placed one after another, groups in order, wrapping
// to the start when a group would run past the end.  At most max_passes
// consecutive groups are live at once, so a ring of the largest such sum
// plus the largest group is enough: the live span then wraps at most once,
// and the space a wrap skips is less than the group that wraps.
int64_t ring_need(const std::vector<Step>& steps, const std::vector<int32_t>& grp, int32_t max_passes) {
  std::vector<int64_t> g(steps.empty() ? 0 : (size_t)grp.back() + 1, 0);
  for (size_t i = 0; i < steps.size(); ++i) g[(size_t)grp[i]] += ring_region(steps[i]);
  int64_t best = 0, gmax = 0, run = 0;
  for (size_t i = 0; i < g.size(); ++i) {
    run += g[i];
    if (i >= (size_t)max_passes) run -= g[i - (size_t)max_passes];
    best = std::max(best, run);
    gmax = std::max(gmax, g[i]);
  }
  return best + gmax;
}

int64_t place_ring(std::vector<Step>& steps, const std::vector<int32_t>& grp, int32_t max_passes) {
  const int64_t cap = ring_need(steps, grp, max_passes);
  int64_t head = 0;
  for (size_t i0 = 0; i0 < steps.size();) {
    size_t i1 = i0;
    int64_t size = 0;
    while (i1 < steps.size() && grp[i1] == grp[i0]) size += ring_region(steps[i1++]);
    if (head + size > cap) head = 0;
    for (size_t i = i0; i < i1; ++i) {
      steps[i].ring_pos = head;
      head += ring_region(steps[i]);
    }
    i0 = i1;
  }
  return cap;
}

// Groups of consecutive steps: each closes once it holds about `target`
// tiles (all passes), or once its ring share would pass
// budget / (max_passes + 1), which keeps ring_need within the budget unless
// a single step alone is larger.  `fixed` > 0 instead takes that many steps
// per group.
std::vector<int32_t> group_steps(const std::vector<Step>& steps, int64_t target, int64_t budget_elems,
                                 int32_t max_passes, int64_t fixed) {
  std::vector<int32_t> grp(steps.size(), 0);
  const int64_t share = max_passes > 1 ? budget_elems / (max_passes + 1) : INT64_MAX;
  int32_t g = 0;
  int64_t tiles = 0, ring = 0, n = 0;
  for (size_t i = 0; i < steps.size(); ++i) {
    const int64_t t = steps[i].total_tiles, r = ring_region(steps[i]);
    const bool full = fixed > 0 ? n >= fixed : (tiles + t > target || ring + r > share);
    if (n > 0 && full) {
      ++g;
      tiles = ring = n = 0;
    }
    grp[i] = g;
    tiles += t;
    ring += r;
    ++n;
  }
  return grp;
}

}  // namespace

int64_t phase_lds(const Phase& ph) {
  return (int64_t(1) << ph.depth) * ph.stride * esz_of(ph) + (ph.last ? (int64_t)kScratchBytes : 0);
}

// Every tile a phase can produce must read and write inside its buffers (its
// octave series, its step's two intermediate buffers in the ring, its own
// trials, one workgroup's LDS), and every tile it reads must come from an
// earlier launch.  Checked once per queue, before anything can be launched.
bool queue_valid(const std::vector<Step>& steps, const Queue& q, int acc_int) {
  const size_t ns = steps.size();
  std::vector<int32_t> first_win(ns, -1), last_win(ns, -1);
  std::vector<int32_t> pass_win(ns * kMaxPasses, -1);
  int64_t expect = 0;
  int32_t prev_launch = 0;
  for (size_t i = 0; i < q.phases.size(); ++i) {
    const Phase& ph = q.phases[i];
    if (ph.tile0 != expect || ph.ntiles < 1) return false;
    expect += ph.ntiles;
    if (ph.step < 0 || ph.step >= (int32_t)ns) return false;
    if (ph.launch < prev_launch || ph.launch >= (int32_t)q.launches.size()) return false;
    prev_launch = ph.launch;
    const Launch& w = q.launches[(size_t)ph.launch];
    if (ph.tile0 < w.tile0 || ph.tile0 + ph.ntiles > w.tile0 + w.ntiles) return false;
    const Step& s = steps[ph.step];
    const int32_t dp = ph.depth;
    if (ph.pass < 0 || ph.pass >= s.n_passes || dp != s.depth[ph.pass] || dp < 1 || dp > 24) return false;
    if (ph.series != s.series) return false;
    int32_t D = 0;
    for (int32_t j = 0; j < ph.pass; ++j) D += s.depth[j];
    const bool last = ph.pass == s.n_passes - 1;
    if (ph.D != D || ph.last != (int32_t)last || ph.P0 != s.P0 || ph.M != s.M) return false;
    const int64_t R = int64_t(1) << dp;
    const int64_t Q = int64_t(1) << D;
    const int64_t MP = (int64_t)s.M * s.P0;
    if ((int64_t)ph.ntiles != Q * ph.ng || ph.ng < 1 || ph.vin < 1) return false;
    if (ph.halo < std::min<int64_t>(R / 2, s.P0) || ph.halo > s.P0) return false;
    if (ph.stride < s.P0 + ph.halo || (last && ph.stride < s.P0 + s.wmax + 1)) return false;
    if (ph.u16 && (ph.pass != 0 || last || !acc_int || s.octave + dp > 8)) return false;
    const int64_t lds = phase_lds(ph);
    if (lds > (int64_t)kLdsBytes || lds > w.lds_bytes || ph.P0 > w.max_P0) return false;
    if (ph.wofs != s.wofs || ph.nw != s.nw || (last && s.nw < 1)) return false;
    if (s.n_passes > 1 && (s.ring_pos < 0 || s.ring_pos % 64 || (int64_t)ph.ring64 * 64 != s.ring_pos ||
                           s.ring_pos + ring_region(s) > q.ring_elems || ring_region(s) < MP * (s.n_passes > 2 ? 2 : 1)))
      return false;
    const int64_t Gin = (int64_t)s.M >> D;
    for (int64_t k = 0; k < ph.ntiles; ++k) {
      if (q.tile_phase[(size_t)(ph.tile0 + k)] != (int32_t)i) return false;
      const int64_t qq = k / ph.ng, h = k % ph.ng;
      const int64_t valid = std::min<int64_t>(R, ph.vin - (h << dp));
      if (valid < 1) return false;
      const int64_t src = (qq * Gin + (h << dp)) * s.P0;  // relative to the input buffer
      if (ph.pass == 0) {
        if (ph.oct_off != s.oct_off || s.oct_off < 0) return false;
        if (src < 0 || src + valid * s.P0 > (int64_t)s.m * s.P0) return false;
        if (s.oct_off + (int64_t)s.m * s.P0 > s.in_end) return false;
      } else if (src < 0 || src + valid * s.P0 > MP) {
        return false;
      }
      if (!last) {
        const int64_t Gout = Gin >> dp;
        const int64_t dst = ((qq << dp) * Gout + h) * s.P0;
        if (Gout < 1 || dst < 0 || dst + (R - 1) * Gout * s.P0 + s.P0 > MP) return false;
      } else if ((qq << dp) + R > s.M) {
        return false;
      }
    }
    // the previous pass of the step ran in an earlier launch
    if (ph.pass > 0 && !(pass_win[(size_t)ph.step * kMaxPasses + ph.pass - 1] >= 0 &&
                         pass_win[(size_t)ph.step * kMaxPasses + ph.pass - 1] < ph.launch))
      return false;
    pass_win[(size_t)ph.step * kMaxPasses + ph.pass] = ph.launch;
    if (ph.pass == 0) first_win[(size_t)ph.step] = ph.launch;
    if (last) last_win[(size_t)ph.step] = ph.launch;
  }
  if (expect != q.n_tiles || (int64_t)q.tile_phase.size() != q.n_tiles) return false;
  // ring: two multi-pass steps whose launches overlap hold disjoint ranges
  std::vector<size_t> multi;
  for (size_t si = 0; si < ns; ++si) {
    if (first_win[si] < 0 || last_win[si] < 0) return false;
    if (steps[si].n_passes > 1) multi.push_back(si);
  }
  std::stable_sort(multi.begin(), multi.end(), [&](size_t a, size_t b) { return first_win[a] < first_win[b]; });
  std::vector<size_t> live;
  for (size_t si : multi) {
    const Step& s = steps[si];
    live.erase(std::remove_if(live.begin(), live.end(), [&](size_t o) { return last_win[o] < first_win[si]; }),
               live.end());
    for (size_t o : live) {
      const Step& t = steps[o];
      if (s.ring_pos < t.ring_pos + ring_region(t) && t.ring_pos < s.ring_pos + ring_region(s)) return false;
    }
    live.push_back(si);
  }
  return true;
}

// Queue order: windows of consecutive step groups (about window_tiles tiles
// each, within the ring budget), pass p of group g in window g + p, each
// window one launch per occupancy class.  The previous pass of a step is then
// always in an earlier window.
ffa_status build_queue(std::vector<Step>& steps, std::vector<Phase>& nat, const QueueKnobs& kn, Queue* q) {
  *q = Queue();
  int64_t tiles_total = 0;
  for (const Step& s : steps) {
    tiles_total += s.total_tiles;
    q->max_passes = std::max(q->max_passes, s.n_passes);
    q->lds_bytes = std::max(q->lds_bytes, s.lds_bytes);
    q->max_P0 = std::max(q->max_P0, s.P0);
  }
  q->n_tiles = tiles_total;
  if (tiles_total >= (int64_t(1) << 31)) return fail(FFA_ERR_UNSUPPORTED, "too many tiles in one queue");
  const std::vector<int32_t> grp =
      group_steps(steps, kn.window_tiles, kn.ring_bytes / 4, q->max_passes, kn.fixed_steps);
  q->ring_elems = place_ring(steps, grp, q->max_passes);
  {
    int32_t most = 0;
    for (size_t i0 = 0, i1 = 0; i0 < grp.size(); i0 = i1) {
      while (i1 < grp.size() && grp[i1] == grp[i0]) ++i1;
      most = std::max<int32_t>(most, (int32_t)(i1 - i0));
    }
    q->lookahead = most;
  }
  for (Phase& ph : nat) ph.ring64 = (int32_t)(steps[(size_t)ph.step].ring_pos / 64);
  // occupancy class: workgroups per CU that the phase's LDS footprint allows
  auto occ_class = [&](const Phase& ph) {
    if (!kn.split_occupancy) return (int32_t)0;
    return (int32_t)std::min<int64_t>(4, (int64_t)kLdsBytes / std::max<int64_t>(phase_lds(ph), 1));
  };
  struct Key {
    int64_t key;  // window
    int32_t pass, step, cls;
  };
  std::vector<Key> order;
  order.reserve(nat.size());
  for (size_t i = 0; i < nat.size(); ++i)
    order.push_back({(int64_t)grp[(size_t)nat[i].step] + nat[i].pass, nat[i].pass, nat[i].step, occ_class(nat[i])});
  std::stable_sort(order.begin(), order.end(), [](const Key& a, const Key& b) {
    if (a.key != b.key) return a.key < b.key;  // window
    if (a.cls != b.cls) return a.cls < b.cls;
    return a.step != b.step ? a.step < b.step : a.pass < b.pass;
  });
  int64_t t0 = 0, cur_win = -1;
  int32_t cur_cls = -1;
  q->tile_phase.reserve((size_t)tiles_total);
  q->phases.reserve(nat.size());
  for (const Key& k : order) {
    Phase ph = nat[(size_t)(steps[(size_t)k.step].fold_phase0 + k.pass)];
    if (k.key != cur_win || k.cls != cur_cls) {
      q->launches.push_back(Launch{t0, 0, 0, 0});
      cur_win = k.key;
      cur_cls = k.cls;
    }
    Launch& ln = q->launches.back();
    ph.launch = (int32_t)(q->launches.size() - 1);
    ph.tile0 = t0;
    ln.ntiles += ph.ntiles;
    ln.lds_bytes = std::max<int32_t>(ln.lds_bytes, (int32_t)phase_lds(ph));
    ln.max_P0 = std::max(ln.max_P0, ph.P0);
    const int32_t idx = (int32_t)q->phases.size();
    q->tile_phase.insert(q->tile_phase.end(), (size_t)ph.ntiles, idx);
    t0 += ph.ntiles;
    q->phases.push_back(ph);
  }
  return FFA_OK;
}

ffa_status fail(ffa_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ffa_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return FFA_OK;
  return fail(FFA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error_cstr() { return g_last_error.c_str(); }

void plan_dered(DeredPlan& dp) {
  dp.block_seg.clear();
  dp.launches.clear();
  // blocks of one segment that fit a CU together (1024 threads each: at most 2)
  std::vector<int32_t> lds(dp.segs.size());
  std::vector<int32_t> per_cu(dp.segs.size());
  for (size_t i = 0; i < dp.segs.size(); ++i) {
    int32_t use_stage = 0;
    lds[i] = (int32_t)dered_block_lds(dp.segs[i].n, dp.segs[i].window, &use_stage);
    dp.segs[i].use_stage = use_stage;
    per_cu[i] = (int32_t)std::max<size_t>(1, std::min<size_t>(2, kLdsBytes / (size_t)lds[i]));
  }
  std::vector<size_t> order(dp.segs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return per_cu[a] > per_cu[b]; });
  std::vector<DeredSeg> segs;
  int64_t blk = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    const size_t i = order[k];
    if (dp.launches.empty() || per_cu[i] != per_cu[order[k - 1]])
      dp.launches.push_back(DeredLaunch{blk, 0, 0});
    DeredLaunch& L = dp.launches.back();
    DeredSeg sg = dp.segs[i];
    sg.block0 = blk;
    const int64_t nb = dered_block_count(sg.n);
    for (int64_t b = 0; b < nb; ++b) dp.block_seg.push_back((int32_t)segs.size());
    segs.push_back(sg);
    blk += nb;
    L.blocks += nb;
    L.lds = std::max(L.lds, lds[i]);
  }
  dp.segs = std::move(segs);
}

ffa_status upload_dered(const DeredPlan& dp, DeredSeg** segs, int32_t** block_seg) {
  *segs = nullptr;
  *block_seg = nullptr;
  if (dp.segs.empty()) return FFA_OK;
  const size_t sb = dp.segs.size() * sizeof(DeredSeg), bb = dp.block_seg.size() * sizeof(int32_t);
  if (hipMalloc(segs, sb) != hipSuccess || hipMalloc(block_seg, bb) != hipSuccess) {
    if (*segs) (void)hipFree(*segs);
    *segs = nullptr;
    *block_seg = nullptr;
    (void)hipGetLastError();
    return fail(FFA_ERR_NOMEM, "dereddening tables: hipMalloc failed");
  }
  ffa_status st = check_hip(prepare_dered_batch(), "dereddening kernel attributes");
  if (st == FFA_OK)
    st = check_hip(hipMemcpy(*segs, dp.segs.data(), sb, hipMemcpyHostToDevice), "upload dereddening plan");
  if (st == FFA_OK)
    st = check_hip(hipMemcpy(*block_seg, dp.block_seg.data(), bb, hipMemcpyHostToDevice),
                   "upload dereddening block map");
  if (st != FFA_OK) {
    (void)hipFree(*segs);
    (void)hipFree(*block_seg);
    *segs = nullptr;
    *block_seg = nullptr;
  }
  return st;
}

ffa_status run_dered(const DeredPlan& dp, const DeredSeg* d_segs, const int32_t* d_block_seg, void* ws,
                     hipStream_t st) {
  for (const DeredLaunch& L : dp.launches) {
    const ffa_status s = check_hip(launch_dered_batch(d_segs, d_block_seg, L, ws, st), "dereddening kernel");
    if (s != FFA_OK) return s;
  }
  return FFA_OK;
}

ffa_status find_device_tables(ffa_plan p, const DeviceTables** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(p->dev_mu);
  for (auto& t : p->dev)
    if (t.device == dev) {
      *out = &t;
      return FFA_OK;
    }
  return fail(FFA_ERR_INVALID, "the plan has no device tables on this GPU yet (ffa_plan_upload makes them)");
}

ffa_status device_tables(ffa_plan p, const DeviceTables** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(p->dev_mu);
  for (auto& t : p->dev)
    if (t.device == dev) {
      *out = &t;
      return FFA_OK;
    }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(FFA_ERR_DEVICE, "hipGetDeviceProperties failed");
  if (prop.sharedMemPerBlock < kLdsBytes)
    return fail(FFA_ERR_UNSUPPORTED, "device has less than 160 KiB of LDS per workgroup (" +
                                         std::to_string(prop.sharedMemPerBlock) + " B)");
  DeviceTables t;
  t.device = dev;
  const size_t pb = p->phases.size() * sizeof(Phase);
  const size_t fb = p->fold_phases.size() * sizeof(Phase);
  const size_t tb = p->tile_phase.size() * sizeof(int32_t);
  std::vector<StepDev> sd;
  for (const Step& st : p->steps) sd.push_back(StepDev{st.first_trial, st.f, st.P0, st.m, st.M});
  const size_t sdb = sd.size() * sizeof(StepDev);
  const size_t wb = std::max<size_t>(p->wtab.size(), 1) * sizeof(int32_t);
  const size_t sb = std::max<size_t>(p->sqrtw.size(), 1) * sizeof(double);
  auto free_all = [&] {
    if (t.phases) (void)hipFree(t.phases);
    if (t.fold_phases) (void)hipFree(t.fold_phases);
    if (t.tile_phase) (void)hipFree(t.tile_phase);
    if (t.steps) (void)hipFree(t.steps);
    if (t.widths) (void)hipFree(t.widths);
    if (t.sqrtw) (void)hipFree(t.sqrtw);
  };
  if (hipMalloc(&t.phases, pb) != hipSuccess || hipMalloc(&t.fold_phases, fb) != hipSuccess ||
      hipMalloc(&t.tile_phase, tb) != hipSuccess || hipMalloc(&t.steps, sdb) != hipSuccess ||
      hipMalloc(&t.widths, wb) != hipSuccess || hipMalloc(&t.sqrtw, sb) != hipSuccess) {
    free_all();
    return fail(FFA_ERR_NOMEM, "device tables: hipMalloc failed");
  }
  ffa_status st = check_hip(hipMemcpy(t.phases, p->phases.data(), pb, hipMemcpyHostToDevice), "upload phases");
  if (st == FFA_OK)
    st = check_hip(hipMemcpy(t.fold_phases, p->fold_phases.data(), fb, hipMemcpyHostToDevice),
                   "upload fold phases");
  if (st == FFA_OK)
    st = check_hip(hipMemcpy(t.tile_phase, p->tile_phase.data(), tb, hipMemcpyHostToDevice),
                   "upload tile map");
  if (st == FFA_OK)
    st = check_hip(hipMemcpy(t.steps, sd.data(), sdb, hipMemcpyHostToDevice), "upload steps");
  if (st == FFA_OK && !p->wtab.empty())
    st = check_hip(hipMemcpy(t.widths, p->wtab.data(), p->wtab.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice), "upload widths");
  if (st == FFA_OK && !p->sqrtw.empty())
    st = check_hip(hipMemcpy(t.sqrtw, p->sqrtw.data(), p->sqrtw.size() * sizeof(double),
                             hipMemcpyHostToDevice), "upload sqrt widths");
  if (st == FFA_OK) st = upload_dered(p->dered, &t.dered_segs, &t.dered_block_seg);
  if (st != FFA_OK) {
    free_all();
    return st;
  }
  p->dev.push_back(t);
  *out = &p->dev.back();
  return FFA_OK;
}

}  // namespace ffa

using namespace ffa;

extern "C" ffa_status ffa_plan_create(const ffa_plan_desc* d, ffa_plan* out) {
  return ffa_plan_create_opts(d, nullptr, out);
}

extern "C" ffa_status ffa_plan_create_opts(const ffa_plan_desc* d, const ffa_plan_opts* opts_in, ffa_plan* out) {
  if (!d || !out) return fail(FFA_ERR_INVALID, "null argument");
  *out = nullptr;
  if (d->N < 2) return fail(FFA_ERR_INVALID, "N must be >= 2");
  if (!(d->tsamp_s > 0) || !std::isfinite(d->tsamp_s)) return fail(FFA_ERR_INVALID, "tsamp must be > 0");
  if (!(d->pmin_s > 0) || !(d->pmax_s > d->pmin_s) || !std::isfinite(d->pmax_s))
    return fail(FFA_ERR_INVALID, "need 0 < pmin < pmax");
  if (d->bins_min < 2 || d->bins_min > kMaxBinsMin)
    return fail(FFA_ERR_INVALID, "bins_min must be in [2, 1024]");
  if (d->dtype != FFA_IN_F32 && d->dtype != FFA_IN_U8) return fail(FFA_ERR_INVALID, "bad dtype");
  if (d->snr != FFA_SNR_ALG1_MAD && d->snr != FFA_SNR_ALG2_OFFPULSE)
    return fail(FFA_ERR_INVALID, "bad snr algorithm");
  if (d->n_widths < 0 || d->n_widths > kMaxWidths) return fail(FFA_ERR_INVALID, "n_widths must be in [0, 32]");
  if (d->n_widths > 0 && !d->widths) return fail(FFA_ERR_INVALID, "widths is NULL");
  if (d->max_octaves < 0) return fail(FFA_ERR_INVALID, "max_octaves must be >= 0");
  for (int i = 0; i < d->n_widths; ++i)
    if (d->widths[i] < 1) return fail(FFA_ERR_INVALID, "widths must be >= 1");
  if (d->dered_window < -1) return fail(FFA_ERR_INVALID, "dered_window must be -1, 0 or > 0");
  if (d->dered_stride < 0) return fail(FFA_ERR_INVALID, "dered_stride must be >= 0");
  if (d->dtype == FFA_IN_U8 && d->dered_window == 0 && 255.0 * (double)d->N >= 2147483648.0)
    return fail(FFA_ERR_UNSUPPORTED, "uint8 series longer than (2^31-1)/255 samples");
  ffa_plan_opts opts{};
  if (opts_in) opts = *opts_in;
  if (opts.tile_lds_bytes != 0 && (opts.tile_lds_bytes < 16384 || opts.tile_lds_bytes > (int32_t)kLdsBytes))
    return fail(FFA_ERR_INVALID, "tile_lds_bytes must be 0 or in [16384, 163840]");
  if (opts.window_tiles < 0 || opts.window_tiles > (1 << 24))
    return fail(FFA_ERR_INVALID, "window_tiles must be in [0, 2^24]");
  if (opts.ring_mb < 0 || opts.ring_mb > (1 << 20)) return fail(FFA_ERR_INVALID, "ring_mb must be in [0, 2^20]");
  if (opts.steps_per_window < 0 || opts.steps_per_window > 4096)
    return fail(FFA_ERR_INVALID, "steps_per_window must be in [0, 4096]");
  if ((opts.no_u16 != 0 && opts.no_u16 != 1) || (opts.no_split_occupancy != 0 && opts.no_split_occupancy != 1))
    return fail(FFA_ERR_INVALID, "no_u16 and no_split_occupancy must be 0 or 1");
  if (opts.select_cand < 0 || opts.select_cand > 64) return fail(FFA_ERR_INVALID, "select_cand must be in [0, 64]");

  ffa_plan_s* p = new (std::nothrow) ffa_plan_s();
  if (!p) return fail(FFA_ERR_NOMEM, "plan allocation");
  static std::atomic<uint64_t> next_uid{1};
  p->uid = next_uid.fetch_add(1);
  p->desc = *d;
  p->user_widths.assign(d->widths, d->widths + d->n_widths);
  p->desc.widths = nullptr;

  // LDS per tile: the whole workgroup LDS by default; a smaller budget gives
  // smaller tiles (more passes) at higher occupancy.
  const int64_t lds_budget = opts.tile_lds_bytes ? (int64_t)opts.tile_lds_bytes : (int64_t)kLdsBytes;
  // 16-bit first passes (uint8 input without dereddening): see below
  const bool int_mode = d->dtype == FFA_IN_U8 && d->dered_window == 0;
  const bool allow_u16 = int_mode && !opts.no_u16;

  // --- steps (octave f = 2^o; P0 in [B, 2B) with pmin <= P0*f*tsamp < pmax)
  const int64_t B = d->bins_min;
  std::vector<int32_t> wl;
  int64_t trials = 0;
  int32_t max_oct = -1;
  for (int32_t o = 0; o < 62; ++o) {
    if (d->max_octaves > 0 && o >= d->max_octaves) break;
    const int64_t f = int64_t(1) << o;
    if ((double)B * (double)f * d->tsamp_s >= d->pmax_s) break;
    const int64_t Nf = d->N / f;
    if (Nf < 2 * B) break;
    for (int64_t P0 = B; P0 < 2 * B; ++P0) {
      const double per = (double)P0 * (double)f * d->tsamp_s;
      if (per < d->pmin_s || per >= d->pmax_s) continue;
      const int64_t m = Nf / P0;
      if (m < 2) continue;
      if (m > (int64_t(1) << 30)) {
        delete p;
        return fail(FFA_ERR_UNSUPPORTED, "too many rows in one step");
      }
      Step s{};
      s.f = (int32_t)f;
      s.octave = o;
      s.P0 = (int32_t)P0;
      s.m = (int32_t)m;
      s.M = next_pow2(m);
      s.L = ilog2(s.M);
      s.first_trial = trials;
      step_widths(p->user_widths, s.P0, &wl);
      if (wl.empty()) {
        delete p;
        return fail(FFA_ERR_INVALID, "a step has no width <= P0");
      }
      s.wofs = (int32_t)p->wtab.size();
      s.nw = (int32_t)wl.size();
      s.wmax = *std::max_element(wl.begin(), wl.end());
      for (int32_t w : wl) {
        p->wtab.push_back(w);
        p->sqrtw.push_back(std::sqrt((double)w));
      }
      split_passes(&s, lds_budget);
      // A two-pass step whose last pass needs more than half the CU's LDS
      // runs one workgroup per CU there.  For uint8 input the first pass can
      // hold its sums in 16 bits while 255 * 2^(octave + depth) < 2^16; the
      // half-size rows let it take more levels, and the last pass fewer, so
      // that two scoring workgroups share a CU (profiles of up to 512 bins,
      // whose kernel holds 8 waves per SIMD).
      if (allow_u16 && s.n_passes == 2 && s.P0 <= 512 && lds_of(s, s.depth[1], true) > (int64_t)kLdsBytes / 2) {
        for (int32_t dl = s.depth[1] - 1; dl >= 1; --dl) {
          const int32_t d0 = s.L - dl;
          if (o + d0 > 8) break;
          if (lds_of(s, dl, true) <= (int64_t)kLdsBytes / 2 && lds_of(s, d0, false, 2) <= lds_budget) {
            s.depth[0] = d0;
            s.depth[1] = dl;
            s.u16_first = 1;
            break;
          }
        }
      }
      // Likewise a first pass that needs more than half the LDS in 32 bits
      // but not in 16 runs two workgroups per CU with 16-bit rows.
      if (allow_u16 && s.n_passes == 2 && !s.u16_first && s.P0 <= 512 && o + s.depth[0] <= 8 &&
          lds_of(s, s.depth[0], false) > (int64_t)kLdsBytes / 2 &&
          lds_of(s, s.depth[0], false, 2) <= std::min<int64_t>((int64_t)kLdsBytes / 2, lds_budget))
        s.u16_first = 1;
      if (s.n_passes > kMaxPasses) {
        delete p;
        return fail(FFA_ERR_UNSUPPORTED, "step needs too many passes");
      }
      trials += s.M;
      max_oct = std::max(max_oct, o);
      p->steps.push_back(s);
    }
  }
  if (p->steps.empty()) {
    delete p;
    return fail(FFA_ERR_INVALID, "the period range holds no step");
  }
  p->n_trials = trials;
  // 1/sqrt(width) after the sqrt(width) values (used to rank widths)
  const int32_t nsq = (int32_t)p->sqrtw.size();
  for (int32_t i = 0; i < nsq; ++i) p->sqrtw.push_back(1.0 / p->sqrtw[i]);

  // --- dereddening (Sec. 2.3.1): window in samples of every octave series
  if (d->dered_window != 0) {
    double w = d->dered_window > 0 ? (double)d->dered_window
                                   : std::min(2.0 * d->pmax_s / d->tsamp_s, 4.0 * d->pmin_s / d->tsamp_s);
    w = std::max(1.0, std::min(w, 2147483647.0));
    p->dered_W = (int32_t)std::llround(w);
    p->dered_stride = d->dered_stride > 1 ? d->dered_stride : 1;  // 0 or 1: the exact running median
  }
  p->acc_int = d->dtype == FFA_IN_U8 && p->dered_W == 0;
  p->dered_oct0 = p->steps.front().octave;

  // --- series region: header | octave series | knot medians
  p->hdr_elems = 2112;  // 1024 partial sums (double) + centring constant, 8448 B
  p->n_octaves = max_oct + 1;
  int64_t cur = p->hdr_elems;
  for (int32_t o = 0; o < p->n_octaves; ++o) {
    p->oct_off.push_back(cur);
    p->oct_len.push_back(d->N >> o);
    cur = round_up(cur + (d->N >> o), 64);
  }
  p->knots_off = cur;
  if (p->dered_W > 0) cur = round_up(cur + 2 * ((d->N - 1) / p->dered_stride + 1), 64);
  if (p->dered_W > 0 && d->dtype == FFA_IN_F32) {
    // float input: raw octave series in double, dereddened into the float ones
    for (int32_t o = 0; o < p->n_octaves; ++o) {
      p->raw_off.push_back(cur);
      cur = round_up(cur + 2 * (d->N >> o), 64);
    }
    // the exact filter runs every used octave in one plan of launches
    if (p->dered_stride == 1) {
      for (int32_t o = p->dered_oct0; o < p->n_octaves; ++o)
        if (p->oct_len[(size_t)o] > 0)
          p->dered.segs.push_back(DeredSeg{p->raw_off[(size_t)o], p->oct_off[(size_t)o], p->oct_len[(size_t)o], 0,
                                           p->dered_W, 0});
      plan_dered(p->dered);
    }
  }
  p->series_elems = cur;

  // --- phases: one per (step, pass), tiles Q * ng
  for (Step& s : p->steps) {
    s.oct_off = p->oct_off[(size_t)s.octave];
    s.in_end = s.oct_off + p->oct_len[(size_t)s.octave];
  }
  std::vector<Phase>& nat = p->nat_phases;  // natural order: step, then pass
  for (int32_t si = 0; si < (int32_t)p->steps.size(); ++si) {
    Step& s = p->steps[si];
    int32_t D = 0;
    s.total_tiles = 0;
    s.lds_bytes = 0;
    s.fold_phase0 = (int32_t)nat.size();
    for (int32_t pass = 0; pass < s.n_passes; ++pass) {
      const int32_t dp = s.depth[pass];
      const bool last = pass == s.n_passes - 1;
      const int64_t vin = ((int64_t)s.m + (int64_t(1) << D) - 1) >> D;
      const int64_t ng = (vin + (int64_t(1) << dp) - 1) >> dp;
      const int64_t nt = (int64_t(1) << D) * ng;
      if (nt > (int64_t(1) << 30)) {
        delete p;
        return fail(FFA_ERR_UNSUPPORTED, "step too large");
      }
      Phase ph{};
      ph.oct_off = s.oct_off;
      ph.first_trial = s.first_trial;
      ph.ntiles = (int32_t)nt;
      ph.ng = (int32_t)ng;
      ph.step = si;
      ph.pass = pass;
      ph.last = last ? 1 : 0;
      ph.P0 = s.P0;
      ph.M = s.M;
      ph.depth = dp;
      ph.D = D;
      ph.vin = (int32_t)vin;
      ph.u16 = pass == 0 && s.u16_first ? 1 : 0;
      ph.stride = stride_of(s, dp, last, esz_of(ph));
      ph.halo = halo_of(s.P0, dp);
      ph.wofs = s.wofs;
      ph.nw = s.nw;
      ph.isqrt_ofs = nsq + s.wofs;
      ph.series = 0;
      s.tiles[pass] = (int32_t)nt;
      s.total_tiles += (int32_t)nt;
      s.lds_bytes = std::max<int32_t>(s.lds_bytes, (int32_t)phase_lds(ph));
      nat.push_back(ph);
      D += dp;
    }
  }
  p->knobs.window_tiles = opts.window_tiles ? opts.window_tiles : 32768;
  p->knobs.ring_bytes = (opts.ring_mb ? (int64_t)opts.ring_mb : 4096) << 20;
  p->knobs.fixed_steps = opts.steps_per_window;
  p->knobs.split_occupancy = !opts.no_split_occupancy;
  {
    Queue q;
    const ffa_status qs = build_queue(p->steps, nat, p->knobs, &q);
    if (qs != FFA_OK) {
      delete p;
      return qs;
    }
    if (!queue_valid(p->steps, q, p->acc_int)) {
      delete p;
      return fail(FFA_ERR_INVALID, "internal planning error: a tile reaches outside its buffers");
    }
    p->phases = std::move(q.phases);
    p->tile_phase = std::move(q.tile_phase);
    p->launches = std::move(q.launches);
    p->n_tiles = q.n_tiles;
    p->ring_elems = q.ring_elems;
    p->max_passes = q.max_passes;
    p->lookahead = q.lookahead;
    p->lds_bytes = q.lds_bytes;
    p->max_P0 = q.max_P0;
  }
  // fold order: each step's passes in order, tiles counted from the step's start
  for (const Step& s : p->steps) {
    int64_t f0 = 0;
    for (int32_t pass = 0; pass < s.n_passes; ++pass) {
      Phase ph = nat[(size_t)(s.fold_phase0 + pass)];
      ph.tile0 = f0;
      ph.launch = pass;
      f0 += ph.ntiles;
      p->fold_phases.push_back(ph);
    }
  }
  // workspace: series region, then the ring (which ffa_sift reuses as scratch)
  p->ring_off = round_up(p->series_elems, 64);
  {
    const int64_t nb = (p->n_trials + kSiftBlock - 1) / kSiftBlock;
    p->sift_elems = round_up(2 * p->n_trials, 64) + 2 * round_up(nb + 1, 64) + 64 + 8 * (int64_t)kSiftMaxPeaks;
  }
  p->ws_bytes = (size_t)round_up(
      std::max<int64_t>(p->ring_off + p->ring_elems, p->ring_off + p->sift_elems) * 4,
      (int64_t)kWsAlign);
  // the selection's exits (tests force its fallback paths)
  p->select_iters = opts.select_iters == 0 ? 64 : std::max(0, opts.select_iters);
  p->select_cand = opts.select_cand == 0 ? 64 : opts.select_cand;
  *out = p;
  return FFA_OK;
}

extern "C" ffa_status ffa_plan_upload(ffa_plan p) {
  if (!p) return fail(FFA_ERR_INVALID, "null plan");
  const DeviceTables* dt = nullptr;
  return device_tables(p, &dt);
}

extern "C" ffa_status ffa_plan_destroy(ffa_plan p) {
  if (!p) return fail(FFA_ERR_INVALID, "null plan");
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (auto& t : p->dev) {
    if (t.device != cur) (void)hipSetDevice(t.device);
    (void)hipFree(t.phases);
    (void)hipFree(t.fold_phases);
    (void)hipFree(t.tile_phase);
    (void)hipFree(t.steps);
    (void)hipFree(t.widths);
    (void)hipFree(t.sqrtw);
    if (t.dered_segs) (void)hipFree(t.dered_segs);
    if (t.dered_block_seg) (void)hipFree(t.dered_block_seg);
    if (t.device != cur && cur >= 0) (void)hipSetDevice(cur);
  }
  delete p;
  return FFA_OK;
}

extern "C" ffa_status ffa_plan_query(ffa_plan p, int64_t* n_trials, int32_t* n_steps,
                                     size_t* ws_bytes) {
  if (!p) return fail(FFA_ERR_INVALID, "null plan");
  if (n_trials) *n_trials = p->n_trials;
  if (n_steps) *n_steps = (int32_t)p->steps.size();
  if (ws_bytes) *ws_bytes = p->ws_bytes;
  return FFA_OK;
}

extern "C" ffa_status ffa_plan_step(ffa_plan p, int32_t s, int32_t* f, int32_t* P0, int32_t* m,
                                    int32_t* M, int64_t* first_trial) {
  if (!p) return fail(FFA_ERR_INVALID, "null plan");
  if (s < 0 || s >= (int32_t)p->steps.size()) return fail(FFA_ERR_INVALID, "step out of range");
  const Step& st = p->steps[s];
  if (f) *f = st.f;
  if (P0) *P0 = st.P0;
  if (m) *m = st.m;
  if (M) *M = st.M;
  if (first_trial) *first_trial = st.first_trial;
  return FFA_OK;
}

extern "C" ffa_status ffa_plan_passes(ffa_plan p, int32_t s, int32_t* n_passes, int32_t* depths) {
  if (!p) return fail(FFA_ERR_INVALID, "null plan");
  if (s < 0 || s >= (int32_t)p->steps.size()) return fail(FFA_ERR_INVALID, "step out of range");
  const Step& st = p->steps[s];
  if (n_passes) *n_passes = st.n_passes;
  if (depths)
    for (int32_t i = 0; i < st.n_passes; ++i) depths[i] = st.depth[i];
  return FFA_OK;
}

extern "C" ffa_status ffa_plan_periods(ffa_plan p, double* out) {
  if (!p || !out) return fail(FFA_ERR_INVALID, "null argument");
  for (const Step& s : p->steps) {
    const double scale = (double)s.f * p->desc.tsamp_s;
    for (int32_t k = 0; k < s.M; ++k)
      out[s.first_trial + k] = scale * ((double)s.P0 + (double)k / (double)(s.M - 1));
  }
  return FFA_OK;
}

// Test hook (not in the public header): the plan's dereddening plan.  Writes
// 6 values per segment (x_off, out_off, n, block0, window, use_stage), then
// 3 per launch (block0, blocks, lds); returns the segment count (launch count
// in *n_launches), -1 for a null plan.  Nothing is written when cap is short.
extern "C" int64_t ffa_debug_dered(ffa_plan p, int64_t* out, int64_t cap, int64_t* n_launches) {
  if (!p) return -1;
  const DeredPlan& dp = p->dered;
  const int64_t ns = (int64_t)dp.segs.size(), nl = (int64_t)dp.launches.size();
  if (n_launches) *n_launches = nl;
  if (!out || cap < 6 * ns + 3 * nl) return ns;
  for (const DeredSeg& g : dp.segs) {
    *out++ = g.x_off;
    *out++ = g.out_off;
    *out++ = g.n;
    *out++ = g.block0;
    *out++ = g.window;
    *out++ = g.use_stage;
  }
  for (const DeredLaunch& L : dp.launches) {
    *out++ = L.block0;
    *out++ = L.blocks;
    *out++ = L.lds;
  }
  return ns;
}

// Test hooks (not in the public header): the plan's queue-ordered phases and
// its workspace layout and launches, so host tests can check the kernel's
// index arithmetic against the buffers without a GPU.
extern "C" int64_t ffa_debug_phases(ffa_plan p, void* out, int64_t cap) {
  if (!p) return -1;
  const int64_t n = (int64_t)p->phases.size();
  if (out && cap >= n) std::memcpy(out, p->phases.data(), (size_t)n * sizeof(Phase));
  return n;
}

extern "C" int64_t ffa_debug_layout(ffa_plan p, int64_t* out, int64_t cap) {
  if (!p) return -1;
  const int64_t nw = (int64_t)p->launches.size();
  const int64_t need = 8 + 4 * nw;
  if (!out || cap < need) return need;
  out[0] = p->ring_off;
  out[1] = p->ring_elems;
  out[2] = 0;
  out[3] = p->n_tiles;
  out[4] = p->lds_bytes;
  out[5] = p->max_P0;
  out[6] = (int64_t)p->ws_bytes;
  out[7] = p->lookahead;
  for (int64_t i = 0; i < nw; ++i) {
    const Launch& w = p->launches[(size_t)i];
    out[8 + 4 * i] = w.tile0;
    out[9 + 4 * i] = w.ntiles;
    out[10 + 4 * i] = w.lds_bytes;
    out[11 + 4 * i] = w.max_P0;
  }
  return need;
}
