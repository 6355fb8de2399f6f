// Search planning: steps, pass split, work tiles, workspace layout.
//
// A plan is built on the host only; its device tables are uploaded on first
// use on a GPU (device_tables), so plans can be made and inspected without a
// GPU.
#include <algorithm>
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
int32_t halo_of(int32_t P0, int32_t d) { return std::min<int32_t>(int32_t(1) << (d - 1), P0); }
constexpr int32_t kMaxHalo = 1 << 30;  // no limit on the halo
int32_t stride_of(const Step& s, int32_t d, bool last) {
  const int32_t h = halo_of(s.P0, d);
  return s.P0 + std::max<int32_t>(h, last ? s.wmax + 1 : 0);
}
int64_t lds_of(const Step& s, int32_t d, bool last) {
  return (int64_t(1) << d) * stride_of(s, d, last) * 4 + (last ? (int64_t)kScratchBytes : 0);
}

void split_passes(Step* s) {
  int32_t dfin = 1, dmid = 1;
  auto fits = [&](int32_t d, bool last) {
    return lds_of(*s, d, last) <= (int64_t)kLdsBytes && (halo_of(s->P0, d) <= kMaxHalo || s->P0 <= kMaxHalo);
  };
  while (dfin < 24 && fits(dfin + 1, true)) ++dfin;
  while (dmid < 24 && fits(dmid + 1, false)) ++dmid;
  if (s->L <= dfin) {
    s->n_passes = 1;
    s->depth[0] = s->L;
    return;
  }
  const int32_t rest = s->L - dfin;
  const int32_t np = (rest + dmid - 1) / dmid;
  for (int32_t i = 0; i < np; ++i) s->depth[i] = rest / np + (i < rest % np ? 1 : 0);
  s->depth[np] = dfin;
  s->n_passes = np + 1;
}

size_t chunk_budget_elems() {
  int64_t mb = 128;
  if (const char* e = std::getenv("FFA_CHUNK_MB")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v > 0 && v < (1 << 20)) mb = v;
  }
  return (size_t)mb * 1024 * 1024 / 4;
}

// Every tile's reads and writes must stay inside the buffers of its step:
// the octave series (first pass), the step's intermediate buffers, its own
// trial range, and the LDS of one workgroup.  Checked once per plan, before
// anything can be launched.
bool tiles_in_bounds(const ffa_plan_s* p) {
  const int64_t inter_end = p->inter_off + p->inter_elems;
  for (const Step& s : p->steps) {
    const int64_t MP = (int64_t)s.M * s.P0;
    if (s.n_passes >= 2 && (s.buf_off[0] < p->inter_off || s.buf_off[0] + MP > inter_end)) return false;
    if (s.n_passes >= 3 && (s.buf_off[1] < s.buf_off[0] + MP || s.buf_off[1] + MP > inter_end)) return false;
    int32_t D = 0;
    for (int32_t pass = 0; pass < s.n_passes; ++pass) {
      const int32_t dp = s.depth[pass];
      const bool last = pass == s.n_passes - 1;
      if (dp < 1 || dp > 24) return false;
      for (int64_t ti = s.tile_begin[pass]; ti < s.tile_end[pass]; ++ti) {
        const Tile& t = p->tiles[ti];
        const int64_t rows = int64_t(1) << dp;
        if (t.P0 != s.P0 || t.depth != dp || t.valid < 1 || t.valid > rows) return false;
        if (t.halo < 1 || t.halo > s.P0 || t.halo < std::min<int64_t>(rows / 2, s.P0)) return false;
        if (t.halo > kMaxHalo && s.P0 > kMaxHalo) return false;
        if (t.stride < s.P0 + t.halo || t.stride < s.P0 + (last ? s.wmax + 1 : 0)) return false;
        if (rows * t.stride * 4 + (last ? (int64_t)kScratchBytes : 0) > (int64_t)kLdsBytes) return false;
        if (t.nw != s.nw || t.wofs != s.wofs) return false;
        int64_t lo, hi;
        if (pass == 0) {
          lo = p->oct_off[s.octave];
          hi = lo + (int64_t)s.m * s.P0;
        } else {
          lo = s.buf_off[(pass - 1) % 2];
          hi = lo + MP;
        }
        if (t.src < lo || t.src + (int64_t)t.valid * s.P0 > hi) return false;
        if (!last) {
          const int64_t b = s.buf_off[pass % 2];
          if (t.final_ || t.dst < b || t.dst + (rows - 1) * (int64_t)t.dst_step + s.P0 > b + MP) return false;
          if (t.dst_step < s.P0) return false;
        } else {
          if (!t.final_ || t.dst < s.first_trial || t.dst + rows > s.first_trial + s.M) return false;
        }
      }
      D += dp;
    }
    if (D != s.L) return false;
  }
  return true;
}

}  // namespace

ffa_status fail(ffa_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ffa_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return FFA_OK;
  return fail(FFA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error_cstr() { return g_last_error.c_str(); }

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
  const size_t tb = p->tiles.size() * sizeof(Tile);
  const size_t wb = std::max<size_t>(p->wtab.size(), 1) * sizeof(int32_t);
  const size_t sb = std::max<size_t>(p->sqrtw.size(), 1) * sizeof(double);
  if (hipMalloc(&t.tiles, std::max<size_t>(tb, 64)) != hipSuccess ||
      hipMalloc(&t.widths, wb) != hipSuccess || hipMalloc(&t.sqrtw, sb) != hipSuccess) {
    if (t.tiles) (void)hipFree(t.tiles);
    if (t.widths) (void)hipFree(t.widths);
    if (t.sqrtw) (void)hipFree(t.sqrtw);
    return fail(FFA_ERR_NOMEM, "device tables: hipMalloc failed");
  }
  ffa_status st = FFA_OK;
  if (tb) st = check_hip(hipMemcpy(t.tiles, p->tiles.data(), tb, hipMemcpyHostToDevice), "upload tiles");
  if (st == FFA_OK && !p->wtab.empty())
    st = check_hip(hipMemcpy(t.widths, p->wtab.data(), p->wtab.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice), "upload widths");
  if (st == FFA_OK && !p->sqrtw.empty())
    st = check_hip(hipMemcpy(t.sqrtw, p->sqrtw.data(), p->sqrtw.size() * sizeof(double),
                             hipMemcpyHostToDevice), "upload sqrt widths");
  if (st != FFA_OK) {
    (void)hipFree(t.tiles);
    (void)hipFree(t.widths);
    (void)hipFree(t.sqrtw);
    return st;
  }
  p->dev.push_back(t);
  *out = &p->dev.back();
  return FFA_OK;
}

}  // namespace ffa

using namespace ffa;

extern "C" ffa_status ffa_plan_create(const ffa_plan_desc* d, ffa_plan* out) {
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
  if (d->snr == FFA_SNR_ALG2_OFFPULSE) return fail(FFA_ERR_UNSUPPORTED, "Algorithm 2 not built");
  if (d->n_widths < 0 || d->n_widths > kMaxWidths) return fail(FFA_ERR_INVALID, "n_widths must be in [0, 32]");
  if (d->n_widths > 0 && !d->widths) return fail(FFA_ERR_INVALID, "widths is NULL");
  if (d->max_octaves < 0) return fail(FFA_ERR_INVALID, "max_octaves must be >= 0");
  for (int i = 0; i < d->n_widths; ++i)
    if (d->widths[i] < 1) return fail(FFA_ERR_INVALID, "widths must be >= 1");
  if (d->dtype == FFA_IN_U8 && 255.0 * (double)d->N >= 2147483648.0)
    return fail(FFA_ERR_UNSUPPORTED, "uint8 series longer than (2^31-1)/255 samples");

  ffa_plan_s* p = new (std::nothrow) ffa_plan_s();
  if (!p) return fail(FFA_ERR_NOMEM, "plan allocation");
  p->desc = *d;
  p->user_widths.assign(d->widths, d->widths + d->n_widths);
  p->desc.widths = nullptr;

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
      split_passes(&s);
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

  // --- workspace: header | octave series | intermediate region
  p->hdr_elems = 2112;  // 1024 partial sums (double) + centring constant, 8448 B
  p->n_octaves = max_oct + 1;
  int64_t cur = p->hdr_elems;
  for (int32_t o = 0; o < p->n_octaves; ++o) {
    p->oct_off.push_back(cur);
    p->oct_len.push_back(d->N >> o);
    cur = round_up(cur + (d->N >> o), 64);
  }
  p->inter_off = cur;

  // --- chunks of steps whose intermediates fit the budget together
  int64_t max_need = 0;
  for (auto& s : p->steps) {
    const int64_t need = (int64_t)(s.n_passes >= 2 ? 1 : 0) * s.M * s.P0 +
                         (int64_t)(s.n_passes >= 3 ? 1 : 0) * s.M * s.P0;
    max_need = std::max(max_need, round_up(need, 64) + 128);
  }
  const int64_t budget = std::max<int64_t>((int64_t)chunk_budget_elems(), max_need);
  {
    Chunk c{};
    c.step_begin = 0;
    int64_t used = 0;
    for (int32_t si = 0; si < (int32_t)p->steps.size(); ++si) {
      Step& s = p->steps[si];
      const int64_t a = s.n_passes >= 2 ? round_up((int64_t)s.M * s.P0, 64) : 0;
      const int64_t b = s.n_passes >= 3 ? round_up((int64_t)s.M * s.P0, 64) : 0;
      if (used + a + b > budget && si > c.step_begin) {
        c.step_end = si;
        p->chunks.push_back(c);
        c = Chunk{};
        c.step_begin = si;
        used = 0;
      }
      s.buf_off[0] = p->inter_off + used;
      s.buf_off[1] = p->inter_off + used + a;
      used += a + b;
      s.chunk = (int32_t)p->chunks.size();
      p->inter_elems = std::max(p->inter_elems, used);
    }
    c.step_end = (int32_t)p->steps.size();
    p->chunks.push_back(c);
  }

  // --- tiles: chunk, then pass, then step, then problem q, then group h
  for (auto& c : p->chunks) {
    c.n_passes = 0;
    c.max_P0 = 0;
    for (int32_t si = c.step_begin; si < c.step_end; ++si) {
      c.n_passes = std::max(c.n_passes, p->steps[si].n_passes);
      c.max_P0 = std::max(c.max_P0, p->steps[si].P0);
    }
    for (int32_t pass = 0; pass < c.n_passes; ++pass) {
      c.tile_begin[pass] = (int64_t)p->tiles.size();
      c.lds_bytes[pass] = 0;
      for (int32_t si = c.step_begin; si < c.step_end; ++si) {
        Step& s = p->steps[si];
        if (pass >= s.n_passes) continue;
        s.tile_begin[pass] = (int64_t)p->tiles.size();
        int32_t D = 0;
        for (int32_t i = 0; i < pass; ++i) D += s.depth[i];
        const int32_t dp = s.depth[pass];
        const int64_t Q = int64_t(1) << D;
        const int64_t Gin = (int64_t)s.M >> D;
        const int64_t vin = ((int64_t)s.m + (int64_t(1) << D) - 1) >> D;
        const int64_t ng = (vin + (int64_t(1) << dp) - 1) >> dp;
        const bool last = pass == s.n_passes - 1;
        const int64_t src_base = pass == 0 ? p->oct_off[s.octave] : s.buf_off[(pass - 1) % 2];
        const int32_t stride = stride_of(s, dp, last);
        s.lds_bytes[pass] = (int32_t)lds_of(s, dp, last);
        c.lds_bytes[pass] = std::max(c.lds_bytes[pass], s.lds_bytes[pass]);
        for (int64_t q = 0; q < Q; ++q) {
          for (int64_t h = 0; h < ng; ++h) {
            Tile t{};
            t.P0 = s.P0;
            t.depth = dp;
            t.src = src_base + (q * Gin + (h << dp)) * s.P0;
            t.valid = (int32_t)std::min<int64_t>(int64_t(1) << dp, vin - (h << dp));
            t.stride = stride;
            t.halo = halo_of(s.P0, dp);
            t.wofs = s.wofs;
            t.nw = s.nw;
            t.step = si;
            if (!last) {
              const int64_t Gout = Gin >> dp;
              t.dst = s.buf_off[pass % 2] + ((q << dp) * Gout + h) * s.P0;
              t.dst_step = (int32_t)(Gout * s.P0);
              t.h = (int32_t)h;
              t.final_ = 0;
            } else {
              t.dst = s.first_trial + (q << dp);
              t.final_ = 1;
            }
            p->tiles.push_back(t);
          }
        }
        s.tile_end[pass] = (int64_t)p->tiles.size();
      }
      c.tile_end[pass] = (int64_t)p->tiles.size();
    }
  }
  p->ws_bytes = (size_t)round_up((p->inter_off + p->inter_elems) * 4, (int64_t)kWsAlign);
  // test knobs: force the selection's fallback paths
  if (const char* e = std::getenv("FFA_SELECT_ITERS")) p->select_iters = std::max(0, std::atoi(e));
  if (const char* e = std::getenv("FFA_SELECT_CAND")) p->select_cand = std::min(64, std::max(1, std::atoi(e)));
  if (!tiles_in_bounds(p)) {
    delete p;
    return fail(FFA_ERR_INVALID, "internal planning error: a tile reaches outside its buffers");
  }
  *out = p;
  return FFA_OK;
}

extern "C" ffa_status ffa_plan_destroy(ffa_plan p) {
  if (!p) return fail(FFA_ERR_INVALID, "null plan");
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (auto& t : p->dev) {
    if (t.device != cur) (void)hipSetDevice(t.device);
    (void)hipFree(t.tiles);
    (void)hipFree(t.widths);
    (void)hipFree(t.sqrtw);
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
