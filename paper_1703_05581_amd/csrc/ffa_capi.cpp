// C ABI entry points that enqueue GPU work: prepare, search, fold, best.
#include <cmath>
#include <cstdint>

#include "ffa_internal.h"

namespace ffa {
const char* last_error_cstr();
}

using namespace ffa;

namespace {

ffa_status check_ws(size_t need, const void* ws, size_t ws_bytes) {
  if (!ws) return fail(FFA_ERR_INVALID, "null workspace");
  if (ws_bytes < need) return fail(FFA_ERR_INVALID, "workspace smaller than the plan's ws_bytes");
  if (reinterpret_cast<uintptr_t>(ws) % kWsAlign) return fail(FFA_ERR_INVALID, "workspace not 256-byte aligned");
  return FFA_OK;
}

TileArgs base_args(ffa_plan p, const DeviceTables* dt) {
  TileArgs a{};
  a.widths = dt->widths;
  a.sqrtw = dt->sqrtw;
  a.oct_base = 0;
  a.ring_off = p->ring_off;
  a.alg = p->desc.snr == FFA_SNR_ALG2_OFFPULSE ? 2 : 1;
  a.select_iters = p->select_iters;
  a.select_cand = p->select_cand;
  return a;
}

}  // namespace

namespace ffa {

// Octave series 0..last_octave of one series into the series region at the
// start of `ws`.  Float input is centred on its mean when `center`.
ffa_status build_octaves(ffa_plan p, const void* series, void* ws, int32_t last_octave, int center,
                         hipStream_t st, const DeviceTables* dt, bool dered) {
  const int int_sums = p->desc.dtype == FFA_IN_U8;
  ffa_status s = FFA_OK;
  if (p->dered_W > 0 && !int_sums) {
    // float input, dereddened: raw octave series summed in double, then each
    // used octave dereddened into its float32 series (one rounding)
    s = check_hip(launch_prep_f64(reinterpret_cast<const float*>(series), p->desc.N, ws, p->raw_off[0], st),
                  "prep kernel");
    for (int32_t o = 1; o <= last_octave && s == FFA_OK; ++o)
      s = check_hip(launch_halve_f64(ws, p->raw_off[o - 1], p->oct_len[o], p->raw_off[o], st),
                    "downsample kernel");
    if (s != FFA_OK || !dered) return s;
    // the exact filter of every octave at once, from the plan's tables
    if (dt && dt->dered_segs && last_octave == p->n_octaves - 1)
      return run_dered(p->dered, dt->dered_segs, dt->dered_block_seg, ws, st);
    for (int32_t o = p->dered_oct0; o <= last_octave && s == FFA_OK; ++o)
      s = check_hip(launch_deredden(ws, 2, p->raw_off[o], p->oct_len[o], p->dered_W, p->dered_stride,
                                    p->knots_off, p->oct_off[o], st),
                    "dereddening kernels");
    return s;
  }
  // uint8 input is summed exactly in int32; float input is centred on its mean
  if (!int_sums && center) {
    s = check_hip(launch_mean(reinterpret_cast<const float*>(series), p->desc.N, ws, st), "mean kernel");
    if (s != FFA_OK) return s;
  }
  s = check_hip(launch_prep(series, int_sums, p->desc.N, ws, p->oct_off[0], center, st), "prep kernel");
  if (s != FFA_OK) return s;
  for (int32_t o = 1; o <= last_octave; ++o) {
    s = check_hip(launch_halve(ws, int_sums, p->oct_off[o - 1], p->oct_len[o], p->oct_off[o], st),
                  "downsample kernel");
    if (s != FFA_OK) return s;
  }
  // dynamic dereddening (Sec. 2.3.1) of uint8 input: every octave a step
  // folds, each from its exact int32 sums (all halvings are done), same
  // window in its own samples, written over them as float32
  if (p->dered_W > 0) {
    for (int32_t o = p->dered_oct0; o <= last_octave; ++o) {
      s = check_hip(launch_deredden(ws, 0, p->oct_off[o], p->oct_len[o], p->dered_W, p->dered_stride,
                                    p->knots_off, p->oct_off[o], st),
                    "dereddening kernels");
      if (s != FFA_OK) return s;
    }
  }
  return FFA_OK;
}

ffa_status run_launches(ffa_plan p, const DeviceTables* dt, float* snr, int32_t* width, void* ws,
                       hipStream_t st) {
  const int is_int = p->acc_int;
  TileArgs a = base_args(p, dt);
  a.phases = dt->phases;
  a.tile_phase = dt->tile_phase;
  a.snr = snr;
  a.width = width;
  a.mode = kModeScore;
  for (const Launch& w : p->launches) {
    if (w.ntiles == 0) continue;
    a.tile0 = w.tile0;
    ffa_status s = check_hip(launch_tiles(a, w.ntiles, w.lds_bytes, w.max_P0, is_int, ws, st),
                             "FFA kernel");
    if (s != FFA_OK) return s;
  }
  return FFA_OK;
}

}  // namespace ffa

extern "C" ffa_status ffa_prepare(ffa_plan p, const void* d_series, void* d_ws, size_t ws_bytes,
                                  void* stream) {
  if (!p || !d_series) return fail(FFA_ERR_INVALID, "null argument");
  ffa_status s = check_ws(p->ws_bytes, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const DeviceTables* dt = nullptr;
  s = device_tables(p, &dt);
  if (s != FFA_OK) return s;
  return build_octaves(p, d_series, d_ws, p->n_octaves - 1, 1, reinterpret_cast<hipStream_t>(stream), dt);
}

extern "C" ffa_status ffa_search_prepared(ffa_plan p, float* d_snr, int32_t* d_width, void* d_ws,
                                          size_t ws_bytes, void* stream) {
  if (!p || !d_snr || !d_width) return fail(FFA_ERR_INVALID, "null argument");
  ffa_status s = check_ws(p->ws_bytes, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const DeviceTables* dt = nullptr;
  s = device_tables(p, &dt);
  if (s != FFA_OK) return s;
  return run_launches(p, dt, d_snr, d_width, d_ws, reinterpret_cast<hipStream_t>(stream));
}

extern "C" ffa_status ffa_search(ffa_plan p, const void* d_series, float* d_snr, int32_t* d_width,
                                 void* d_ws, size_t ws_bytes, void* stream) {
  if (!p || !d_series || !d_snr || !d_width) return fail(FFA_ERR_INVALID, "null argument");
  ffa_status s = ffa_prepare(p, d_series, d_ws, ws_bytes, stream);
  if (s != FFA_OK) return s;
  return ffa_search_prepared(p, d_snr, d_width, d_ws, ws_bytes, stream);
}

extern "C" ffa_status ffa_fold(ffa_plan p, const void* d_series, int32_t step, void* d_profiles,
                               void* d_ws, size_t ws_bytes, void* stream) {
  if (!p || !d_series || !d_profiles) return fail(FFA_ERR_INVALID, "null argument");
  if (step < 0 || step >= (int32_t)p->steps.size()) return fail(FFA_ERR_INVALID, "step out of range");
  ffa_status s = check_ws(p->ws_bytes, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const DeviceTables* dt = nullptr;
  s = device_tables(p, &dt);
  if (s != FFA_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Step& sp = p->steps[step];
  s = build_octaves(p, d_series, d_ws, sp.octave, 0, st, dt);
  if (s != FFA_OK) return s;
  // the step's passes in order, one launch each
  const int is_int = p->acc_int;
  TileArgs a = base_args(p, dt);
  a.tile_phase = nullptr;
  a.profiles = d_profiles;
  a.trial_base = sp.first_trial;
  a.mode = kModeProfiles;
  for (int32_t pass = 0; pass < sp.n_passes; ++pass) {
    const Phase& ph = p->fold_phases[(size_t)sp.fold_phase0 + pass];
    a.phases = dt->fold_phases + sp.fold_phase0 + pass;
    a.tile0 = ph.tile0;
    // the pass's LDS rows at the element size it was planned with (a 16-bit
    // first pass of a uint8 step keeps 2-byte rows)
    const int64_t esz = ph.u16 ? 2 : 4;
    const int lds = (int)(((int64_t)1 << ph.depth) * ph.stride * esz + (ph.last ? (int64_t)kScratchBytes : 0));
    s = check_hip(launch_tiles(a, ph.ntiles, lds, ph.P0, is_int, d_ws, st), "FFA kernel");
    if (s != FFA_OK) return s;
  }
  return FFA_OK;
}

extern "C" ffa_status ffa_sift(ffa_plan p, const float* d_snr, const int32_t* d_width,
                               const ffa_sift_params* prm, ffa_candidate* d_cands, int32_t max_cands,
                               int32_t* d_n_cands, void* d_ws, size_t ws_bytes, void* stream) {
  if (!p || !d_snr || !d_width || !prm || !d_n_cands || (max_cands > 0 && !d_cands))
    return fail(FFA_ERR_INVALID, "null argument");
  if (max_cands < 0) return fail(FFA_ERR_INVALID, "max_cands must be >= 0");
  if (!std::isfinite(prm->min_snr) || !(prm->frac_fall >= 0.0f && prm->frac_fall <= 1.0f) ||
      !(prm->abs_fall >= 0.0f) || !std::isfinite(prm->abs_fall) || !(prm->group_widths >= 0.0f) ||
      !std::isfinite(prm->group_widths) || prm->harmonic_primes > 1000 || !(prm->harmonic_tol >= 0.0f) ||
      !std::isfinite(prm->harmonic_tol))
    return fail(FFA_ERR_INVALID, "bad sift parameters");
  ffa_status s = check_ws(p->ws_bytes, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const DeviceTables* dt = nullptr;
  s = device_tables(p, &dt);
  if (s != FFA_OK) return s;
  return check_hip(launch_sift(d_snr, d_width, p->n_trials, *prm, dt->steps, (int32_t)p->steps.size(),
                               p->desc.tsamp_s, d_ws, p->ring_off, d_cands, max_cands, d_n_cands,
                               reinterpret_cast<hipStream_t>(stream)),
                   "sift kernels");
}

extern "C" ffa_status ffa_best(const float* d_snr, int64_t n_trials, int64_t* d_best, void* stream) {
  if (!d_snr || !d_best || n_trials < 1) return fail(FFA_ERR_INVALID, "bad argument");
  if (n_trials > 0xffffffffll) return fail(FFA_ERR_INVALID, "n_trials must be below 2^32");
  return check_hip(launch_best(d_snr, n_trials, d_best, reinterpret_cast<hipStream_t>(stream)),
                   "best kernel");
}

extern "C" const char* ffa_status_str(ffa_status st) {
  switch (st) {
    case FFA_OK: return "FFA_OK";
    case FFA_ERR_INVALID: return "FFA_ERR_INVALID";
    case FFA_ERR_NOMEM: return "FFA_ERR_NOMEM";
    case FFA_ERR_DEVICE: return "FFA_ERR_DEVICE";
    case FFA_ERR_UNSUPPORTED: return "FFA_ERR_UNSUPPORTED";
    case FFA_ERR_BUSY: return "FFA_ERR_BUSY";
    case FFA_ERR_TIMEOUT: return "FFA_ERR_TIMEOUT";
  }
  return "FFA_ERR_UNKNOWN";
}

extern "C" const char* ffa_last_error(void) { return last_error_cstr(); }
