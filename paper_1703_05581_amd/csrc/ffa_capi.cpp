// C ABI entry points that enqueue GPU work: search, fold, best.
#include <cstdint>

#include "ffa_internal.h"

namespace ffa {
const char* last_error_cstr();
}

using namespace ffa;

namespace {

ffa_status check_ws(ffa_plan p, const void* ws, size_t ws_bytes) {
  if (!ws) return fail(FFA_ERR_INVALID, "null workspace");
  if (ws_bytes < p->ws_bytes) return fail(FFA_ERR_INVALID, "workspace smaller than ffa_plan_query's ws_bytes");
  if (reinterpret_cast<uintptr_t>(ws) % kWsAlign) return fail(FFA_ERR_INVALID, "workspace not 256-byte aligned");
  return FFA_OK;
}

// Octave series 0..last_octave into the workspace.  Float input is centred
// on its mean when `center` is set.
ffa_status build_octaves(ffa_plan p, const void* series, void* ws, int32_t last_octave,
                         int center, hipStream_t st) {
  const int is_int = p->desc.dtype == FFA_IN_U8;
  if (!is_int && center) {
    ffa_status s = check_hip(launch_mean(reinterpret_cast<const float*>(series), p->desc.N, ws, st),
                             "mean kernel");
    if (s != FFA_OK) return s;
  }
  ffa_status s = check_hip(launch_prep(series, is_int, p->desc.N, ws, p->oct_off[0], center, st),
                           "prep kernel");
  if (s != FFA_OK) return s;
  for (int32_t o = 1; o <= last_octave; ++o) {
    s = check_hip(launch_halve(ws, is_int, p->oct_off[o - 1], p->oct_len[o], p->oct_off[o], st),
                  "downsample kernel");
    if (s != FFA_OK) return s;
  }
  return FFA_OK;
}

}  // namespace

extern "C" ffa_status ffa_search(ffa_plan p, const void* d_series, float* d_snr, int32_t* d_width,
                                 void* d_ws, size_t ws_bytes, void* stream) {
  if (!p || !d_series || !d_snr || !d_width) return fail(FFA_ERR_INVALID, "null argument");
  ffa_status s = check_ws(p, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const DeviceTables* dt = nullptr;
  s = device_tables(p, &dt);
  if (s != FFA_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int is_int = p->desc.dtype == FFA_IN_U8;
  s = build_octaves(p, d_series, d_ws, p->n_octaves - 1, 1, st);
  if (s != FFA_OK) return s;
  for (const Chunk& c : p->chunks) {
    for (int32_t pass = 0; pass < c.n_passes; ++pass) {
      s = check_hip(launch_pass(dt->tiles + c.tile_begin[pass], c.tile_end[pass] - c.tile_begin[pass],
                                c.lds_bytes[pass], c.max_P0, is_int, d_ws, d_snr, d_width, nullptr, 0,
                                kModeScore, dt->widths, dt->sqrtw, p->select_iters,
                                p->select_cand, st),
                    "FFA pass kernel");
      if (s != FFA_OK) return s;
    }
  }
  return FFA_OK;
}

extern "C" ffa_status ffa_fold(ffa_plan p, const void* d_series, int32_t step, void* d_profiles,
                               void* d_ws, size_t ws_bytes, void* stream) {
  if (!p || !d_series || !d_profiles) return fail(FFA_ERR_INVALID, "null argument");
  if (step < 0 || step >= (int32_t)p->steps.size()) return fail(FFA_ERR_INVALID, "step out of range");
  ffa_status s = check_ws(p, d_ws, ws_bytes);
  if (s != FFA_OK) return s;
  const DeviceTables* dt = nullptr;
  s = device_tables(p, &dt);
  if (s != FFA_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int is_int = p->desc.dtype == FFA_IN_U8;
  const Step& sp = p->steps[step];
  s = build_octaves(p, d_series, d_ws, sp.octave, 0, st);
  if (s != FFA_OK) return s;
  for (int32_t pass = 0; pass < sp.n_passes; ++pass) {
    s = check_hip(launch_pass(dt->tiles + sp.tile_begin[pass], sp.tile_end[pass] - sp.tile_begin[pass],
                              sp.lds_bytes[pass], sp.P0, is_int, d_ws, nullptr, nullptr, d_profiles,
                              sp.first_trial, kModeProfiles, dt->widths, dt->sqrtw,
                              p->select_iters, p->select_cand, st),
                  "FFA pass kernel");
    if (s != FFA_OK) return s;
  }
  return FFA_OK;
}

extern "C" ffa_status ffa_best(const float* d_snr, int64_t n_trials, int64_t* d_best, void* stream) {
  if (!d_snr || !d_best || n_trials < 1) return fail(FFA_ERR_INVALID, "bad argument");
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
