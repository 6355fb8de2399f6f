// Internal declarations of the FFA library: plan layout, work tiles and the
// kernel launchers.  Not part of the public ABI (include/ffa.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "ffa.h"

namespace ffa {

constexpr int kMaxWidths = 32;
constexpr int kMaxBinsMin = 1024;      // P0 < 2*B <= 2048
constexpr int kMaxPasses = 8;
constexpr int kThreads = 1024;         // threads per workgroup of the FFA kernels
constexpr size_t kLdsBytes = 160 * 1024;  // gfx950 LDS per workgroup
constexpr size_t kWsAlign = 256;
constexpr size_t kScratchBytes = (kThreads / 64) * 64 * 4;  // per-wave selection scratch

// sigma = K * MAD (paper Sec. 2.2.1): K is 1 / (75% quantile of the unit normal).
constexpr double kMadK = 1.482602218505602;

// Output modes of the last pass of a step.
enum : int32_t { kModeIntermediate = 0, kModeScore = 1, kModeProfiles = 2 };

// One workgroup's work: 2^depth rows of P0 bins (a "group"), all butterfly
// levels of one pass run on chip, then either written back (rotated) for the
// next pass or scored / written as profiles.
struct Tile {
  int64_t src;       // element offset in the workspace of row 0 of the group
  int64_t dst;       // intermediate: element offset of output t = 0
                     // last pass: global trial index of output t = 0
  int32_t P0;
  int32_t depth;     // rows = 1 << depth
  int32_t valid;     // rows >= valid are zero and not read
  int32_t h;         // group index: output t is rotated left by t*h bins
  int32_t dst_step;  // intermediate: elements between outputs t and t+1
  int32_t final_;    // 1 on the last pass of the step
  int32_t wofs;      // offset of the step's widths in the width tables
  int32_t nw;        // number of widths of the step
  int32_t stride;    // LDS row stride in elements
  int32_t step;      // step index (diagnostics)
  int32_t halo;      // LDS bins after P0 that repeat bins 0..halo-1
  int32_t pad_;
};
static_assert(sizeof(Tile) == 64, "tile layout");

struct Step {
  int32_t f, octave, P0, m, M, L;
  int64_t first_trial;
  int32_t n_passes;
  int32_t depth[kMaxPasses];
  int32_t wofs, nw, wmax;
  int32_t chunk;
  // tiles of pass p: [tile_begin[p], tile_end[p]) in Plan::tiles
  int64_t tile_begin[kMaxPasses], tile_end[kMaxPasses];
  int64_t buf_off[2];  // intermediate ping-pong buffers (elements, workspace-relative)
  int32_t lds_bytes[kMaxPasses];
};

struct Chunk {
  int32_t step_begin, step_end;
  int32_t n_passes;  // max over its steps
  int64_t tile_begin[kMaxPasses], tile_end[kMaxPasses];
  int32_t lds_bytes[kMaxPasses];
  int32_t max_P0;
};

// Device copies of a plan's tables (made on first use on a device).
struct DeviceTables {
  int device = -1;
  Tile* tiles = nullptr;
  int32_t* widths = nullptr;
  double* sqrtw = nullptr;
};

}  // namespace ffa

struct ffa_plan_s {
  ffa_plan_desc desc;
  std::vector<int32_t> user_widths;
  std::vector<ffa::Step> steps;
  std::vector<ffa::Chunk> chunks;
  std::vector<ffa::Tile> tiles;
  std::vector<int32_t> wtab;     // widths of every step, concatenated
  std::vector<double> sqrtw;     // sqrt(width), same layout
  int64_t n_trials = 0;
  int32_t n_octaves = 0;         // octaves 0..n_octaves-1 are built
  std::vector<int64_t> oct_off;  // element offset of each octave series
  std::vector<int64_t> oct_len;
  int64_t hdr_elems = 0;         // header (centring scratch) in elements
  int64_t inter_off = 0;         // element offset of the intermediate region
  int64_t inter_elems = 0;
  size_t ws_bytes = 0;
  int32_t select_iters = 64;     // counting rounds before the sort fallback
  int32_t select_cand = 64;      // candidates handed to the exact in-lane select
  std::mutex dev_mu;
  std::deque<ffa::DeviceTables> dev;  // one entry per device used (stable addresses)
};

namespace ffa {

// Error reporting (thread-local detail string).
ffa_status fail(ffa_status st, const std::string& msg);
ffa_status check_hip(hipError_t e, const char* what);

// Device tables of plan p on the current device (creates them on first use).
ffa_status device_tables(ffa_plan p, const DeviceTables** out);

// Kernel launchers (ffa_kernels.hip).  All element offsets are in 4-byte
// elements relative to ws.  is_int selects int32 accumulation (uint8 input).
hipError_t launch_mean(const float* x, int64_t n, void* ws, hipStream_t st);
hipError_t launch_prep(const void* series, int is_int, int64_t n, void* ws,
                       int64_t out_off, int center, hipStream_t st);
hipError_t launch_halve(void* ws, int is_int, int64_t in_off, int64_t n_out,
                        int64_t out_off, hipStream_t st);
hipError_t launch_pass(const Tile* tiles, int64_t n_tiles, int lds_bytes, int max_P0,
                       int is_int, void* ws, float* snr, int32_t* width,
                       void* profiles, int64_t trial_base, int mode,
                       const int32_t* wtab, const double* sqrtw,
                       int select_iters, int select_cand, hipStream_t st);
hipError_t launch_best(const float* snr, int64_t n, int64_t* best,
                       hipStream_t st);

}  // namespace ffa
