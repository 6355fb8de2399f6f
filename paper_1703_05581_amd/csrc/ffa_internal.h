// Internal declarations of the FFA library: plan layout, work queue and the
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
constexpr int kMaxBinsMin = 1024;         // P0 < 2*B <= 2048
constexpr int kMaxPasses = 8;
constexpr int kThreads = 1024;            // threads per workgroup of the FFA kernel
constexpr size_t kLdsBytes = 160 * 1024;  // gfx950 LDS per workgroup
constexpr size_t kWsAlign = 256;
constexpr size_t kScratchBytes = (kThreads / 64) * 64 * 4;  // per-wave selection scratch

// sigma = K * MAD (paper Sec. 2.2.1): K is 1 / (75% quantile of the unit normal).
constexpr double kMadK = 1.482602218505602;

// What the last pass of a step does with its profiles.
enum : int32_t { kModeScore = 1, kModeProfiles = 2 };

// One pass of one step: Q*ng tiles, each 2^depth rows of P0 bins (a "group")
// whose butterfly levels run on chip.  Tile k is problem q = k / ng, group
// h = k % ng.
struct Phase {
  int64_t tile0;        // first tile of the phase in its plan's queue order
  int64_t oct_off;      // pass 0: element offset of the octave series in the workspace
  int64_t first_trial;  // trial index of the step's trial 0
  int32_t ntiles;
  int32_t ng;           // groups with data per problem
  int32_t step;         // step index in the plan
  int32_t pass;
  int32_t last;         // 1 on the step's last pass
  int32_t P0;
  int32_t M;
  int32_t depth;        // levels run by this pass
  int32_t D;            // levels run by the earlier passes
  int32_t vin;          // rows with data per problem
  int32_t stride;       // LDS row stride (elements)
  int32_t halo;         // LDS bins after P0 that repeat bins 0..halo-1
  int32_t wofs;         // the step's widths in the width tables
  int32_t nw;
  int32_t isqrt_ofs;    // the step's 1/sqrt(width) values in the sqrt table
  int32_t launch;       // index of the launch that runs the phase
  int32_t u16;          // 1: the tile keeps its rows as 16-bit sums in LDS
  int32_t ring64;       // multi-pass step: its intermediates start at ring_off + 64*ring64
  int32_t series;       // series of a batch (index of its output pointers); 0 for one plan
  int32_t reserved;
};
static_assert(sizeof(Phase) == 104, "phase layout");

// Periodogram outputs of one series of a batch (device table, one entry per
// series, indexed by Phase::series).
struct SeriesOut {
  float* snr;
  int32_t* width;
};

// Arguments of one launch of the FFA kernel: tiles tile0 .. tile0+grid-1 of a
// plan's queue (or of one step's passes, for a fold).
struct TileArgs {
  const Phase* phases;        // queue-ordered phases (or one fold phase)
  const int32_t* tile_phase;  // phase index of every queue tile; null: all tiles are phases[0]
  const int32_t* widths;
  const double* sqrtw;
  float* snr;
  int32_t* width;
  const SeriesOut* outs;      // batch: per-series outputs (replaces snr/width); null otherwise
  void* profiles;             // fold: M*P0 output of the step
  int64_t tile0;
  int64_t oct_base;           // element offset of the series region in the workspace
  int64_t ring_off;           // element offset of the intermediate ring
  int64_t trial_base;         // fold: trial index of output row 0
  int32_t mode;
  int32_t alg;                // profile score: 1 = Algorithm 1, 2 = Algorithm 2
  int32_t select_iters;
  int32_t select_cand;
};

struct Step {
  int32_t f, octave, P0, m, M, L;
  int64_t first_trial;
  int32_t n_passes;
  int32_t depth[kMaxPasses];
  int32_t wofs, nw, wmax;
  int32_t tiles[kMaxPasses];  // tiles of each pass
  int32_t total_tiles;
  int32_t lds_bytes;          // largest LDS footprint of its passes
  int32_t fold_phase0;        // its phases in pass order, in Plan::fold_phases
  int64_t lds_budget = 0;     // LDS bytes a tile may use
  int32_t u16_first = 0;      // the first of two passes keeps 16-bit sums
  int64_t ring_pos = 0;       // multi-pass: element offset of its intermediates in the ring
  int32_t series = 0;         // series of a batch
  int64_t oct_off = 0;        // element offset (in the workspace) of the octave series it folds
  int64_t in_end = 0;         // end of that octave series: pass 0 reads within [oct_off, in_end)
};

// One launch of a search: a window of the queue whose tiles depend only on
// tiles of earlier launches.
struct Launch {
  int64_t tile0, ntiles;
  int32_t lds_bytes;
  int32_t max_P0;
};

// Launch knobs of a work queue (they change the launches, never a result).
struct QueueKnobs {
  int64_t window_tiles = 32768;          // target tiles per window group (all passes)
  int64_t ring_bytes = int64_t(4096) << 20;  // intermediate ring budget
  int64_t fixed_steps = 0;               // > 0: that many steps per window group instead
  bool split_occupancy = true;           // one launch per LDS occupancy class in each window
};

// The work queue of a list of steps (one plan's, or every step of a batch of
// plans): their passes' phases in queue order, the tile -> phase map, the
// launches, and the intermediate ring the multi-pass steps share.
struct Queue {
  std::vector<Phase> phases;     // queue order: pass p of step group g in window g + p
  std::vector<int32_t> tile_phase;
  std::vector<Launch> launches;
  int64_t n_tiles = 0;
  int64_t ring_elems = 0;
  int32_t max_passes = 1;
  int32_t lookahead = 1;         // steps in the largest window group
  int32_t lds_bytes = 0;
  int32_t max_P0 = 0;
};

// Orders the phases of `steps` into a queue.  `nat` holds every step's passes
// in order (steps[i].fold_phase0 indexes it).  Sets each multi-pass step's
// ring_pos and the phases' ring64.  Returns FFA_ERR_UNSUPPORTED when the
// queue has 2^31 tiles or more.
ffa_status build_queue(std::vector<Step>& steps, std::vector<Phase>& nat, const QueueKnobs& kn, Queue* q);
// Every tile of the queue reads and writes inside its buffers and reads only
// what an earlier launch wrote (checked on the host before any launch).
// acc_int: the queue folds exact integer sums (16-bit first passes allowed).
bool queue_valid(const std::vector<Step>& steps, const Queue& q, int acc_int);
// Bytes of LDS a phase's tile uses (its rows at the planned element size, and
// the selection scratch on a scoring pass).
int64_t phase_lds(const Phase& ph);

// A step as the candidate sifting needs it (trial -> period).
struct StepDev {
  int64_t first_trial;
  int32_t f, P0, m, M;
};

constexpr int32_t kSiftMaxPeaks = 16384;
constexpr int kSiftBlock = 1024;  // trials per block of the compaction

// Device copies of a plan's tables (made on first use on a device).
// One series of the exact running-median dereddening (paper Sec. 2.3.1) in
// a launch over many: the raw octave series at x_off (doubles) is filtered
// into the float32 series at out_off (offsets in 4-byte elements from the
// workspace base), with `window` samples.
struct DeredSeg {
  int64_t x_off;
  int64_t out_off;
  int64_t n;
  int64_t block0;     // first block of the segment (blocks are numbered across all launches)
  int32_t window;
  int32_t use_stage;  // the union of a block's windows is staged in LDS
};

// Blocks [block0, block0 + blocks) of a dereddening plan, `lds` bytes each.
struct DeredLaunch {
  int64_t block0;
  int64_t blocks;
  int32_t lds;
};

// The exact dereddening of several series as a few launches: segments grouped
// by how many of their blocks share a CU, and the segment of every block.
struct DeredPlan {
  std::vector<DeredSeg> segs;
  std::vector<int32_t> block_seg;
  std::vector<DeredLaunch> launches;
};

struct DeviceTables {
  int device = -1;
  StepDev* steps = nullptr;
  Phase* phases = nullptr;
  Phase* fold_phases = nullptr;
  int32_t* tile_phase = nullptr;
  int32_t* widths = nullptr;
  double* sqrtw = nullptr;
  DeredSeg* dered_segs = nullptr;       // the plan's dereddening plan (float input, exact filter)
  int32_t* dered_block_seg = nullptr;
};

}  // namespace ffa

struct ffa_plan_s {
  ffa_plan_desc desc;
  std::vector<int32_t> user_widths;
  uint64_t uid = 0;                     // unique per plan created in the process
  std::vector<ffa::Step> steps;
  std::vector<ffa::Phase> nat_phases;   // per step, its passes in order (ring placement unset)
  std::vector<ffa::Phase> phases;       // queue order: pass p of step group g in window g + p
  std::vector<ffa::Phase> fold_phases;  // per step, its passes in order
  std::vector<int32_t> tile_phase;      // queue tile -> index in phases
  std::vector<ffa::Launch> launches;     // launches of a search, in order
  ffa::QueueKnobs knobs;                // the knobs the queue was built with
  std::vector<int32_t> wtab;            // widths of every step, concatenated
  std::vector<double> sqrtw;            // sqrt(width), same layout, then 1/sqrt(width)
  int64_t n_trials = 0;
  int64_t n_tiles = 0;
  int32_t max_passes = 1;
  int32_t lookahead = 1;                // steps in the largest window group
  int64_t ring_elems = 0;               // elements of the intermediate ring
  int32_t lds_bytes = 0;                // largest tile LDS footprint
  int32_t max_P0 = 0;
  int32_t n_octaves = 0;                // octaves 0..n_octaves-1 are built
  std::vector<int64_t> oct_off;         // series-relative offset of each octave series
  std::vector<int64_t> oct_len;
  int64_t hdr_elems = 0;                // header (centring scratch) in elements
  int64_t series_elems = 0;             // header + octave series
  int32_t acc_int = 0;                  // folds in exact int32 (uint8 input, no dereddening)
  int32_t dered_W = 0;                  // dereddening window in samples (0: off)
  int32_t dered_stride = 1;             // knot spacing
  int32_t dered_oct0 = 0;               // first octave a step uses (the ones below only feed halving)
  int64_t knots_off = 0;                // workspace: knot medians (double) of one octave series
  std::vector<int64_t> raw_off;         // float input, dereddened: raw octave series in double
  ffa::DeredPlan dered;                 // float input, exact filter: every octave's dereddening at once
  int64_t ring_off = 0;                 // workspace: series region, knots, then the ring
  int64_t sift_elems = 0;               // scratch of ffa_sift, from ring_off
  size_t ws_bytes = 0;
  int32_t select_iters = 64;            // counting rounds before key halving
  int32_t select_cand = 64;             // candidates handed to the in-lane select
  std::mutex dev_mu;
  std::deque<ffa::DeviceTables> dev;    // one entry per device used (stable addresses)
};

namespace ffa {

// Error reporting (thread-local detail string).
ffa_status fail(ffa_status st, const std::string& msg);
ffa_status check_hip(hipError_t e, const char* what);

// Device tables of plan p on the current device (creates them on first use).
ffa_status device_tables(ffa_plan p, const DeviceTables** out);
// The same tables if they already exist on the current device (allocates
// nothing); FFA_ERR_INVALID otherwise.
ffa_status find_device_tables(ffa_plan p, const DeviceTables** out);

// dt: the plan's device tables on the current GPU (null: the octaves are
// dereddened one launch each); dered = false leaves the dereddening of float
// input to the caller (a batch runs it for all its series at once).
ffa_status build_octaves(ffa_plan p, const void* series, void* ws, int32_t last_octave,
                         int center, hipStream_t st, const DeviceTables* dt, bool dered = true);
// Groups the segments of dp (x_off, out_off, n and window set) into
// launches and numbers their blocks.
void plan_dered(DeredPlan& dp);
// Copies a dereddening plan's tables to the device (null pointers when it is empty).
ffa_status upload_dered(const DeredPlan& dp, DeredSeg** segs, int32_t** block_seg);
// Runs every launch of dp on ws.
ffa_status run_dered(const DeredPlan& dp, const DeredSeg* d_segs, const int32_t* d_block_seg, void* ws,
                     hipStream_t st);
// Every launch of plan p's search on `st`, workspace `ws` already holding the
// octave series.
ffa_status run_launches(ffa_plan p, const DeviceTables* dt, float* snr, int32_t* width, void* ws,
                       hipStream_t st);

// Kernel launchers (ffa_kernels.hip).  All element offsets are in 4-byte
// elements relative to ws.  is_int selects int32 accumulation (uint8 input).
hipError_t launch_mean(const float* x, int64_t n, void* ws, hipStream_t st);
hipError_t launch_prep(const void* series, int is_int, int64_t n, void* ws, int64_t out_off,
                       int center, hipStream_t st);
hipError_t launch_halve(void* ws, int is_int, int64_t in_off, int64_t n_out, int64_t out_off,
                        hipStream_t st);
// Running-median dereddening of the n-sample series at element src_off of
// ws (src_type 0: int32 sums, 1: float, 2: double), written as float32 at
// element out_off (may equal src_off for 4-byte sources); knot medians
// (double) in ws[knots_off ..) (see ffa_plan_desc.dered_window).
hipError_t launch_deredden(void* ws, int src_type, int64_t src_off, int64_t n, int32_t window, int32_t stride,
                           int64_t knots_off, int64_t out_off, hipStream_t st);
// LDS bytes of one block of the exact running median of an n-sample series
// (and whether it stages the union of its windows), and its block count.
size_t dered_block_lds(int64_t n, int32_t window, int32_t* use_stage);
int64_t dered_block_count(int64_t n);
// Allows the dereddening kernel the CU's whole LDS on the current device
// (called where its tables are made, outside any stream capture).
hipError_t prepare_dered_batch();
// One launch of a dereddening plan (device tables).
hipError_t launch_dered_batch(const DeredSeg* segs, const int32_t* block_seg, const DeredLaunch& L, void* ws,
                              hipStream_t st);
// float32 -> double copy, and one halving of a double series (element offsets)
hipError_t launch_prep_f64(const float* series, int64_t n, void* ws, int64_t out_off, hipStream_t st);
hipError_t launch_halve_f64(void* ws, int64_t in_off, int64_t n_out, int64_t out_off, hipStream_t st);
// Checks that the kernel variant for max_P0 fits lds_bytes of dynamic LDS on
// the current device (static LDS included); caches the answer.
bool tiles_fit(int is_int, int max_P0, int lds_bytes, int alg);
hipError_t launch_tiles(const TileArgs& a, int64_t ntiles, int lds_bytes, int max_P0, int is_int,
                        void* ws, hipStream_t st);
hipError_t launch_best(const float* snr, int64_t n, int64_t* best, hipStream_t st);
// Writes the n entries of host array src to the device table dst (kernel
// arguments carry the values, so nothing on the host must outlive the call).
hipError_t launch_set_outs(SeriesOut* dst, const SeriesOut* src, int32_t n, hipStream_t st);
constexpr int32_t kHistMaxBins = 16384;
hipError_t launch_snr_histogram(const float* snr, int64_t n, float lo, float bins_per_unit, int32_t n_bins,
                                uint64_t* hist, hipStream_t st);
// Candidate sifting (ffa_sift); scratch at element `scratch` of ws.
hipError_t launch_sift(const float* snr, const int32_t* width, int64_t n, const ffa_sift_params& prm,
                       const StepDev* steps, int32_t n_steps, double tsamp, void* ws, int64_t scratch,
                       ffa_candidate* out, int32_t max_out, int32_t* n_out, hipStream_t st);

}  // namespace ffa
