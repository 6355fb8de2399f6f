/*
 * ffa.h -- C ABI of the MI355X FFA periodicity search.
 *
 * The library folds a time series at every trial period of a period range
 * with the Fast Folding Algorithm and scores every folded profile with a
 * boxcar matched filter, producing a periodogram (Cameron et al. 2017,
 * "An investigation of pulsar searching techniques with the Fast Folding
 * Algorithm", MNRAS; referred to below as "the paper").
 *
 * Conventions for every call:
 *   - Pointers named d_* are device (HBM) pointers on the GPU that was
 *     current when the plan was created; everything else is host memory.
 *   - The caller owns every data buffer and every workspace.  The library
 *     owns plans and servers and never frees caller memory.
 *   - Calls that take a stream enqueue work on it and return before the GPU
 *     is done (asynchronous).  `stream` is a hipStream_t passed as void*;
 *     NULL is the default stream.  Argument errors are detected on the host
 *     and returned before anything is enqueued.
 *   - A launch error is returned as FFA_ERR_DEVICE by the call that made it.
 *   - No C++ exception crosses this boundary.  ffa_last_error() gives a
 *     human-readable detail of the calling thread's last failure.
 *   - Input samples must be finite.
 */
#ifndef FFA_H_
#define FFA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffa_plan_s* ffa_plan;
typedef struct ffa_server_s* ffa_server;

typedef enum {
  FFA_OK = 0,
  FFA_ERR_INVALID = -1,     /* bad argument; nothing enqueued */
  FFA_ERR_NOMEM = -2,       /* host or device allocation failed */
  FFA_ERR_DEVICE = -3,      /* HIP call or kernel launch failed */
  FFA_ERR_UNSUPPORTED = -4, /* valid but outside what the library handles */
  FFA_ERR_BUSY = -5,        /* server admission queue full */
  FFA_ERR_TIMEOUT = -6      /* wait ran out of time */
} ffa_status;

/* Sample type of the input series (the two formats the paper's search reads,
 * Sec. 2.3.1): 32-bit float, or 8-bit unsigned summed exactly in integers. */
typedef enum { FFA_IN_F32 = 0, FFA_IN_U8 = 1 } ffa_dtype;

/* Profile score.  ALG1: boxcar matched filter on the profile normalised by its
 * median and K*MAD (Sec. 2.2.1, Eqs. 3-4).  ALG2: boxcar first, then mean and
 * standard deviation outside a 20% window around the peak (Sec. 2.2.2,
 * Eq. 5). */
typedef enum { FFA_SNR_ALG1_MAD = 1, FFA_SNR_ALG2_OFFPULSE = 2 } ffa_snr;

/* Search description.
 *   N          samples in the series (>= 2)
 *   tsamp_s    sampling interval in seconds
 *   pmin_s, pmax_s   period range [pmin, pmax) in seconds
 *   widths, n_widths boxcar widths in bins (copied; NULL/0 selects the
 *              paper's rule per step: 1, 2, 4, ... up to and including the
 *              first power of two above 20% of P0, Sec. 2.2.1).  Widths larger
 *              than a step's P0 are skipped for that step.  At most 32.
 *   bins_min   B: the base period P0 (in downsampled bins) runs over [B, 2B)
 *              in each octave; octave o searches the series downsampled by
 *              f = 2^o (Sec. 2.3.1).  2 <= B <= 1024.
 *   max_octaves  0 = as many as pmax needs, else at most this many octaves.
 *   dtype      ffa_dtype;   snr  ffa_snr.
 *   dered_window  dynamic running-median dereddening (Sec. 2.3.1): 0 = off;
 *              -1 = the paper's default window, the smaller of 2*pmax and
 *              4*pmin in samples (rounded); > 0 = that many samples.  Every
 *              octave series is filtered with the same number of its own
 *              samples, so the window doubles relative to the input with
 *              each downsampling.  The filter subtracts from each sample the
 *              median of the window's samples starting window/2 before it
 *              (clipped to the series; an even count takes the mean of the
 *              middle two).  A dereddened search runs in float32 also for
 *              uint8 input.
 *   dered_stride  0 or 1: that running median at every sample (exact);
 *              > 1: a faster approximation, the median only at knots every
 *              dered_stride samples with the baseline interpolated linearly
 *              between them (the last knot's median after it).
 *
 * Steps: for each octave f = 1, 2, 4, ... and each integer P0 in [B, 2B)
 * with pmin <= P0*f*tsamp < pmax, one FFA execution folds m = floor(N_f/P0)
 * rows of the series downsampled by f (N_f = floor(N/f) samples; the tail is
 * dropped), zero-padded to M = 2^ceil(log2 m) rows (Sec. 2.1).  Steps with
 * m < 2 are skipped.  Trial k = 0..M-1 of a step has period
 * f*tsamp*(P0 + k/(M-1)) seconds (Eqs. 1-2 with N replaced by M*P0).
 * Trials are numbered in step order: octave ascending, then P0 ascending,
 * then k. */
typedef struct {
  int64_t N;
  double tsamp_s;
  double pmin_s;
  double pmax_s;
  const int32_t* widths;
  int32_t n_widths;
  int32_t bins_min;
  int32_t max_octaves;
  int32_t dtype;
  int32_t snr;
  int32_t dered_window;
  int32_t dered_stride;
} ffa_plan_desc;

/* Build a plan: step list, pass split of every step, work queue.  Host
 * only (no device call); the plan's device tables are made on a GPU by the
 * first call there that needs them, or by ffa_plan_upload.  Errors:
 * FFA_ERR_INVALID (bad field, no step, a step with no usable width),
 * FFA_ERR_UNSUPPORTED (uint8 series with 255*N >= 2^31, or a step too large
 * for the kernels), FFA_ERR_NOMEM. */
ffa_status ffa_plan_create(const ffa_plan_desc* desc, ffa_plan* out);
ffa_status ffa_plan_destroy(ffa_plan plan);

/* Makes the plan's device tables on the current GPU now (the first search on
 * a GPU otherwise makes them).  Errors: FFA_ERR_UNSUPPORTED (a GPU with less
 * than 160 KiB of LDS per workgroup), FFA_ERR_NOMEM, FFA_ERR_DEVICE. */
ffa_status ffa_plan_upload(ffa_plan plan);

/* Launch options of a plan.  They change how the work is cut into tiles,
 * passes and launches (and so the speed), never a result: every setting
 * gives the same periodogram, bit for bit.  A zeroed struct selects the
 * defaults, which is what ffa_plan_create uses.
 *   tile_lds_bytes   LDS budget of one tile, 16384..163840 (0: 163840)
 *   window_tiles     tiles (all passes) per window group, 1..2^24 (0: 32768)
 *   ring_mb          budget of the intermediate ring in MiB, 1..2^20 (0: 4096)
 *   steps_per_window > 0: that many steps per window group instead (0: by tiles)
 *   no_u16           1: uint8 steps keep 32-bit rows in every pass (0: a first
 *                    pass may keep exact 16-bit sums where they fit)
 *   no_split_occupancy  1: one launch per window (0: one per LDS occupancy class)
 *   select_iters, select_cand   exits of the median/MAD selection, for tests:
 *                    counting rounds before key halving (0: 64; < 0: none)
 *                    and candidates handed to the in-register select (0: 64,
 *                    else 1..64)
 * Out-of-range values give FFA_ERR_INVALID. */
typedef struct {
  int32_t tile_lds_bytes;
  int32_t window_tiles;
  int32_t ring_mb;
  int32_t steps_per_window;
  int32_t no_u16;
  int32_t no_split_occupancy;
  int32_t select_iters;
  int32_t select_cand;
} ffa_plan_opts;

/* ffa_plan_create with launch options (opts NULL: the defaults). */
ffa_status ffa_plan_create_opts(const ffa_plan_desc* desc, const ffa_plan_opts* opts, ffa_plan* out);

/* Totals of a plan.  ws_bytes is the device workspace ffa_search and
 * ffa_fold need.  Any output pointer may be NULL. */
ffa_status ffa_plan_query(ffa_plan plan, int64_t* n_trials, int32_t* n_steps,
                          size_t* ws_bytes);

/* Shape of step s: octave factor f, base period P0, data rows m, padded rows
 * M, index of its first trial.  Any output pointer may be NULL. */
ffa_status ffa_plan_step(ffa_plan plan, int32_t s, int32_t* f, int32_t* P0,
                         int32_t* m, int32_t* M, int64_t* first_trial);

/* Pass split of step s: number of FFA passes and the butterfly levels each
 * pass runs on chip (depths[0..n_passes-1], at most 8 entries written). */
ffa_status ffa_plan_passes(ffa_plan plan, int32_t s, int32_t* n_passes,
                           int32_t* depths);

/* Trial periods in seconds, host array of n_trials doubles. */
ffa_status ffa_plan_periods(ffa_plan plan, double* host_periods_s);

/* Periodogram of one series (Sec. 2.2: one score per folded profile, plotted
 * against trial period).
 *   d_series  N samples, float32 or uint8 per the plan's dtype
 *   d_snr     n_trials float32: score of each trial (0 where the profile's
 *             MAD is 0)
 *   d_width   n_trials int32: boxcar width in bins that gave the score (first
 *             width in list order on ties; 0 where MAD is 0)
 *   d_ws      workspace of at least ws_bytes (ffa_plan_query), 256-B aligned
 * Float series are centred on their mean before folding; the scores of both
 * algorithms are unchanged by an offset.  uint8 series are summed exactly in
 * 32-bit integers.  Errors: FFA_ERR_INVALID (NULL pointer, small workspace,
 * wrong device), FFA_ERR_DEVICE. */
ffa_status ffa_search(ffa_plan plan, const void* d_series, float* d_snr,
                      int32_t* d_width, void* d_ws, size_t ws_bytes,
                      void* stream);

/* ffa_search for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is a fixed 64 MiB array the library holds on each GPU for the
 * life of the process, instead of d_ws, and nothing is allocated.  Every
 * call on a GPU shares that array, so two calls that overlap on one GPU
 * race (serialise them, e.g. on one stream); no contents carry over between
 * calls.  The plan's device tables must already exist on the current GPU
 * (ffa_plan_upload, or an earlier search).  Results equal ffa_search's.
 * Errors: FFA_ERR_INVALID (NULL pointer, no device tables on this GPU),
 * FFA_ERR_UNSUPPORTED (the plan's ws_bytes above 64 MiB: lower its ring_mb),
 * FFA_ERR_DEVICE. */
ffa_status ffa_search_noalloc(ffa_plan plan, const void* d_series, float* d_snr,
                              int32_t* d_width, void* stream);

/* ffa_search in two parts.  ffa_prepare builds the downsampled octave series
 * of `d_series` in the workspace (centred on the mean for float input);
 * ffa_search_prepared then runs every FFA pass and the scoring of every
 * profile, reading the octave series that the last ffa_prepare on the same
 * workspace and plan left there.  Same arguments and errors as ffa_search. */
ffa_status ffa_prepare(ffa_plan plan, const void* d_series, void* d_ws,
                       size_t ws_bytes, void* stream);
ffa_status ffa_search_prepared(ffa_plan plan, float* d_snr, int32_t* d_width,
                               void* d_ws, size_t ws_bytes, void* stream);

/* Raw folded profiles of step `step` (Sec. 2.1): M rows of P0 bins, row k is
 * trial k.  float32 series give float32 sums; uint8 series give exact int32
 * sums, or float32 sums of the dereddened series when the plan dereddens.
 * Not centred (apart from dereddening).  Errors as ffa_search. */
ffa_status ffa_fold(ffa_plan plan, const void* d_series, int32_t step,
                    void* d_profiles, void* d_ws, size_t ws_bytes,
                    void* stream);

/* Best trial of a periodogram (the peak of Sec. 2.2's periodogram): the
 * largest score, the first trial on ties; NaN scores never win, -0 equals +0.
 *   d_snr        n_trials scores (as from ffa_search), 1 <= n_trials < 2^32
 *   d_best       one int64 on the device: index of the best trial (also used
 *                as the reduction's accumulator while the call runs)
 * Errors: FFA_ERR_INVALID, FFA_ERR_DEVICE. */
ffa_status ffa_best(const float* d_snr, int64_t n_trials, int64_t* d_best,
                    void* stream);

/* Candidate sifting of a periodogram on the GPU, after the paper's ffa2best
 * (Sec. 2.3.3; the settings of Sec. 4 are min_snr 9, primes up to 31,
 * tolerance 1e-5 for Algorithm 1 and 1e-4 for Algorithm 2).  The paper does
 * not give the exact rules; the ones used:
 *   peaks: trials in plan order (period non-decreasing); a trial with
 *     S/N >= min_snr opens a candidate when none is open; a higher S/N moves
 *     the open candidate there; it closes once the S/N has fallen from it by
 *     at least frac_fall * its S/N and by at least abs_fall, or below min_snr
 *     (NaN counts as below).
 *   grouping (group_widths > 0): strongest first (ties: lower trial), a
 *     surviving candidate removes weaker ones whose period differs by at most
 *     group_widths * W * P / T, W its boxcar width in seconds and T the
 *     folded span m*P0*f*tsamp of its step (the smear of one pulse width
 *     per group_widths across the data).
 *   harmonics (harmonic_primes >= 2): strongest first, a surviving candidate
 *     removes weaker ones within a relative harmonic_tol of P*n/x or P*x/n,
 *     x prime <= harmonic_primes, 0 < n < x. */
typedef struct {
  float min_snr;
  float frac_fall;
  float abs_fall;
  float group_widths;
  int32_t harmonic_primes;
  float harmonic_tol;
} ffa_sift_params;

typedef struct {
  int64_t trial;     /* index in the periodogram */
  double period_s;   /* f*tsamp*(P0 + k/(M-1)) */
  float snr;
  int32_t width;     /* boxcar width in bins of the step's octave */
} ffa_candidate;

/* Sift the periodogram (d_snr, d_width: n_trials entries of `plan`) into
 * d_cands (device, room for max_cands), strongest first.  *d_n_cands
 * (device) receives the number of candidates found (only the first max_cands
 * are written), or -1 when more than 16384 peaks pass the thresholds (raise
 * min_snr).  The plan's workspace (d_ws, at least the plan's ws_bytes,
 * 256-B aligned) is used as scratch; its contents are not needed after a
 * search.  Parameters: min_snr finite, 0 <= frac_fall <= 1, abs_fall,
 * group_widths and harmonic_tol finite and >= 0, harmonic_primes <= 1000,
 * max_cands >= 0 (0: count only).  Asynchronous on `stream`.  Errors:
 * FFA_ERR_INVALID (bad parameter, small workspace), FFA_ERR_DEVICE. */
ffa_status ffa_sift(ffa_plan plan, const float* d_snr, const int32_t* d_width,
                    const ffa_sift_params* params, ffa_candidate* d_cands,
                    int32_t max_cands, int32_t* d_n_cands, void* d_ws,
                    size_t ws_bytes, void* stream);

/* False-alarm statistics (Sec. 4.1.2).  The paper calibrates significance
 * by searching data without pulsars and mapping each S/N to a Gaussian-
 * equivalent sigma through the fraction of trials that reach it.  The counts
 * come from a histogram that any number of searches accumulate into; the
 * mapping runs on the host over the histogram.
 *
 * ffa_snr_histogram: adds the n scores of d_snr (device) to d_hist (device,
 * n_bins uint64 counts, which the caller zeroes before the first call).  Bin
 * b holds the scores with floor((s - lo) * bins_per_unit) == b, the product
 * taken in float; scores below lo count in bin 0 and scores past the top in
 * bin n_bins - 1, so the count at or above every inner edge
 * lo + b / bins_per_unit (b >= 1) is exact.  NaN is not counted.
 *   1 <= n_bins <= 16384, lo and bins_per_unit finite, bins_per_unit > 0,
 *   n >= 0 (0 does nothing).  Asynchronous on `stream`.
 * Errors: FFA_ERR_INVALID, FFA_ERR_DEVICE. */
ffa_status ffa_snr_histogram(const float* d_snr, int64_t n, float lo,
                             float bins_per_unit, int32_t n_bins,
                             uint64_t* d_hist, void* stream);

/* Host.  sigma[b] (n_bins doubles) = the Gaussian-equivalent sigma at the
 * lower edge of bin b: with Q the fraction of counts in bins b and above,
 * the sigma that a standard normal variable exceeds with probability Q.
 * Bin 0 (Q = 1) gives -inf, an edge no count reaches +inf.
 * Errors: FFA_ERR_INVALID (NULL pointer, n_bins < 1, empty histogram). */
ffa_status ffa_sigma_gauss(const uint64_t* hist, int32_t n_bins, double* sigma);

/* Host.  *snr = the S/N that a `sigma`-sigma detection needs: the lowest
 * inner edge lo + b / bins_per_unit (b >= 1, in double) at or above which
 * the count is at most Phi(-sigma) times the total.  Errors: FFA_ERR_INVALID
 * (NULL pointer, empty histogram, or a top bin that already holds more than
 * that fraction: widen the histogram). */
ffa_status ffa_sigma_threshold(const uint64_t* hist, int32_t n_bins, float lo,
                               float bins_per_unit, double sigma, double* snr);

/* Batched search: the periodograms of n series, each with its own plan (any
 * mix of lengths, period ranges, sample types and algorithms).  Sec. 4 of
 * the paper searches many dedispersed series of one observation; a batch
 * runs them as one work queue.  The steps of all its series are cut into
 * window groups of about window_tiles tiles, whatever series they belong to,
 * so one launch runs the tiles of many series (one queue per kind of
 * arithmetic: exact integer or float folds, Algorithm 1 or 2).
 *
 * ffa_batch_create plans a batch of the n plans (host only; the plans must
 * outlive the batch, which keeps pointers to them).  Device tables are made
 * on the first search on a GPU.  ffa_batch_query gives the workspace bytes a
 * search needs, the tiles and the kernel launches of one search (any output
 * pointer may be NULL).  ffa_batch_destroy frees the batch; the caller makes
 * sure no search of it is still running.
 *
 * ffa_batch_search enqueues the search of all n series on `stream`:
 *   d_series[i], d_snr[i], d_width[i]  host arrays of n device pointers:
 *          series i (N_i samples of plan i's type) and its periodogram
 *          (n_trials_i floats and ints, as ffa_search writes them)
 *   d_ws   workspace of at least the batch's ws_bytes, 256-B aligned
 * Results equal those of ffa_search on each series, bit for bit.
 * Errors: FFA_ERR_INVALID (NULL pointer, small workspace),
 * FFA_ERR_NOMEM, FFA_ERR_DEVICE; after a launch error, work already enqueued
 * still runs to its end.
 *
 * ffa_batch_workspace and ffa_search_batch do the same from the plan list
 * itself: the library keeps the batches of the last few plan lists it was
 * given (a destroyed plan never matches), so a repeated call does not plan
 * again, and frees an evicted batch once its last search is done. */
typedef struct ffa_batch_s* ffa_batch;
ffa_status ffa_batch_create(int32_t n, const ffa_plan* plans, ffa_batch* out);
ffa_status ffa_batch_destroy(ffa_batch batch);
ffa_status ffa_batch_query(ffa_batch batch, size_t* ws_bytes, int64_t* n_tiles, int32_t* n_launches);
ffa_status ffa_batch_search(ffa_batch batch, const void* const* d_series, float* const* d_snr,
                            int32_t* const* d_width, void* d_ws, size_t ws_bytes, void* stream);
/* ffa_batch_search in two parts, like ffa_prepare and ffa_search_prepared:
 * the octave series of every series (each in its region of d_ws), then
 * every FFA pass and the scoring of every profile, reading what the last
 * ffa_batch_prepare on the same workspace and batch left there.  Same
 * arguments and errors as ffa_batch_search. */
ffa_status ffa_batch_prepare(ffa_batch batch, const void* const* d_series, void* d_ws, size_t ws_bytes,
                             void* stream);
ffa_status ffa_batch_search_prepared(ffa_batch batch, float* const* d_snr, int32_t* const* d_width,
                                     void* d_ws, size_t ws_bytes, void* stream);
ffa_status ffa_batch_workspace(int32_t n, const ffa_plan* plans,
                               size_t* ws_bytes);
ffa_status ffa_search_batch(int32_t n, const ffa_plan* plans,
                            const void* const* d_series, float* const* d_snr,
                            int32_t* const* d_width, void* d_ws,
                            size_t ws_bytes, void* stream);

/* Search server: continuous batching of requests that arrive over time
 * (Sec. 4 searches many dedispersed series of one observation).
 *
 * ffa_server_create allocates one device pool of hbm_budget_bytes on the
 * current GPU and n_streams streams (1..16, default priority).  A scheduler
 * thread admits pending requests in arrival order whenever the head
 * request's footprint -- series copy (host input only) + the plan's
 * ws_bytes + the periodogram (8 B per trial) -- fits in what is free, and
 * enqueues it on the least-loaded stream, next to the requests already
 * running.  When the head does not fit, a later request (among the next 64)
 * that fits is admitted before it (backfill), until max_bypass requests have
 * passed that head; then admission waits until the head fits.  max_bypass 0
 * admits in strict arrival order (under heavy load it kept the tail latency
 * lower than backfill, which delays the largest requests).  A request keeps
 * its memory until it is
 * waited on.  All server calls are thread-safe; ffa_server_destroy must not
 * race with the others.
 * Errors: FFA_ERR_INVALID (budget below 256 B, n_streams out of range,
 * max_bypass < 0), FFA_ERR_NOMEM (pool allocation), FFA_ERR_DEVICE. */
ffa_status ffa_server_create(size_t hbm_budget_bytes, int32_t n_streams,
                             int32_t max_bypass, ffa_server* out);

/* Submit a search of `series` with `plan`.  Host input (is_device == 0) is
 * copied at the call, so the caller may reuse its buffer at once;
 * producer_stream is ignored.  A device series (is_device != 0) is read
 * only after the work queued on producer_stream (a hipStream_t of the
 * server's device; NULL = the null stream) before this call has finished:
 * an event is recorded there now and the request's stream waits on it.  The
 * series must stay valid and unmodified until the request completes, and the
 * server's device must be current.  The plan must outlive the request.
 * Returns a ticket (> 0, issued in order from 1).  Errors: FFA_ERR_INVALID,
 * FFA_ERR_UNSUPPORTED (footprint above the whole budget), FFA_ERR_BUSY
 * (65536 requests pending), FFA_ERR_NOMEM, FFA_ERR_DEVICE (event record). */
ffa_status ffa_server_submit(ffa_server s, ffa_plan plan, const void* series,
                             int is_device, void* producer_stream,
                             int64_t* ticket);

/* Wait for a ticket (timeout_us < 0: forever; 0: poll).  Copies the
 * periodogram to the host arrays (n_trials entries each; either may be NULL),
 * releases the request's device memory, and reports its latency: submit to
 * the end of its search on the GPU (the result copy is not included).  A
 * ticket can be waited on once.  Errors: FFA_ERR_INVALID (unknown or already
 * collected ticket), FFA_ERR_TIMEOUT (the request stays pending),
 * FFA_ERR_DEVICE (the request's launch failed; other requests are
 * unaffected). */
ffa_status ffa_server_wait(ffa_server s, int64_t ticket, int64_t timeout_us,
                           float* host_snr, int32_t* host_width,
                           double* latency_s);

/* Stops admitting, lets the running requests finish, frees the pool and the
 * streams.  Requests not yet collected are dropped. */
ffa_status ffa_server_destroy(ffa_server s);

/* Test hook for the failure path of ffa_server_wait: the request with this
 * ticket (issued already or later) fails with FFA_ERR_DEVICE when it is
 * admitted, before any of its work is enqueued, as a launch the runtime
 * refused would; every other request is served as usual.  Errors:
 * FFA_ERR_INVALID (null server, ticket <= 0). */
ffa_status ffa_debug_server_fail(ffa_server s, int64_t ticket);

const char* ffa_status_str(ffa_status st);
const char* ffa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FFA_H_ */
