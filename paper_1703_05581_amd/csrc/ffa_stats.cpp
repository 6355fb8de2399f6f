// False-alarm statistics (Sec. 4.1.2): the S/N histogram entry point and the
// host-side mapping of its counts to Gaussian-equivalent sigma.
#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

#include "ffa.h"
#include "ffa_internal.h"

namespace {

using ffa::fail;

// Probability that a standard normal variable exceeds x.
double normal_sf(double x) { return 0.5 * std::erfc(x / std::sqrt(2.0)); }

// The x with normal_sf(x) = q, 0 < q < 1, by bisection: normal_sf falls
// monotonically, and 200 halvings of [-40, 40] reach the spacing of doubles.
double normal_isf(double q) {
  if (q <= 0.0) return std::numeric_limits<double>::infinity();
  if (q >= 1.0) return -std::numeric_limits<double>::infinity();
  double lo = -40.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (normal_sf(mid) > q)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

// tail[b] = counts in bins b..n_bins-1
std::vector<uint64_t> tails(const uint64_t* hist, int32_t n_bins) {
  std::vector<uint64_t> t(n_bins);
  uint64_t acc = 0;
  for (int32_t b = n_bins - 1; b >= 0; --b) {
    acc += hist[b];
    t[b] = acc;
  }
  return t;
}

}  // namespace

extern "C" ffa_status ffa_snr_histogram(const float* d_snr, int64_t n, float lo, float bins_per_unit,
                                        int32_t n_bins, uint64_t* d_hist, void* stream) {
  if (!d_hist || (n > 0 && !d_snr)) return fail(FFA_ERR_INVALID, "null argument");
  if (n < 0) return fail(FFA_ERR_INVALID, "n must be >= 0");
  if (n_bins < 1 || n_bins > ffa::kHistMaxBins) return fail(FFA_ERR_INVALID, "n_bins must be in 1..16384");
  if (!std::isfinite(lo) || !std::isfinite(bins_per_unit) || !(bins_per_unit > 0.0f))
    return fail(FFA_ERR_INVALID, "lo and bins_per_unit must be finite, bins_per_unit > 0");
  return ffa::check_hip(ffa::launch_snr_histogram(d_snr, n, lo, bins_per_unit, n_bins, d_hist,
                                                  reinterpret_cast<hipStream_t>(stream)),
                        "histogram kernel");
}

extern "C" ffa_status ffa_sigma_gauss(const uint64_t* hist, int32_t n_bins, double* sigma) {
  if (!hist || !sigma) return fail(FFA_ERR_INVALID, "null argument");
  if (n_bins < 1) return fail(FFA_ERR_INVALID, "n_bins must be >= 1");
  const std::vector<uint64_t> t = tails(hist, n_bins);
  if (t[0] == 0) return fail(FFA_ERR_INVALID, "empty histogram");
  const double total = (double)t[0];
  for (int32_t b = 0; b < n_bins; ++b) sigma[b] = normal_isf((double)t[b] / total);
  return FFA_OK;
}

extern "C" ffa_status ffa_sigma_threshold(const uint64_t* hist, int32_t n_bins, float lo, float bins_per_unit,
                                          double sigma, double* snr) {
  if (!hist || !snr) return fail(FFA_ERR_INVALID, "null argument");
  if (n_bins < 1) return fail(FFA_ERR_INVALID, "n_bins must be >= 1");
  if (!std::isfinite(sigma)) return fail(FFA_ERR_INVALID, "sigma must be finite");
  const std::vector<uint64_t> t = tails(hist, n_bins);
  if (t[0] == 0) return fail(FFA_ERR_INVALID, "empty histogram");
  const double limit = normal_sf(sigma) * (double)t[0];
  for (int32_t b = 1; b < n_bins; ++b) {
    if ((double)t[b] <= limit) {
      *snr = (double)lo + (double)b / (double)bins_per_unit;
      return FFA_OK;
    }
  }
  return fail(FFA_ERR_INVALID, "the top bin holds more than the allowed fraction; widen the histogram");
}
