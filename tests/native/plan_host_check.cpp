// Host sanitizer driver for the library's host code (test infrastructure).
//
// Built with AddressSanitizer and UndefinedBehaviorSanitizer on the host
// side of every library source, it drives the calls that need no GPU --
// plan creation with random descriptions and launch options (valid and
// not), the plan's queries, periods and queue tables, batch planning over
// random sets of plans, the false-alarm statistics and the host-side
// argument checks of the device calls -- so that an out-of-bounds access,
// a use after free, a leak or undefined arithmetic in the planner, the work
// queue builder or the batch planner stops the run.  Prints one summary
// line; exits 0 when every call returned as documented.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "ffa.h"

typedef struct ffa_batch_s* ffa_batch;
extern "C" {
int64_t ffa_debug_phases(ffa_plan p, void* out, int64_t cap);
int64_t ffa_debug_layout(ffa_plan p, int64_t* out, int64_t cap);
int64_t ffa_debug_batch(ffa_batch b, int32_t c, void* phases, int64_t cap, int64_t* layout, int64_t lcap);
int64_t ffa_debug_batch_series_base(ffa_batch b, int32_t i);
}

namespace {

uint64_t g_state = 0x2545f4914f6cdd1dull;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
int64_t irange(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }
double unif() { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

int g_fail = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      g_fail = 1;                                                         \
    }                                                                     \
  } while (0)

bool known_status(ffa_status s) { return s <= 0 && s >= FFA_ERR_TIMEOUT; }

// Walks everything a plan reports on the host.
void inspect(ffa_plan p) {
  int64_t nt = 0;
  int32_t ns = 0;
  size_t ws = 0;
  CHECK(ffa_plan_query(p, &nt, &ns, &ws) == FFA_OK);
  CHECK(nt > 0 && ns > 0 && ws > 0);
  int64_t trials = 0;
  for (int32_t s = 0; s < ns; ++s) {
    int32_t f, P0, m, M, np, depths[8];
    int64_t first;
    CHECK(ffa_plan_step(p, s, &f, &P0, &m, &M, &first) == FFA_OK);
    CHECK(first == trials && m >= 2 && M >= m && M < 2 * m);
    trials += M;
    CHECK(ffa_plan_passes(p, s, &np, depths) == FFA_OK);
    int32_t lv = 0;
    for (int32_t i = 0; i < np; ++i) lv += depths[i];
    CHECK(np >= 1 && np <= 8 && (1 << lv) == M);
  }
  CHECK(trials == nt);
  CHECK(ffa_plan_step(p, ns, nullptr, nullptr, nullptr, nullptr, nullptr) == FFA_ERR_INVALID);
  CHECK(ffa_plan_step(p, -1, nullptr, nullptr, nullptr, nullptr, nullptr) == FFA_ERR_INVALID);
  std::vector<double> per((size_t)nt);
  CHECK(ffa_plan_periods(p, per.data()) == FFA_OK);
  for (int64_t i = 0; i < nt; ++i) CHECK(per[(size_t)i] > 0.0 && std::isfinite(per[(size_t)i]));
  const int64_t nph = ffa_debug_phases(p, nullptr, 0);
  CHECK(nph > 0);
  std::vector<unsigned char> ph((size_t)nph * 104);
  CHECK(ffa_debug_phases(p, ph.data(), nph) == nph);
  const int64_t need = ffa_debug_layout(p, nullptr, 0);
  CHECK(need >= 8);
  std::vector<int64_t> lay((size_t)need);
  CHECK(ffa_debug_layout(p, lay.data(), need) == need);
}

ffa_plan random_plan(bool valid_only) {
  std::vector<int32_t> widths;
  ffa_plan_desc d{};
  d.N = irange(0, 9) == 0 ? irange(-5, 200) : irange(256, (int64_t)1 << 22);
  d.tsamp_s = irange(0, 30) == 0 ? 0.0 : 1e-3 * (0.2 + unif());
  d.bins_min = (int32_t)(irange(0, 20) == 0 ? irange(-3, 1100) : irange(2, 600));
  d.pmin_s = d.bins_min * d.tsamp_s * (0.5 + 2.0 * unif());
  d.pmax_s = d.pmin_s * (irange(0, 25) == 0 ? 0.9 : 1.01 + 20.0 * unif());
  const int64_t nw = irange(0, 4) == 0 ? 0 : irange(1, irange(0, 30) == 0 ? 33 : 10);
  for (int64_t i = 0; i < nw; ++i) widths.push_back((int32_t)(irange(0, 40) == 0 ? irange(-2, 0) : irange(1, 70)));
  d.widths = widths.empty() ? nullptr : widths.data();
  d.n_widths = (int32_t)widths.size();
  d.max_octaves = (int32_t)(irange(0, 3) == 0 ? irange(-1, 5) : 0);
  d.dtype = (int32_t)(irange(0, 40) == 0 ? 2 : irange(0, 1));
  d.snr = (int32_t)(irange(0, 40) == 0 ? 0 : irange(1, 2));
  d.dered_window = (int32_t)(irange(0, 2) == 0 ? irange(-2, 5000) : 0);
  d.dered_stride = (int32_t)(d.dered_window ? irange(-1, 40) : 0);
  ffa_plan_opts o{};
  const bool use_opts = irange(0, 1) == 1;
  if (use_opts) {
    o.tile_lds_bytes = (int32_t)(irange(0, 10) == 0 ? irange(-1, 200000) : irange(0, 1) * irange(16384, 163840));
    o.window_tiles = (int32_t)(irange(0, 2) == 0 ? irange(1, 5000) : 0);
    o.ring_mb = (int32_t)(irange(0, 2) == 0 ? irange(1, 64) : 0);
    o.steps_per_window = (int32_t)(irange(0, 4) == 0 ? irange(1, 7) : 0);
    o.no_u16 = (int32_t)irange(0, 1);
    o.no_split_occupancy = (int32_t)irange(0, 1);
    o.select_iters = (int32_t)(irange(0, 4) == 0 ? irange(-1, 64) : 0);
    o.select_cand = (int32_t)(irange(0, 4) == 0 ? irange(0, 70) : 0);
  }
  ffa_plan p = nullptr;
  const ffa_status st = ffa_plan_create_opts(&d, use_opts ? &o : nullptr, &p);
  CHECK(known_status(st));
  CHECK((st == FFA_OK) == (p != nullptr));
  if (st != FFA_OK) CHECK(ffa_last_error()[0] != '\0');
  (void)valid_only;
  return p;
}

void batches(const std::vector<ffa_plan>& pool) {
  for (int it = 0; it < 40 && !pool.empty(); ++it) {
    const int32_t n = (int32_t)irange(1, 12);
    std::vector<ffa_plan> pick;
    for (int32_t i = 0; i < n; ++i) pick.push_back(pool[(size_t)irange(0, (int64_t)pool.size() - 1)]);
    size_t ws = 0;
    CHECK(ffa_batch_workspace(n, pick.data(), &ws) == FFA_OK && ws > 0);
    ffa_batch b = nullptr;
    CHECK(ffa_batch_create(n, pick.data(), &b) == FFA_OK);
    if (!b) continue;
    size_t ws2 = 0;
    int64_t tiles = 0;
    int32_t launches = 0;
    CHECK(ffa_batch_query(b, &ws2, &tiles, &launches) == FFA_OK);
    CHECK(ws2 == ws && tiles > 0 && launches > 0);
    for (int32_t c = 0;; ++c) {
      const int64_t nph = ffa_debug_batch(b, c, nullptr, 0, nullptr, 0);
      if (nph < 0) break;
      std::vector<unsigned char> ph((size_t)nph * 104);
      std::vector<int64_t> lay(8 + 4 * (size_t)launches);
      CHECK(ffa_debug_batch(b, c, ph.data(), nph, lay.data(), (int64_t)lay.size()) == nph);
    }
    for (int32_t i = 0; i < n; ++i) CHECK(ffa_debug_batch_series_base(b, i) >= 0);
    CHECK(ffa_debug_batch_series_base(b, n) == -1);
    CHECK(ffa_batch_destroy(b) == FFA_OK);
  }
  ffa_batch b = nullptr;
  CHECK(ffa_batch_create(0, pool.data(), &b) == FFA_ERR_INVALID);
  std::vector<ffa_plan> with_null{pool.empty() ? nullptr : pool[0], nullptr};
  CHECK(ffa_batch_create(2, with_null.data(), &b) == FFA_ERR_INVALID);
}

void statistics() {
  for (int it = 0; it < 200; ++it) {
    const int32_t nb = (int32_t)irange(1, 300);
    std::vector<uint64_t> h((size_t)nb);
    for (auto& v : h) v = irange(0, 3) == 0 ? 0 : (uint64_t)irange(0, 100000);
    std::vector<double> sig((size_t)nb);
    CHECK(known_status(ffa_sigma_gauss(h.data(), nb, sig.data())));
    double snr = 0.0;
    CHECK(known_status(ffa_sigma_threshold(h.data(), nb, -2.0f, 8.0f, 1.0 + 5.0 * unif(), &snr)));
  }
  CHECK(ffa_sigma_gauss(nullptr, 4, nullptr) == FFA_ERR_INVALID);
}

void argument_checks(ffa_plan p) {
  // refused on the host, before any device call
  CHECK(ffa_search(p, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == FFA_ERR_INVALID);
  CHECK(ffa_search(nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == FFA_ERR_INVALID);
  CHECK(ffa_plan_query(nullptr, nullptr, nullptr, nullptr) == FFA_ERR_INVALID);
  CHECK(ffa_plan_destroy(nullptr) == FFA_ERR_INVALID);
  ffa_server s = nullptr;
  CHECK(ffa_server_create(1 << 20, 0, 0, &s) == FFA_ERR_INVALID);
  CHECK(ffa_server_create(1 << 20, 2, -1, &s) == FFA_ERR_INVALID);
  int64_t t = 0;
  CHECK(ffa_server_submit(nullptr, p, nullptr, 0, nullptr, &t) == FFA_ERR_INVALID);
  CHECK(ffa_debug_server_fail(nullptr, 1) == FFA_ERR_INVALID);
  for (int k = -8; k <= 1; ++k) CHECK(ffa_status_str((ffa_status)k) != nullptr);
}

}  // namespace

int main() {
  std::vector<ffa_plan> pool;
  int made = 0, refused = 0;
  for (int it = 0; it < 600; ++it) {
    ffa_plan p = random_plan(false);
    if (!p) {
      ++refused;
      continue;
    }
    ++made;
    inspect(p);
    if (pool.size() < 16)
      pool.push_back(p);
    else
      CHECK(ffa_plan_destroy(p) == FFA_OK);
  }
  batches(pool);
  statistics();
  argument_checks(pool.empty() ? nullptr : pool[0]);
  for (ffa_plan p : pool) CHECK(ffa_plan_destroy(p) == FFA_OK);
  std::printf("library host check: %s (%d plans made, %d refused)\n", g_fail ? "FAILED" : "ok", made, refused);
  return g_fail;
}
