/* Host sanitizer driver for the CPU oracle (test infrastructure).
 *
 * Built with AddressSanitizer and UndefinedBehaviorSanitizer together with
 * oracle/ffa_oracle.c, it calls every exported oracle routine on seeded
 * random small inputs -- plans, octave downsampling, folds, both scores,
 * dereddening (exact and knots, windows shorter and longer than the series),
 * whole searches of float32 and uint8 series, sifting and the S/N histogram
 * -- so that an out-of-bounds access, a use after free or undefined
 * arithmetic anywhere on those paths stops the run.  Prints one summary
 * line; exits 0 when every call returned as documented. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_plan(int64_t N, double tsamp, double pmin, double pmax, int32_t bins_min, int32_t max_octaves,
                int32_t cap, int32_t* f_out, int32_t* P0_out, int32_t* m_out, int32_t* M_out, int64_t* first_out);
void oracle_downsample_f64(const double* x, int64_t n, int32_t octave, double* out);
void oracle_downsample_i64(const int64_t* x, int64_t n, int32_t octave, int64_t* out);
void oracle_fold_f64(const double* x, int32_t P0, int32_t m, int32_t M, double* out);
void oracle_fold_i64(const int64_t* x, int32_t P0, int32_t m, int32_t M, int64_t* out);
double oracle_alg1_f64(const double* F, int32_t P0, const int32_t* widths, int32_t nw, int32_t* best_w);
double oracle_alg1_i64(const int64_t* F, int32_t P0, const int32_t* widths, int32_t nw, int32_t* best_w);
double oracle_alg2_f64(const double* F, int32_t P0, const int32_t* widths, int32_t nw, int32_t* best_w);
double oracle_alg2_i64(const int64_t* F, int32_t P0, const int32_t* widths, int32_t nw, int32_t* best_w);
int32_t oracle_default_widths(int32_t P0, int32_t* w);
int oracle_score_profiles(const double* profiles, int64_t n, int32_t P0, const int32_t* widths, int32_t nw,
                          int32_t alg, int32_t threads, float* snr);
int32_t oracle_dered_default_window(double tsamp, double pmin, double pmax);
int oracle_deredden_f64(const double* x, int64_t n, int32_t window, int32_t stride, double* out);
int oracle_search(const void* series, int32_t dtype, int64_t N, int32_t n_steps, const int32_t* f_arr,
                  const int32_t* P0_arr, const int32_t* m_arr, const int32_t* M_arr, const int64_t* first_arr,
                  int32_t n_sel, const int32_t* sel, const int32_t* widths, int32_t nw, int32_t alg,
                  int32_t threads, int32_t dered_window, int32_t dered_stride, float* snr, int32_t* width);
int oracle_fold_step(const void* series, int32_t dtype, int64_t N, int32_t f, int32_t P0, int32_t m, int32_t M,
                     int32_t dered_window, int32_t dered_stride, void* out);
int64_t oracle_sift(const float* snr, const int32_t* width, int64_t n_trials, int32_t n_steps,
                    const int32_t* f_arr, const int32_t* P0_arr, const int32_t* m_arr, const int32_t* M_arr,
                    const int64_t* first_arr, double tsamp, float min_snr, float frac_fall, float abs_fall,
                    float group_widths, int32_t harmonic_primes, float harmonic_tol, int64_t* out_trial,
                    double* out_period, float* out_snr, int32_t* out_width);
void oracle_snr_histogram(const float* snr, int64_t n, float lo, float bins_per_unit, int32_t n_bins,
                          uint64_t* hist);

static uint64_t g_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_u64(void) { /* splitmix64 */
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static int64_t irange(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }
static double unif(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }
static double gauss(void) {
  double u = unif() + 1e-300, v = unif();
  return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
}

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      g_fail = 1;                                                     \
    }                                                                 \
  } while (0)

static void scores(void) {
  for (int it = 0; it < 400; ++it) {
    int32_t P0 = (int32_t)irange(1, 300);
    double* F = malloc(sizeof(double) * (size_t)P0);
    int64_t* I = malloc(sizeof(int64_t) * (size_t)P0);
    int kind = (int)irange(0, 2); /* noise, flat, spike */
    for (int32_t j = 0; j < P0; ++j) {
      F[j] = kind == 1 ? 3.0 : gauss();
      I[j] = kind == 1 ? 7 : irange(0, 4000);
    }
    if (kind == 2) {
      F[irange(0, P0 - 1)] += 50.0;
      I[irange(0, P0 - 1)] += 90000;
    }
    int32_t w[32], nw = oracle_default_widths(P0, w);
    for (int32_t k = 0; k < nw; ++k)
      if (w[k] > P0) w[k] = P0;
    int32_t bw = -1;
    double a = oracle_alg1_f64(F, P0, w, nw, &bw);
    CHECK(isfinite(a) && bw >= 0 && bw <= P0);
    a = oracle_alg1_i64(I, P0, w, nw, &bw);
    CHECK(isfinite(a) && bw >= 0 && bw <= P0);
    a = oracle_alg2_f64(F, P0, w, nw, &bw);
    CHECK(isfinite(a) && bw >= 0 && bw <= P0);
    a = oracle_alg2_i64(I, P0, w, nw, &bw);
    CHECK(isfinite(a) && bw >= 0 && bw <= P0);
    float s[3];
    double* rows = malloc(sizeof(double) * (size_t)P0 * 3);
    for (int32_t j = 0; j < 3 * P0; ++j) rows[j] = gauss();
    CHECK(oracle_score_profiles(rows, 3, P0, NULL, 0, 1 + (it & 1), 1, s) == 0);
    free(rows);
    free(F);
    free(I);
  }
}

static void dered_and_downsample(void) {
  for (int it = 0; it < 120; ++it) {
    int64_t n = irange(1, 3000);
    double* x = malloc(sizeof(double) * (size_t)n);
    double* y = malloc(sizeof(double) * (size_t)n);
    int64_t* xi = malloc(sizeof(int64_t) * (size_t)n);
    int64_t* yi = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
      x[i] = (it % 5 == 0) ? (double)(i % 3) : gauss() + 0.01 * (double)i;
      xi[i] = irange(0, 255);
    }
    int32_t window = (int32_t)irange(1, 2 * (int32_t)n + 5);
    int32_t stride = (int32_t)irange(0, 3) == 3 ? (int32_t)irange(2, window + 3) : (int32_t)irange(0, 1);
    CHECK(oracle_deredden_f64(x, n, window, stride, y) == 0);
    for (int64_t i = 0; i < n; ++i) CHECK(isfinite(y[i]));
    int32_t oct = (int32_t)irange(0, 6);
    oracle_downsample_f64(x, n, oct, y);
    oracle_downsample_i64(xi, n, oct, yi);
    free(x);
    free(y);
    free(xi);
    free(yi);
  }
  CHECK(oracle_dered_default_window(5e-4, 0.5, 30.0) > 0);
}

static void searches(void) {
  for (int it = 0; it < 60; ++it) {
    int64_t N = irange(64, 6000);
    int32_t B = (int32_t)irange(2, 40);
    double tsamp = 1e-3;
    double pmin = B * tsamp * (1.0 + unif());
    double pmax = pmin * (1.5 + 6.0 * unif());
    int32_t ns = oracle_plan(N, tsamp, pmin, pmax, B, 0, 0, NULL, NULL, NULL, NULL, NULL);
    if (ns <= 0) continue;
    int32_t *f = malloc(4 * (size_t)ns), *P0 = malloc(4 * (size_t)ns), *m = malloc(4 * (size_t)ns),
            *M = malloc(4 * (size_t)ns);
    int64_t* first = malloc(8 * (size_t)ns);
    CHECK(oracle_plan(N, tsamp, pmin, pmax, B, 0, ns, f, P0, m, M, first) == ns);
    int64_t trials = first[ns - 1] + M[ns - 1];
    int dtype = (int)(it & 1);
    void* series = malloc(dtype ? (size_t)N : 4 * (size_t)N);
    for (int64_t i = 0; i < N; ++i) {
      if (dtype)
        ((uint8_t*)series)[i] = (uint8_t)irange(0, 255);
      else
        ((float*)series)[i] = (float)gauss();
    }
    float* snr = malloc(sizeof(float) * (size_t)trials);
    int32_t* wid = malloc(sizeof(int32_t) * (size_t)trials);
    int32_t widths[4] = {1, 2, 3, 5};
    int32_t dw = (it % 3 == 0) ? (int32_t)irange(1, 400) : 0;
    int32_t dst = dw ? (int32_t)irange(0, 9) : 0;
    int32_t alg = 1 + (int32_t)((it >> 1) & 1);
    int use_w = it % 4 == 1 && B >= 5;
    CHECK(oracle_search(series, dtype, N, ns, f, P0, m, M, first, 0, NULL, use_w ? widths : NULL, use_w ? 4 : 0,
                        alg, 1, dw, dst, snr, wid) == 0);
    for (int32_t s = 0; s < ns; s += 1 + ns / 4) {
      size_t cells = (size_t)M[s] * (size_t)P0[s];
      void* prof = malloc(8 * cells);
      CHECK(oracle_fold_step(series, dtype, N, f[s], P0[s], m[s], M[s], dw, dst, prof) == 0);
      free(prof);
    }
    int64_t* ot = malloc(8 * (size_t)trials);
    double* op = malloc(8 * (size_t)trials);
    float* os = malloc(4 * (size_t)trials);
    int32_t* ow = malloc(4 * (size_t)trials);
    int64_t nc = oracle_sift(snr, wid, trials, ns, f, P0, m, M, first, tsamp, 2.0f, 0.1f, 0.5f, 1.0f, 7, 2e-3f,
                             ot, op, os, ow);
    CHECK(nc >= 0 && nc <= trials);
    uint64_t hist[64] = {0};
    if (trials > 2) snr[1] = NAN;
    oracle_snr_histogram(snr, trials, -2.0f, 4.0f, 64, hist);
    free(ot);
    free(op);
    free(os);
    free(ow);
    free(snr);
    free(wid);
    free(series);
    free(f);
    free(P0);
    free(m);
    free(M);
    free(first);
  }
  CHECK(oracle_plan(1, 1e-3, 0.1, 0.2, 10, 0, 0, NULL, NULL, NULL, NULL, NULL) == -1);
}

int main(void) {
  scores();
  dered_and_downsample();
  searches();
  printf("oracle host check: %s\n", g_fail ? "FAILED" : "ok");
  return g_fail;
}
