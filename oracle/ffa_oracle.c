/*
 * ffa_oracle.c -- plain CPU reference of the FFA periodicity search with
 * boxcar S/N evaluation (Cameron et al. 2017, "An investigation of pulsar
 * searching techniques with the Fast Folding Algorithm").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * Arithmetic: float input is carried in double precision; uint8 input is
 * carried in int64, so folded profiles are exact integers.  The code follows
 * the definitions step by step and is deliberately slow:
 *   - plan      : Sec. 2.1 (trial periods, Eqs. 1-2, with N replaced by the
 *                 padded length M*P0) and Sec. 2.3.1 (automatic octave
 *                 downsampling by 2 each time the period doubles);
 *   - rows      : Sec. 2.1 (pad to a power-of-two row count with zero rows;
 *                 drop the data tail beyond an integer number of rows);
 *   - fold      : the Staelin tree named in Sec. 2.1, level by level;
 *   - Alg. 1    : Sec. 2.2.1 (median/MAD normalisation, Eqs. 3-4; boxcars
 *                 divided by sqrt(width); score = maximum);
 *   - Alg. 2    : Sec. 2.2.2 (boxcar first, 20% exclusion window around the
 *                 maximum, Eq. 5);
 *   - dereddening: Sec. 2.3.1 (running median, default window);
 *   - sifting   : Sec. 2.3.3 (ffa2best's thresholds, grouping, harmonics);
 *   - S/N histogram: Sec. 4.1.2 (false-alarm statistics).
 * Readings of points the paper leaves open are listed next to the code.
 *
 * Parity status: plan, downsampling, fold and Alg. 1 are pinned by the
 * `-m "not gpu"` tests (worked example, closed forms, invariants, library
 * routines, impulse response, injected-pulse recovery).  Alg. 2 is pinned to
 * its stated readings by hand-worked examples, invariances and the top-hat
 * S/N level, and against the paper by its white-noise calibration
 * (Sec. 4.1.2): both algorithms' 5-sigma S/N on white-noise profiles match
 * the paper's 6.6 and 7.1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* sigma = K * MAD (Sec. 2.2.1, Eq. 4).  The paper gives K ~ 1.4826; it is the
 * reciprocal of the normal distribution's 75% quantile, which makes the MAD
 * of normal data an estimate of its standard deviation.  Taken to double
 * precision: 1 / 0.6744897501960817. */
#define ORACLE_K 1.482602218505602

#define ORACLE_IN_F32 0
#define ORACLE_IN_U8 1

#define ORACLE_ALG1 1
#define ORACLE_ALG2 2

/* ------------------------------------------------------------------ plan */

static int32_t next_pow2_i32(int32_t m) {
  int32_t M = 1;
  while (M < m) M <<= 1;
  return M;
}

/* Enumerate the FFA executions ("steps") of a search.
 *
 * Octave o has downsampling factor f = 2^o (Sec. 2.3.1: the series is halved
 * in length each time the trial period doubles).  In each octave the base
 * period P0 (in downsampled bins) takes every integer in [B, 2B) whose period
 * in seconds, P0*f*tsamp, lies in [pmin, pmax).  Per step:
 *   N_f = floor(N / f)             samples after downsampling
 *   m   = floor(N_f / P0)          whole rows of data (tail dropped, Sec. 2.1)
 *   M   = smallest power of two >= m   rows after zero padding (Sec. 2.1)
 * Steps with m < 2 are skipped (the period spacing of Eq. 1 needs two rows).
 * The trials of a step are numbered first_trial + k, k = 0..M-1.
 *
 * Returns the number of steps; when the arrays are non-NULL and the count is
 * at most cap, fills them.  Returns -1 on invalid arguments.
 */
int oracle_plan(int64_t N, double tsamp, double pmin, double pmax,
                int32_t bins_min, int32_t max_octaves, int32_t cap,
                int32_t* f_out, int32_t* P0_out, int32_t* m_out,
                int32_t* M_out, int64_t* first_out) {
  if (N < 2 || !(tsamp > 0) || !(pmin > 0) || !(pmax > pmin) || bins_min < 1)
    return -1;
  int32_t count = 0;
  int64_t trials = 0;
  for (int32_t o = 0; o < 62; ++o) {
    if (max_octaves > 0 && o >= max_octaves) break;
    int64_t f = (int64_t)1 << o;
    if ((double)bins_min * (double)f * tsamp >= pmax) break;
    int64_t Nf = N / f;
    if (Nf < 2 * (int64_t)bins_min) break;
    for (int32_t P0 = bins_min; P0 < 2 * bins_min; ++P0) {
      double p = (double)P0 * (double)f * tsamp;
      if (p < pmin || p >= pmax) continue;
      int64_t m = Nf / P0;
      if (m < 2) continue;
      int32_t M = next_pow2_i32((int32_t)m);
      if (f_out && count < cap) {
        f_out[count] = (int32_t)f;
        P0_out[count] = P0;
        m_out[count] = (int32_t)m;
        M_out[count] = M;
        first_out[count] = trials;
      }
      ++count;
      trials += M;
    }
  }
  return count;
}

/* ----------------------------------------------------------- downsample */

/* One halving of the time resolution (Sec. 2.3.1): y[i] = x[2i] + x[2i+1]
 * for i < floor(n/2); an odd last sample is dropped.  A sum rather than a
 * mean: the two differ by an exact power of two, and both S/N algorithms are
 * invariant to a positive scale. */
static void halve_f64(const double* x, int64_t n, double* y) {
  for (int64_t i = 0; i < n / 2; ++i) y[i] = x[2 * i] + x[2 * i + 1];
}

static void halve_i64(const int64_t* x, int64_t n, int64_t* y) {
  for (int64_t i = 0; i < n / 2; ++i) y[i] = x[2 * i] + x[2 * i + 1];
}

/* Series at factor f = 2^o built by o successive halvings. */
void oracle_downsample_f64(const double* x, int64_t n, int32_t octave,
                           double* out) {
  double* cur = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* nxt = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  memcpy(cur, x, sizeof(double) * (size_t)n);
  int64_t len = n;
  for (int32_t o = 0; o < octave; ++o) {
    halve_f64(cur, len, nxt);
    len /= 2;
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  memcpy(out, cur, sizeof(double) * (size_t)len);
  free(cur);
  free(nxt);
}

void oracle_downsample_i64(const int64_t* x, int64_t n, int32_t octave,
                           int64_t* out) {
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* nxt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  memcpy(cur, x, sizeof(int64_t) * (size_t)n);
  int64_t len = n;
  for (int32_t o = 0; o < octave; ++o) {
    halve_i64(cur, len, nxt);
    len /= 2;
    int64_t* t = cur;
    cur = nxt;
    nxt = t;
  }
  memcpy(out, cur, sizeof(int64_t) * (size_t)len);
  free(cur);
  free(nxt);
}

/* ----------------------------------------------------------------- fold */

/* The FFA of one step (Sec. 2.1, after Staelin 1969).
 *
 * Level 0 holds one partial profile per row: row r is x[r*P0 .. r*P0+P0-1]
 * for r < m and all zeros for m <= r < M (zero padding; the data tail beyond
 * m*P0 samples is not used).
 *
 * At level l = 1..L (L = log2 M) the rows are cut into blocks of 2^l.  Each
 * block has a head half A and a tail half B, each holding 2^(l-1) partial
 * profiles from level l-1.  The block's 2^l new partials are
 *
 *     out_t[j] = A_{t/2}[j] + B_{t/2}[(j + ceil(t/2)) mod P0],
 *     t = 0 .. 2^l - 1,  j = 0 .. P0 - 1,
 *
 * i.e. partial t of the block reuses partial t/2 of both halves, and the tail
 * half is rotated left by ceil(t/2) bins.  Rotating left makes the folding
 * period grow with t.  After level L, out_k is the folded profile of trial k,
 * whose period is P0 + k/(M-1) bins (Eq. 2 with N replaced by M*P0).
 *
 * Reading: the paper gives no shift convention.  This one makes trial k drift
 * the last row by exactly k bins relative to the first, the spacing Eq. 1
 * implies for the padded length, and leaves row 0 unshifted.
 */
#define DEFINE_FOLD(NAME, T)                                                   \
  void NAME(const T* x, int32_t P0, int32_t m, int32_t M, T* out) {            \
    size_t cells = (size_t)M * (size_t)P0;                                     \
    T* cur = (T*)calloc(cells, sizeof(T));                                     \
    T* nxt = (T*)calloc(cells, sizeof(T));                                     \
    for (int32_t r = 0; r < m; ++r)                                            \
      for (int32_t j = 0; j < P0; ++j)                                         \
        cur[(size_t)r * P0 + j] = x[(size_t)r * P0 + j];                       \
    for (int32_t half = 1; half < M; half *= 2) {                              \
      int32_t block = 2 * half;                                                \
      for (int32_t b0 = 0; b0 < M; b0 += block) {                              \
        const T* A = cur + (size_t)b0 * P0;                                    \
        const T* B = cur + (size_t)(b0 + half) * P0;                           \
        for (int32_t t = 0; t < block; ++t) {                                  \
          int32_t src = t / 2;                                                 \
          int32_t shift = (t + 1) / 2;                                         \
          T* o = nxt + (size_t)(b0 + t) * P0;                                  \
          for (int32_t j = 0; j < P0; ++j)                                     \
            o[j] = A[(size_t)src * P0 + j] +                                   \
                   B[(size_t)src * P0 + (j + shift) % P0];                     \
        }                                                                      \
      }                                                                        \
      T* tmp = cur;                                                            \
      cur = nxt;                                                               \
      nxt = tmp;                                                               \
    }                                                                          \
    memcpy(out, cur, cells * sizeof(T));                                       \
    free(cur);                                                                 \
    free(nxt);                                                                 \
  }

DEFINE_FOLD(oracle_fold_f64, double)
DEFINE_FOLD(oracle_fold_i64, int64_t)

/* ------------------------------------------------------ Algorithm 1 (f64) */

static int cmp_f64(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* Median of n values (sorted copy).  Even n: mean of the two middle order
 * statistics (reading; the paper does not say). */
static double median_f64(const double* v, int32_t n, double* scratch) {
  memcpy(scratch, v, sizeof(double) * (size_t)n);
  qsort(scratch, (size_t)n, sizeof(double), cmp_f64);
  if (n % 2) return scratch[n / 2];
  return 0.5 * (scratch[n / 2 - 1] + scratch[n / 2]);
}

/* The circular boxcar of width w: out[j] = sum of the w bins starting at bin
 * j, wrapping around the profile (the profile is one period), for every j.
 * Each box is a difference of two running totals of the profile taken
 * twice over: C[k] = F[0] + ... + F[(k-1) mod P0], box = C[j+w] - C[j]
 * (exact for integers). */
static void boxes_f64(const double* F, int32_t P0, int32_t w, double* out) {
  double* C = (double*)malloc(sizeof(double) * (size_t)(P0 + w + 1));
  C[0] = 0.0;
  for (int32_t k = 0; k < P0 + w; ++k) C[k + 1] = C[k] + F[k % P0];
  for (int32_t j = 0; j < P0; ++j) out[j] = C[j + w] - C[j];
  free(C);
}

static void boxes_i64(const int64_t* F, int32_t P0, int32_t w, int64_t* out) {
  int64_t* C = (int64_t*)malloc(sizeof(int64_t) * (size_t)(P0 + w + 1));
  C[0] = 0;
  for (int32_t k = 0; k < P0 + w; ++k) C[k + 1] = C[k] + F[k % P0];
  for (int32_t j = 0; j < P0; ++j) out[j] = C[j + w] - C[j];
  free(C);
}

/* Algorithm 1 (Sec. 2.2.1).  Normalise the profile by its median and K*MAD
 * (Eqs. 3-4), slide a boxcar of each width over every bin position, divide
 * each boxcar sum by sqrt(width), and keep the maximum.  Written without the
 * explicit normalised copy: (sum_w(F) - w*med) / (K*MAD*sqrt(w)) is the
 * boxcar sum of the normalised profile divided by sqrt(w).
 * Widths larger than the profile are skipped.  MAD = 0 gives score 0 and
 * width 0 (reading: the normalisation is undefined).  Ties between widths
 * keep the first width in the given order. */
double oracle_alg1_f64(const double* F, int32_t P0, const int32_t* widths,
                       int32_t nw, int32_t* best_w) {
  double* tmp = (double*)malloc(sizeof(double) * (size_t)P0);
  double* dev = (double*)malloc(sizeof(double) * (size_t)P0);
  double med = median_f64(F, P0, tmp);
  for (int32_t j = 0; j < P0; ++j) dev[j] = fabs(F[j] - med);
  double mad = median_f64(dev, P0, tmp);
  free(tmp);
  free(dev);
  *best_w = 0;
  if (mad == 0.0) return 0.0;
  double sigma = ORACLE_K * mad;
  double best = 0.0;
  int have = 0;
  double* bx = (double*)malloc(sizeof(double) * (size_t)P0);
  for (int32_t wi = 0; wi < nw; ++wi) {
    int32_t w = widths[wi];
    if (w < 1 || w > P0) continue;
    boxes_f64(F, P0, w, bx);
    double peak = bx[0];
    for (int32_t j = 1; j < P0; ++j)
      if (bx[j] > peak) peak = bx[j];
    double snr = (peak - (double)w * med) / (sigma * sqrt((double)w));
    if (!have || snr > best) {
      best = snr;
      *best_w = w;
      have = 1;
    }
  }
  free(bx);
  return have ? best : 0.0;
}

/* Algorithm 1 on an exact integer profile (uint8 input).  The median and MAD
 * of integers are multiples of 1/2 and 1/4, so the score is formed from
 * exact integers before any rounding:
 *   med2 = 2*median,  mad4 = 4*MAD,
 *   S/N_w = (peak_w - w*median) / (K*MAD*sqrt(w))
 *         = 2*(2*peak_w - w*med2) / (K*mad4*sqrt(w)),
 * evaluated in double as num / ((K*mad4)*sqrt(w)).  Every operation there is
 * correctly rounded, so the result is a fixed function of the integers. */
double oracle_alg1_i64(const int64_t* F, int32_t P0, const int32_t* widths,
                       int32_t nw, int32_t* best_w) {
  int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)P0);
  memcpy(tmp, F, sizeof(int64_t) * (size_t)P0);
  qsort(tmp, (size_t)P0, sizeof(int64_t), cmp_i64);
  int64_t med2 = (P0 % 2) ? 2 * tmp[P0 / 2] : tmp[P0 / 2 - 1] + tmp[P0 / 2];
  /* |2F - med2| = 2*|F - median| */
  for (int32_t j = 0; j < P0; ++j) {
    int64_t d = 2 * F[j] - med2;
    tmp[j] = d < 0 ? -d : d;
  }
  qsort(tmp, (size_t)P0, sizeof(int64_t), cmp_i64);
  int64_t mad4 = (P0 % 2) ? 2 * tmp[P0 / 2] : tmp[P0 / 2 - 1] + tmp[P0 / 2];
  free(tmp);
  *best_w = 0;
  if (mad4 == 0) return 0.0;
  double best = 0.0;
  int have = 0;
  int64_t* bx = (int64_t*)malloc(sizeof(int64_t) * (size_t)P0);
  for (int32_t wi = 0; wi < nw; ++wi) {
    int32_t w = widths[wi];
    if (w < 1 || w > P0) continue;
    boxes_i64(F, P0, w, bx);
    int64_t peak = bx[0];
    for (int32_t j = 1; j < P0; ++j)
      if (bx[j] > peak) peak = bx[j];
    int64_t num = 2 * (2 * peak - (int64_t)w * med2);
    double den = (ORACLE_K * (double)mad4) * sqrt((double)w);
    double snr = (double)num / den;
    if (!have || snr > best) {
      best = snr;
      *best_w = w;
      have = 1;
    }
  }
  free(bx);
  return have ? best : 0.0;
}

/* ------------------------------------------------------ Algorithm 2 (f64) */

/* Algorithm 2 (Sec. 2.2.2, Eq. 5): the boxcar first, then the off-pulse
 * statistics.  For each width w:
 *   - B_w[j] = sum of the w profile bins from bin j (circular), I_max its
 *     maximum, at the first position j* where it occurs;
 *   - the on-pulse window: L = max(round(P0/5), w) profile bins centred on
 *     the box that gave I_max (bins j* .. j*+w-1, centre j* + (w-1)/2), so
 *     starting at bin j* + floor((w - L)/2), wrapping: 20% of the profile,
 *     or the box itself where it is wider;
 *   - I_av and sigma: mean and population standard deviation of the profile
 *     bins outside the window (the remaining 80%);
 *   - A_w = (I_max - w*I_av) / (sigma*sqrt(w)): Eq. 5 for the boxcar sum,
 *     whose off-pulse level is w*I_av and whose noise is sigma*sqrt(w).
 * A_2 = max over widths (first width on ties); sigma = 0 (a flat off-pulse
 * region, or no two bins left outside the window) gives 0.
 * Readings: the paper names the quantities, not the profile they are taken
 * from, the window's placement or the normalisation of the boxcar.  These
 * readings reproduce its white-noise calibration (Sec. 4.1.2: a 5-sigma
 * detection at S/N 7.1), which statistics of the filtered profile do not.
 * The "Ref" variant of Sec. 2.2.2 and Sec. 2.4 is this with one width. */

/* The on-pulse window of a box of width w at j*: first bin and length. */
static void alg2_window(int32_t P0, int32_t jstar, int32_t w, int32_t* start, int32_t* len) {
  const int32_t n_ex = (2 * P0 + 5) / 10; /* round(P0/5) */
  const int32_t L = w > n_ex ? w : n_ex;
  int32_t d = w - L; /* <= 0: floor((w - L)/2) */
  int32_t st = jstar + (d - (d & 1)) / 2;
  *start = ((st % P0) + P0) % P0;
  *len = L;
}

double oracle_alg2_f64(const double* F, int32_t P0, const int32_t* widths,
                       int32_t nw, int32_t* best_w) {
  char* excl = (char*)malloc((size_t)P0);
  double* bx = (double*)malloc(sizeof(double) * (size_t)P0);
  double best = 0.0;
  int have = 0;
  *best_w = 0;
  for (int32_t wi = 0; wi < nw; ++wi) {
    int32_t w = widths[wi];
    if (w < 1 || w > P0) continue;
    boxes_f64(F, P0, w, bx);
    int32_t jmax = 0;
    double imax = bx[0];
    for (int32_t j = 1; j < P0; ++j) {
      double b = bx[j];
      if (b > imax) {
        imax = b;
        jmax = j;
      }
    }
    int32_t start, L;
    alg2_window(P0, jmax, w, &start, &L);
    memset(excl, 0, (size_t)P0);
    for (int32_t i = 0; i < L && i < P0; ++i) excl[(start + i) % P0] = 1;
    double s = 0.0;
    int32_t cnt = 0;
    for (int32_t j = 0; j < P0; ++j)
      if (!excl[j]) {
        s += F[j];
        ++cnt;
      }
    double a = 0.0;
    if (cnt > 1) {
      double mean = s / cnt;
      double v = 0.0;
      for (int32_t j = 0; j < P0; ++j)
        if (!excl[j]) v += (F[j] - mean) * (F[j] - mean);
      double sd = sqrt(v / cnt);
      a = sd > 0.0 ? (imax - (double)w * mean) / (sd * sqrt((double)w)) : 0.0;
    }
    if (!have || a > best) {
      best = a;
      *best_w = w;
      have = 1;
    }
  }
  free(excl);
  free(bx);
  return have ? best : 0.0;
}

/* Algorithm 2 on an exact integer profile (uint8 input).  With c kept bins,
 * s1 their sum and s2 their sum of squares, I_av = s1/c and
 * sigma = sqrt(c*s2 - s1^2)/c, so
 *   A_w = (c*I_max - w*s1) / (sqrt(c*s2 - s1^2) * sqrt(w)),
 * formed from exact integers (each below 2^63 for the sums a plan allows)
 * and evaluated in double as num / (sqrt(D) * sqrt(w)). */
double oracle_alg2_i64(const int64_t* F, int32_t P0, const int32_t* widths,
                       int32_t nw, int32_t* best_w) {
  char* excl = (char*)malloc((size_t)P0);
  int64_t* bx = (int64_t*)malloc(sizeof(int64_t) * (size_t)P0);
  double best = 0.0;
  int have = 0;
  *best_w = 0;
  for (int32_t wi = 0; wi < nw; ++wi) {
    int32_t w = widths[wi];
    if (w < 1 || w > P0) continue;
    boxes_i64(F, P0, w, bx);
    int32_t jmax = 0;
    int64_t imax = bx[0];
    for (int32_t j = 1; j < P0; ++j) {
      int64_t b = bx[j];
      if (b > imax) {
        imax = b;
        jmax = j;
      }
    }
    int32_t start, L;
    alg2_window(P0, jmax, w, &start, &L);
    memset(excl, 0, (size_t)P0);
    for (int32_t i = 0; i < L && i < P0; ++i) excl[(start + i) % P0] = 1;
    int64_t s1 = 0, s2 = 0, c = 0;
    for (int32_t j = 0; j < P0; ++j)
      if (!excl[j]) {
        s1 += F[j];
        s2 += F[j] * F[j];
        ++c;
      }
    double a = 0.0;
    if (c > 1) {
      int64_t D = c * s2 - s1 * s1;
      int64_t num = c * imax - (int64_t)w * s1;
      a = D > 0 ? (double)num / (sqrt((double)D) * sqrt((double)w)) : 0.0;
    }
    if (!have || a > best) {
      best = a;
      *best_w = w;
      have = 1;
    }
  }
  free(excl);
  free(bx);
  return have ? best : 0.0;
}

/* Scores of n profiles of P0 bins each (row-major in `profiles`) with the
 * given algorithm and widths (NULL/0: the default rule for P0), in parallel
 * over profiles (threads <= 0: the OpenMP default).  For the false-alarm
 * statistics of many noise profiles (Sec. 4.1.2). */
int32_t oracle_default_widths(int32_t P0, int32_t* w);
int oracle_score_profiles(const double* profiles, int64_t n, int32_t P0, const int32_t* widths,
                          int32_t nw, int32_t alg, int32_t threads, float* snr) {
  if (n < 0 || P0 < 1 || (alg != ORACLE_ALG1 && alg != ORACLE_ALG2)) return -1;
  int32_t wbuf[32];
  if (!widths || nw <= 0) {
    nw = oracle_default_widths(P0, wbuf);
    widths = wbuf;
  }
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int32_t bw = 0;
    const double* F = profiles + (size_t)i * (size_t)P0;
    snr[i] = (float)(alg == ORACLE_ALG1 ? oracle_alg1_f64(F, P0, widths, nw, &bw)
                                        : oracle_alg2_f64(F, P0, widths, nw, &bw));
  }
  return 0;
}

/* ------------------------------------------------------ dereddening */

/* Default window of the dynamic running-median dereddening (Sec. 2.3.1): the
 * smaller of twice the longest and four times the shortest period searched,
 * in samples of the input series, rounded to the nearest sample. */
int32_t oracle_dered_default_window(double tsamp, double pmin, double pmax) {
  double w = 2.0 * pmax / tsamp;
  double w4 = 4.0 * pmin / tsamp;
  if (w4 < w) w = w4;
  if (w < 1.0) w = 1.0;
  if (w > 2147483647.0) w = 2147483647.0;
  return (int32_t)llround(w);
}

/* Window of the running median at sample i (Sec. 2.3.1, as read here): the
 * `window` samples starting window/2 before i, clipped to the series. */
static void dered_window_at(int64_t i, int64_t n, int32_t window, int64_t* lo, int64_t* hi) {
  int64_t a = i - window / 2, b = a + window;
  *lo = a < 0 ? 0 : a;
  *hi = b > n ? n : b;
}

/* Median of a sorted run of cnt values: the middle one, or the mean of the
 * two middle ones for an even count. */
static double sorted_median(const double* v, int64_t cnt) {
  return cnt % 2 ? v[cnt / 2] : 0.5 * (v[cnt / 2 - 1] + v[cnt / 2]);
}

/* Exact running median of x: med[i] = median of the window at i, for every
 * sample.  The window's values are kept sorted while it slides one sample
 * at a time: the sample that leaves is found by binary search and removed,
 * the one that enters is inserted in order.  The series is cut into chunks
 * (in parallel), each starting from a freshly sorted copy of its first
 * window. */
static void running_median_f64(const double* x, int64_t n, int32_t window, double* med) {
  const int64_t chunk = 16384;
  const int64_t nch = (n + chunk - 1) / chunk;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < nch; ++c) {
    const int64_t i0 = c * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
    int64_t lo, hi;
    dered_window_at(i0, n, window, &lo, &hi);
    /* room for the window, and for one insertion per sample of the chunk */
    double* buf = (double*)malloc(sizeof(double) * (size_t)(window + chunk + 1));
    int64_t cnt = hi - lo;
    memcpy(buf, x + lo, sizeof(double) * (size_t)cnt);
    qsort(buf, (size_t)cnt, sizeof(double), cmp_f64);
    for (int64_t i = i0; i < i1; ++i) {
      med[i] = sorted_median(buf, cnt);
      if (i + 1 == i1) break;
      int64_t lo2, hi2;
      dered_window_at(i + 1, n, window, &lo2, &hi2);
      if (lo2 > lo) { /* x[lo] leaves: remove one entry of its value */
        const double v = x[lo];
        int64_t a = 0, b = cnt; /* first entry >= v */
        while (a < b) {
          int64_t m = (a + b) / 2;
          if (buf[m] < v) a = m + 1;
          else b = m;
        }
        if (a < cnt) { /* always: x[lo] is in the window */
          memmove(buf + a, buf + a + 1, sizeof(double) * (size_t)(cnt - a - 1));
          --cnt;
        }
      }
      if (hi2 > hi) { /* x[hi] enters: insert it in order */
        const double v = x[hi];
        int64_t a = 0, b = cnt; /* first entry > v */
        while (a < b) {
          int64_t m = (a + b) / 2;
          if (buf[m] <= v) a = m + 1;
          else b = m;
        }
        memmove(buf + a + 1, buf + a, sizeof(double) * (size_t)(cnt - a));
        buf[a] = v;
        ++cnt;
      }
      lo = lo2;
      hi = hi2;
    }
    free(buf);
  }
}

/* Running-median dereddening of one series (Sec. 2.3.1: a dynamic running
 * median filter), as read here:
 *   - the baseline at sample i is the median of the `window` samples starting
 *     window/2 before i, clipped to the series (an even count takes the mean
 *     of the two middle values); the output is the series minus it;
 *   - stride 0 or 1 is that filter exactly, at every sample;
 *   - stride > 1 is a cheaper approximation of it: the median only at knots
 *     t_c = c*stride, c = 0 .. (n-1)/stride, the baseline between two knots
 *     their linear interpolation, after the last knot that knot's median.
 * Returns 0, or -1 on bad arguments. */
int oracle_deredden_f64(const double* x, int64_t n, int32_t window, int32_t stride,
                        double* out) {
  if (n < 1 || window < 1 || stride < 0) return -1;
  if (stride <= 1) {
    double* med = (double*)malloc(sizeof(double) * (size_t)n);
    running_median_f64(x, n, window, med);
    for (int64_t i = 0; i < n; ++i) out[i] = x[i] - med[i];
    free(med);
    return 0;
  }
  int64_t nk = (n - 1) / stride + 1;
  double* med = (double*)malloc(sizeof(double) * (size_t)nk);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < nk; ++c) {
    int64_t lo, hi;
    dered_window_at(c * stride, n, window, &lo, &hi);
    int64_t cnt = hi - lo;
    double* buf = (double*)malloc(sizeof(double) * (size_t)cnt);
    memcpy(buf, x + lo, sizeof(double) * (size_t)cnt);
    qsort(buf, (size_t)cnt, sizeof(double), cmp_f64);
    med[c] = sorted_median(buf, cnt);
    free(buf);
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = i / stride;
    double b = med[c];
    if (c + 1 < nk) b += (med[c + 1] - med[c]) * (double)(i - c * stride) / (double)stride;
    out[i] = x[i] - b;
  }
  free(med);
  return 0;
}

/* --------------------------------------------------------------- search */

/* Score one profile with the chosen algorithm.  Integer profiles use the
 * exact-integer Algorithm 1; Algorithm 2 works on the double copy. */
static double score_profile(const void* prof, int is_int, int32_t P0,
                            const int32_t* widths, int32_t nw, int alg,
                            int32_t* best_w, double* dscratch) {
  (void)dscratch;
  if (is_int) {
    const int64_t* F = (const int64_t*)prof;
    if (alg == ORACLE_ALG1) return oracle_alg1_i64(F, P0, widths, nw, best_w);
    return oracle_alg2_i64(F, P0, widths, nw, best_w);
  }
  const double* F = (const double*)prof;
  if (alg == ORACLE_ALG1) return oracle_alg1_f64(F, P0, widths, nw, best_w);
  return oracle_alg2_f64(F, P0, widths, nw, best_w);
}

/* The default width set when none is given (Sec. 2.2.1): 1, 2, 4, ... up to
 * and including the first power of two larger than 20% of the profile
 * length.  Returns the count written to w (at most 31). */
int32_t oracle_default_widths(int32_t P0, int32_t* w) {
  int32_t n = 0;
  for (int32_t v = 1; n < 31; v *= 2) {
    w[n++] = v;
    if (5 * v > P0) break; /* v > 0.2*P0 */
  }
  return n;
}

/* Periodogram of a search, or of a subset of its steps.
 *
 * series : N samples, float32 (dtype 0) or uint8 (dtype 1)
 * steps  : the plan's step list (as from oracle_plan), n_steps entries
 * sel    : indices into the step list to evaluate (NULL = all)
 * widths : width list (NULL/0 = the default rule per step)
 * snr, width : outputs indexed by global trial number first_trial + k
 *              (only the selected steps' entries are written)
 * threads: OpenMP threads (<= 0: library default)
 */
int oracle_search(const void* series, int32_t dtype, int64_t N,
                  int32_t n_steps, const int32_t* f_arr, const int32_t* P0_arr,
                  const int32_t* m_arr, const int32_t* M_arr,
                  const int64_t* first_arr, int32_t n_sel, const int32_t* sel,
                  const int32_t* widths, int32_t nw, int32_t alg,
                  int32_t threads, int32_t dered_window, int32_t dered_stride,
                  float* snr, int32_t* width) {
  if (dtype != ORACLE_IN_F32 && dtype != ORACLE_IN_U8) return -1;
  if (alg != ORACLE_ALG1 && alg != ORACLE_ALG2) return -1;
  if (dered_window < 0 || dered_stride < 0) return -1;
  /* dereddened series are real-valued: the integer path is used only without */
  int is_int = dtype == ORACLE_IN_U8 && dered_window == 0;
  /* octave series: every octave a step uses, built by successive halving */
  int32_t max_oct = 0;
  for (int32_t s = 0; s < n_steps; ++s) {
    int32_t o = 0;
    while ((1 << o) < f_arr[s]) ++o;
    if (o > max_oct) max_oct = o;
  }
  void** oct = (void**)calloc((size_t)max_oct + 1, sizeof(void*));
  size_t esz = is_int ? sizeof(int64_t) : sizeof(double);
  oct[0] = malloc(esz * (size_t)N);
  if (is_int) {
    const uint8_t* u = (const uint8_t*)series;
    for (int64_t i = 0; i < N; ++i) ((int64_t*)oct[0])[i] = u[i];
  } else if (dtype == ORACLE_IN_U8) {
    const uint8_t* u = (const uint8_t*)series;
    for (int64_t i = 0; i < N; ++i) ((double*)oct[0])[i] = u[i];
  } else {
    const float* x = (const float*)series;
    for (int64_t i = 0; i < N; ++i) ((double*)oct[0])[i] = x[i];
  }
  int64_t len = N;
  for (int32_t o = 1; o <= max_oct; ++o) {
    oct[o] = malloc(esz * (size_t)(len / 2 > 0 ? len / 2 : 1));
    if (is_int)
      halve_i64((const int64_t*)oct[o - 1], len, (int64_t*)oct[o]);
    else
      halve_f64((const double*)oct[o - 1], len, (double*)oct[o]);
    len /= 2;
  }
  /* dynamic dereddening (Sec. 2.3.1): each octave series, built from the raw
   * one above, is filtered with the same window in its own samples, i.e. a
   * window that doubles relative to the input with each downsampling (the
   * octaves below the steps' lowest only feed the halving, so they stay raw) */
  if (dered_window > 0) {
    int32_t min_oct = max_oct;
    for (int32_t q = 0; q < (n_sel > 0 && sel ? n_sel : n_steps); ++q) {
      int32_t s = sel ? sel[q] : q, o = 0;
      while ((1 << o) < f_arr[s]) ++o;
      if (o < min_oct) min_oct = o;
    }
    int64_t ln = N;
    for (int32_t o = 0; o <= max_oct; ++o) {
      if (o >= min_oct) {
        double* tmp = (double*)malloc(sizeof(double) * (size_t)(ln > 0 ? ln : 1));
        if (ln > 0) oracle_deredden_f64((const double*)oct[o], ln, dered_window, dered_stride, tmp);
        free(oct[o]);
        oct[o] = tmp;
      }
      ln /= 2;
    }
  }
  int32_t total = n_sel > 0 && sel ? n_sel : n_steps;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t q = 0; q < total; ++q) {
    int32_t s = sel ? sel[q] : q;
    int32_t f = f_arr[s], P0 = P0_arr[s], m = m_arr[s], M = M_arr[s];
    int32_t o = 0;
    while ((1 << o) < f) ++o;
    size_t cells = (size_t)M * (size_t)P0;
    void* prof = malloc(esz * cells);
    double* dscr = (double*)malloc(sizeof(double) * (size_t)P0);
    if (is_int)
      oracle_fold_i64((const int64_t*)oct[o], P0, m, M, (int64_t*)prof);
    else
      oracle_fold_f64((const double*)oct[o], P0, m, M, (double*)prof);
    int32_t wbuf[32];
    const int32_t* wl = widths;
    int32_t nwl = nw;
    if (!widths || nw <= 0) {
      nwl = oracle_default_widths(P0, wbuf);
      wl = wbuf;
    }
    for (int32_t k = 0; k < M; ++k) {
      int32_t bw = 0;
      const char* p = (const char*)prof + esz * (size_t)k * P0;
      double v = score_profile(p, is_int, P0, wl, nwl, alg, &bw, dscr);
      snr[first_arr[s] + k] = (float)v;
      width[first_arr[s] + k] = bw;
    }
    free(dscr);
    free(prof);
  }
  for (int32_t o = 0; o <= max_oct; ++o) free(oct[o]);
  free(oct);
  return 0;
}

/* Folded profiles of one step straight from the input series (for checking
 * raw profiles).  Float input gives double profiles, uint8 gives int64. */
int oracle_fold_step(const void* series, int32_t dtype, int64_t N, int32_t f,
                     int32_t P0, int32_t m, int32_t M, int32_t dered_window,
                     int32_t dered_stride, void* out) {
  if (dtype != ORACLE_IN_F32 && dtype != ORACLE_IN_U8) return -1;
  if (dered_window < 0 || dered_stride < 0) return -1;
  int32_t o = 0;
  while ((1 << o) < f) ++o;
  if (dered_window > 0) { /* the dereddened octave series (double profiles) */
    double* x = (double*)malloc(sizeof(double) * (size_t)N);
    if (dtype == ORACLE_IN_U8)
      for (int64_t i = 0; i < N; ++i) x[i] = ((const uint8_t*)series)[i];
    else
      for (int64_t i = 0; i < N; ++i) x[i] = ((const float*)series)[i];
    double* d = (double*)malloc(sizeof(double) * (size_t)N);
    oracle_downsample_f64(x, N, o, d);
    int64_t n = N >> o;
    if ((int64_t)m * P0 > n) {
      free(x);
      free(d);
      return -1;
    }
    oracle_deredden_f64(d, n, dered_window, dered_stride, x);
    oracle_fold_f64(x, P0, m, M, (double*)out);
    free(x);
    free(d);
    return 0;
  }
  if (dtype == ORACLE_IN_U8) {
    int64_t* x = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    const uint8_t* u = (const uint8_t*)series;
    for (int64_t i = 0; i < N; ++i) x[i] = u[i];
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    oracle_downsample_i64(x, N, o, d);
    if ((int64_t)m * P0 > (N >> o)) {
      free(x);
      free(d);
      return -1;
    }
    oracle_fold_i64(d, P0, m, M, (int64_t*)out);
    free(x);
    free(d);
  } else {
    double* x = (double*)malloc(sizeof(double) * (size_t)N);
    const float* v = (const float*)series;
    for (int64_t i = 0; i < N; ++i) x[i] = v[i];
    double* d = (double*)malloc(sizeof(double) * (size_t)N);
    oracle_downsample_f64(x, N, o, d);
    if ((int64_t)m * P0 > (N >> o)) {
      free(x);
      free(d);
      return -1;
    }
    oracle_fold_f64(d, P0, m, M, (double*)out);
    free(x);
    free(d);
  }
  return 0;
}

/* ------------------------------------------------------- candidates */

/* Candidate sifting of a periodogram, after the paper's ffa2best (Sec. 2.3.3;
 * settings used in Sec. 4).  The paper names three thresholds, grouping of a
 * strong pulsar's smeared response and harmonic matching by the fractions
 * n/x (x prime, 0 < n < x) within a tolerance, but not their exact rules.
 * Readings taken here:
 *
 *  peaks: trials are scanned in plan order (period non-decreasing).  A trial
 *    with S/N >= min_snr opens a candidate when none is open; while one is
 *    open, a higher S/N moves it there; once the S/N has fallen from it by at
 *    least frac_fall * its S/N and by at least abs_fall, the candidate closes,
 *    and so does any S/N below min_snr (NaN counts as below).
 *  grouping (group_widths > 0): in S/N order (ties: lower trial first), a
 *    surviving candidate c removes each weaker one d with
 *    |P_d - P_c| <= group_widths * W_c * P_c / T_c, W_c = its boxcar width in
 *    seconds and T_c its folded span m*P0*f*tsamp: the period offset at which
 *    its pulse drifts by group_widths widths across the data.
 *  harmonics (harmonic_primes >= 2): in the same order, a surviving c removes
 *    each weaker surviving d with |P_d - r*P_c| <= tol * r*P_c for
 *    r = n/x or x/n, x prime <= harmonic_primes, 0 < n < x.
 *
 * Outputs the surviving candidates in S/N order (trial index, period, S/N,
 * width); returns their count, or -1 on bad arguments.  Each output array
 * needs room for every peak (at most n_trials). */
static int64_t sift_step_of(const int64_t* first, int32_t n_steps, int64_t t) {
  int32_t lo = 0, hi = n_steps - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) / 2;
    if (first[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

typedef struct {
  int64_t trial;
  double period, span, wsec;
  float snr;
  int32_t width;
  int alive;
} sift_cand;

static int cmp_cand(const void* a, const void* b) {
  const sift_cand* x = (const sift_cand*)a;
  const sift_cand* y = (const sift_cand*)b;
  if (x->snr != y->snr) return x->snr > y->snr ? -1 : 1;
  return (x->trial > y->trial) - (x->trial < y->trial);
}

int64_t oracle_sift(const float* snr, const int32_t* width, int64_t n_trials, int32_t n_steps,
                    const int32_t* f_arr, const int32_t* P0_arr, const int32_t* m_arr,
                    const int32_t* M_arr, const int64_t* first_arr, double tsamp,
                    float min_snr, float frac_fall, float abs_fall, float group_widths,
                    int32_t harmonic_primes, float harmonic_tol, int64_t* out_trial,
                    double* out_period, float* out_snr, int32_t* out_width) {
  if (n_trials < 0 || n_steps < 1 || !(tsamp > 0.0)) return -1;
  sift_cand* c = (sift_cand*)malloc(sizeof(sift_cand) * (size_t)(n_trials > 0 ? n_trials : 1));
  int64_t nc = 0;
  int open = 0;
  for (int64_t t = 0; t < n_trials; ++t) {
    float s = snr[t];
    if (!(s >= min_snr)) {
      open = 0;
      continue;
    }
    if (!open) {
      c[nc].trial = t;
      c[nc].snr = s;
      ++nc;
      open = 1;
      continue;
    }
    sift_cand* cur = &c[nc - 1];
    if (s > cur->snr) {
      cur->trial = t;
      cur->snr = s;
    } else if (cur->snr - s >= frac_fall * cur->snr && cur->snr - s >= abs_fall) {
      open = 0;
    }
  }
  for (int64_t i = 0; i < nc; ++i) {
    int64_t s = sift_step_of(first_arr, n_steps, c[i].trial);
    int64_t k = c[i].trial - first_arr[s];
    double fts = (double)f_arr[s] * tsamp;
    c[i].period = fts * ((double)P0_arr[s] + (double)k / (double)(M_arr[s] - 1));
    c[i].span = fts * (double)m_arr[s] * (double)P0_arr[s];
    c[i].width = width[c[i].trial];
    c[i].wsec = fts * (double)c[i].width;
    c[i].alive = 1;
  }
  qsort(c, (size_t)nc, sizeof(sift_cand), cmp_cand);
  if (group_widths > 0.0f) {
    for (int64_t i = 0; i < nc; ++i) {
      if (!c[i].alive) continue;
      double lim = (double)group_widths * c[i].wsec * c[i].period / c[i].span;
      for (int64_t j = i + 1; j < nc; ++j)
        if (c[j].alive && fabs(c[j].period - c[i].period) <= lim) c[j].alive = 0;
    }
  }
  if (harmonic_primes >= 2) {
    for (int64_t i = 0; i < nc; ++i) {
      if (!c[i].alive) continue;
      for (int64_t j = i + 1; j < nc; ++j) {
        if (!c[j].alive) continue;
        int related = 0;
        for (int32_t x = 2; x <= harmonic_primes && !related; ++x) {
          int prime = 1;
          for (int32_t q = 2; q * q <= x; ++q)
            if (x % q == 0) prime = 0;
          if (!prime) continue;
          for (int32_t nn = 1; nn < x && !related; ++nn) {
            double r1 = c[i].period * (double)nn / (double)x;
            double r2 = c[i].period * (double)x / (double)nn;
            if (fabs(c[j].period - r1) <= (double)harmonic_tol * r1) related = 1;
            if (fabs(c[j].period - r2) <= (double)harmonic_tol * r2) related = 1;
          }
        }
        if (related) c[j].alive = 0;
      }
    }
  }
  int64_t k = 0;
  for (int64_t i = 0; i < nc; ++i) {
    if (!c[i].alive) continue;
    out_trial[k] = c[i].trial;
    out_period[k] = c[i].period;
    out_snr[k] = c[i].snr;
    out_width[k] = c[i].width;
    ++k;
  }
  free(c);
  return k;
}

/* ---------------------------------------------------------------------------
 * False-alarm statistics (Sec. 4.1.2).  The paper maps each S/N value of a
 * search of pure noise to a Gaussian-equivalent sigma through the fraction of
 * trials that reach it.  The counting step is a histogram: bin b holds the
 * values with floor((s - lo) * bins_per_unit) == b, the product taken in
 * float; values below lo fall in bin 0 and values past the top in the last
 * bin, so the count at or above every inner edge is exact.  NaN is not
 * counted.  Counts are added to hist, so several searches accumulate. */
void oracle_snr_histogram(const float* snr, int64_t n, float lo, float bins_per_unit, int32_t n_bins,
                          uint64_t* hist) {
  for (int64_t i = 0; i < n; ++i) {
    float s = snr[i];
    if (isnan(s)) continue;
    float x = (s - lo) * bins_per_unit;
    int32_t b;
    if (!(x >= 0.0f))
      b = 0;
    else if (x >= (float)(n_bins - 1))
      b = n_bins - 1;
    else
      b = (int32_t)floorf(x);
    hist[b] += 1;
  }
}

double oracle_mad_constant(void) { return ORACLE_K; }
