"""Plant plausible mistakes in copies of the oracle source (on the CPU) and
require that the pins catch every one of them."""
import os
import subprocess

import pytest

from oracle_pins import ALL_PINS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ffa_oracle.c")

# (name, text in the oracle source, planted replacement)
MUTATIONS = [
    ("shift_floor", "int32_t shift = (t + 1) / 2;", "int32_t shift = t / 2;"),
    ("shift_right", "B[(size_t)src * P0 + (j + shift) % P0]", "B[(size_t)src * P0 + (j + P0 - shift) % P0]"),
    ("wrong_partial", "int32_t src = t / 2;", "int32_t src = t % half;"),
    ("shift_on_head", "o[j] = A[(size_t)src * P0 + j] +                                   \\\n                   B[(size_t)src * P0 + (j + shift) % P0];",
     "o[j] = A[(size_t)src * P0 + (j + shift) % P0] +                      \\\n                   B[(size_t)src * P0 + j];"),
    ("median_lower", "return 0.5 * (scratch[n / 2 - 1] + scratch[n / 2]);", "return scratch[n / 2];"),
    ("k_rounded", "#define ORACLE_K 1.482602218505602", "#define ORACLE_K 1.4826"),
    ("box_not_circular", "C[0] = 0.0;\n  for (int32_t k = 0; k < P0 + w; ++k) C[k + 1] = C[k] + F[k % P0];",
     "C[0] = 0.0;\n  for (int32_t k = 0; k < P0 + w; ++k) C[k + 1] = C[k] + (k < P0 ? F[k] : 0.0);"),
    ("divide_by_width", "double snr = (peak - (double)w * med) / (sigma * sqrt((double)w));",
     "double snr = (peak - (double)w * med) / (sigma * (double)w);"),
    ("mad_about_zero", "for (int32_t j = 0; j < P0; ++j) dev[j] = fabs(F[j] - med);",
     "for (int32_t j = 0; j < P0; ++j) dev[j] = fabs(F[j]);"),
    ("int_num_halved", "int64_t num = 2 * (2 * peak - (int64_t)w * med2);", "int64_t num = 2 * peak - (int64_t)w * med2;"),
    ("downsample_dup", "y[i] = x[2 * i] + x[2 * i + 1];\n}\n\nstatic void halve_i64", "y[i] = x[2 * i] + x[2 * i];\n}\n\nstatic void halve_i64"),
    ("rows_ceil", "int64_t m = Nf / P0;", "int64_t m = (Nf + P0 - 1) / P0;"),
    ("pad_one_more", "while (M < m) M <<= 1;", "while (M <= m) M <<= 1;"),
    ("default_width_rule", "if (5 * v > P0) break;", "if (5 * v >= P0) break;"),
    ("alg2_window_trunc", "int32_t st = jstar + (d - (d & 1)) / 2;", "int32_t st = jstar + d / 2;"),
    ("alg2_sample_sigma", "double sd = sqrt(v / cnt);", "double sd = sqrt(v / (cnt - 1));"),
    ("alg2_window_floor", "const int32_t n_ex = (2 * P0 + 5) / 10; /* round(P0/5) */",
     "const int32_t n_ex = P0 / 5;"),
    ("alg2_window_20pct_only", "const int32_t L = w > n_ex ? w : n_ex;", "const int32_t L = n_ex;"),
    ("alg2_window_no_wrap", "excl[(start + i) % P0] = 1;\n    double s = 0.0;",
     "if (start + i < P0) excl[start + i] = 1;\n    double s = 0.0;"),
    ("alg2_last_max", "double b = bx[j];\n      if (b > imax) {", "double b = bx[j];\n      if (b >= imax) {"),
    ("alg2_no_sqrt_w", "a = sd > 0.0 ? (imax - (double)w * mean) / (sd * sqrt((double)w)) : 0.0;",
     "a = sd > 0.0 ? (imax - (double)w * mean) / sd : 0.0;"),
    ("alg2_level_not_scaled", "a = sd > 0.0 ? (imax - (double)w * mean) / (sd * sqrt((double)w)) : 0.0;",
     "a = sd > 0.0 ? (imax - mean) / (sd * sqrt((double)w)) : 0.0;"),
    ("alg2_int_level", "int64_t num = c * imax - (int64_t)w * s1;", "int64_t num = c * imax - s1;"),
    ("dered_window_late", "int64_t a = i - window / 2, b = a + window;", "int64_t a = i, b = a + window;"),
    ("dered_even_upper", "return cnt % 2 ? v[cnt / 2] : 0.5 * (v[cnt / 2 - 1] + v[cnt / 2]);",
     "return v[cnt / 2];"),
    ("dered_remove_largest", "          memmove(buf + a, buf + a + 1, sizeof(double) * (size_t)(cnt - a - 1));",
     "          (void)a;"),
    ("dered_enter_previous", "        const double v = x[hi];", "        const double v = x[hi - 1];"),
    ("dered_no_slide_in", "      if (hi2 > hi) {", "      if (hi2 > hi + 1) {"),
    ("dered_no_interp", "if (c + 1 < nk) b += (med[c + 1] - med[c])", "if (c + 1 < 0) b += (med[c + 1] - med[c])"),
    ("dered_default_2x", "double w4 = 4.0 * pmin / tsamp;", "double w4 = 2.0 * pmin / tsamp;"),
    ("hist_round", "      b = (int32_t)floorf(x);", "      b = (int32_t)roundf(x);"),
    ("hist_drop_top", "      b = n_bins - 1;\n    else", "      continue;\n    else"),
    ("hist_nan_counted", "    if (isnan(s)) continue;\n    float x", "    if (isnan(s)) s = lo;\n    float x"),
    ("sift_fall_either", "} else if (cur->snr - s >= frac_fall * cur->snr && cur->snr - s >= abs_fall) {",
     "} else if (cur->snr - s >= frac_fall * cur->snr || cur->snr - s >= abs_fall) {"),
    ("sift_no_climb", "    if (s > cur->snr) {\n      cur->trial = t;", "    if (0) {\n      cur->trial = t;"),
    ("sift_low_keeps_open", "    if (!(s >= min_snr)) {\n      open = 0;\n      continue;",
     "    if (!(s >= min_snr)) {\n      continue;"),
    ("sift_group_no_span", "c[i].wsec * c[i].period / c[i].span;", "c[i].wsec;"),
    ("sift_harm_one_side", "if (fabs(c[j].period - r2) <= (double)harmonic_tol * r2) related = 1;", ""),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(oracle_mod, tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {name}"
    mut = tmp_path / f"{name}.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(mut), "-lm"],
                   check=True)
    caught = None
    with oracle_mod.library(str(so)):
        for pin in ALL_PINS:
            try:
                pin(oracle_mod)
            except Exception:  # noqa: BLE001 - any failure counts as caught
                caught = pin.__name__
                break
    assert caught, f"planted mistake {name} passed every pin"
