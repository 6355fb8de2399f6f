// HIP kernels of the FFA search for gfx950 (CDNA4, 64-wide wavefronts).
//
// Work is cut into tiles (ffa_internal.h): one workgroup stages 2^d rows of a
// step in LDS, runs d butterfly levels of the FFA tree in place, and then
// either writes the 2^d partial profiles back for the next pass or scores
// each folded profile with Algorithm 1 (paper Sec. 2.2.1).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ffa_internal.h"

namespace ffa {
namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Position of partial t after d in-place levels: its d-bit reversal.
__device__ __forceinline__ int bitrev(int t, int d) {
  return d == 0 ? 0 : (int)(__brev((unsigned)t) >> (32 - d));
}

// Wavefront-scope ordering of this wave's LDS writes before its later reads
// by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// --------------------------------------------------------------- butterfly

// All `d` levels of the FFA tree on 2^d rows held in LDS (row stride S).
//
// Level l merges the two halves A, B of each block of 2^l rows:
//   out_{2v}[j]   = A_v[j] + B_v[(j + v)     mod P0]
//   out_{2v+1}[j] = A_v[j] + B_v[(j + v + 1) mod P0]
// (paper Sec. 2.1, after Staelin 1969).  The pair is written over the slots
// of A_v and B_v, so partial t of a block ends at the bit reversal of t.
// One wave owns a pair of rows per level, so a level needs no barrier inside;
// every read of a B row precedes its writes because the shifted reads wrap.
template <typename T>
__device__ void butterfly(T* lds, int S, int P0, int d) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  const int R = 1 << d;
  constexpr int kMaxE = 32;  // P0 <= 2048
  for (int l = 1; l <= d; ++l) {
    const int half = 1 << (l - 1);
    for (int p = wave; p < (R >> 1); p += nwaves) {
      const int beta = p >> (l - 1);
      const int v = p & (half - 1);
      T* A = lds + (size_t)(beta * 2 * half + bitrev(v, l - 1)) * S;
      T* B = A + (size_t)half * S;
      const int s0 = v % P0;
      const int s1 = (v + 1) % P0;
      T keep[kMaxE];
#pragma unroll
      for (int c = 0; c < kMaxE; ++c) {
        const int j = lane + c * kWave;
        if (c * kWave < P0 && j < P0) {
          int i0 = j + s0;
          i0 -= (i0 >= P0) ? P0 : 0;
          int i1 = j + s1;
          i1 -= (i1 >= P0) ? P0 : 0;
          const T a = A[j];
          const T b0 = B[i0];
          const T b1 = B[i1];
          A[j] = a + b0;  // only this lane reads A[j]
          keep[c] = a + b1;
        }
      }
#pragma unroll
      for (int c = 0; c < kMaxE; ++c) {
        const int j = lane + c * kWave;
        if (c * kWave < P0 && j < P0) B[j] = keep[c];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- selection

template <typename K>
struct Pad;
template <>
struct Pad<float> {
  __device__ static float v() { return INFINITY; }
};
template <>
struct Pad<uint32_t> {
  __device__ static uint32_t v() { return 0xffffffffu; }
};

// Ascending bitonic sort of 64*E keys held blocked across the wave
// (element e = lane*E + r lives in register r of lane e/E).
template <int E, typename K>
__device__ __forceinline__ void wave_sort(K (&x)[E]) {
  const int lane = lane_id();
  constexpr int n = kWave * E;
#pragma unroll
  for (int k = 2; k <= n; k <<= 1) {
#pragma unroll
    for (int s = k >> 1; s > 0; s >>= 1) {
      if (s < E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          if ((r & s) == 0) {
            const bool asc = ((lane * E + r) & k) == 0;
            const K a = x[r], b = x[r | s];
            const K lo = a < b ? a : b;
            const K hi = a < b ? b : a;
            x[r] = asc ? lo : hi;
            x[r | s] = asc ? hi : lo;
          }
        }
      } else {
        const int m = s / E;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int e = lane * E + r;
          const K p = __shfl_xor(x[r], m, kWave);
          const bool lower = (e & s) == 0;
          const bool asc = (e & k) == 0;
          const K lo = x[r] < p ? x[r] : p;
          const K hi = x[r] < p ? p : x[r];
          x[r] = (lower == asc) ? lo : hi;
        }
      }
    }
  }
}

// Element `idx` of a blocked wave array.
template <int E, typename K>
__device__ __forceinline__ K wave_get(const K (&x)[E], int idx) {
  const int r = idx % E;
  K v = x[0];
#pragma unroll
  for (int i = 1; i < E; ++i)
    if (i == r) v = x[i];
  return __shfl(v, idx / E, kWave);
}

template <typename K>
__device__ __forceinline__ K wave_max(K v) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) {
    const K o = __shfl_xor(v, m, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Exclusive prefix over the wave of one value per lane.
template <typename K>
__device__ __forceinline__ K wave_exclusive_scan(K v) {
  const int lane = lane_id();
  K inc = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const K u = __shfl_up(inc, o, kWave);
    if (lane >= o) inc = inc + u;
  }
  return inc - v;
}

// ----------------------------------------------------------- Algorithm 1

template <bool INT>
struct Types;
template <>
struct Types<true> {
  using T = int32_t;   // stored sums (non-negative, < 2^31)
  using K = uint32_t;  // key / modular prefix type
};
template <>
struct Types<false> {
  using T = float;
  using K = float;
};

// Score one folded profile with Algorithm 1 (paper Sec. 2.2.1): median and
// MAD of the profile (Eqs. 3-4), circular boxcars of every width, score =
// max_w (max_j box_w[j] - w*median) / (K*MAD*sqrt(w)).  The whole wave works
// on one profile held in LDS row `row` (stride >= P0 + wmax + 1); the row is
// overwritten with the circular prefix sums.
//
// Integer profiles are scored exactly: med2 = 2*median, mad4 = 4*MAD, and
// S/N = 2*(2*peak - w*med2) / ((K*mad4)*sqrt(w)) in double, with sqrt(w)
// from a host table, so every rounding is a correctly rounded IEEE operation.
template <int E, bool INT>
__device__ void score_profile(typename Types<INT>::T* row, int P0, int wmax,
                              const int32_t* widths, const double* sqrtw,
                              int nw, float* snr_out, int32_t* width_out) {
  using T = typename Types<INT>::T;
  using K = typename Types<INT>::K;
  const int lane = lane_id();
  const int a = (P0 - 1) / 2;
  const int b = P0 / 2;

  K x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    x[r] = e < P0 ? (K)row[e] : Pad<K>::v();
  }
  wave_sort<E>(x);
  const K xa = wave_get<E>(x, a);
  const K xb = wave_get<E>(x, b);

  // deviations from the median
  int64_t med2 = 0;
  float med = 0.f;
  if constexpr (INT) {
    med2 = (int64_t)xa + (int64_t)xb;
  } else {
    med = (float)(0.5 * ((double)xa + (double)xb));
  }
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    if constexpr (INT) {
      const int64_t dv = 2 * (int64_t)x[r] - med2;
      x[r] = e < P0 ? (K)(dv < 0 ? -dv : dv) : Pad<K>::v();
    } else {
      x[r] = e < P0 ? fabsf(x[r] - med) : Pad<K>::v();
    }
  }
  wave_sort<E>(x);
  const K da = wave_get<E>(x, a);
  const K db = wave_get<E>(x, b);
  bool mad_zero;
  uint64_t mad4 = 0;
  float mad = 0.f;
  if constexpr (INT) {
    mad4 = (uint64_t)da + (uint64_t)db;
    mad_zero = mad4 == 0;
  } else {
    mad = (float)(0.5 * ((double)da + (double)db));
    mad_zero = mad == 0.f;
  }
  if (mad_zero) {
    if (lane == 0) {
      *snr_out = 0.f;
      *width_out = 0;
    }
    return;
  }

  // circular prefix sums C[k] = sum_{i<k} F[i mod P0], k <= P0 + wmax
  K y[E];
  K run = 0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    const K v = e < P0 ? (K)row[e] : (K)0;
    run = run + v;
    y[r] = run;
  }
  const K base = wave_exclusive_scan(run);
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = lane * E + r;
    if (e < P0) row[e + 1] = (T)(base + y[r]);
  }
  if (lane == 0) row[0] = (T)0;
  wave_lds_sync();
  const K total = (K)row[P0];
  for (int i = lane; i < wmax; i += kWave) row[P0 + 1 + i] = (T)(total + (K)row[1 + i]);
  wave_lds_sync();

  K mx[kMaxWidths];
#pragma unroll
  for (int i = 0; i < kMaxWidths; ++i) {
    if constexpr (INT) mx[i] = 0u;
    else mx[i] = -INFINITY;
  }
  for (int j = lane; j < P0; j += kWave) {
    const K c0 = (K)row[j];
#pragma unroll
    for (int i = 0; i < kMaxWidths; ++i) {
      if (i < nw) {
        const K v = (K)row[j + widths[i]] - c0;
        mx[i] = v > mx[i] ? v : mx[i];
      }
    }
  }
  double best = 0.0;
  int32_t bw = 0;
#pragma unroll
  for (int i = 0; i < kMaxWidths; ++i) {
    if (i < nw) {
      const K peak = wave_max(mx[i]);
      const int32_t w = widths[i];
      double s;
      if constexpr (INT) {
        const int64_t num = 2 * (2 * (int64_t)peak - (int64_t)w * med2);
        const double den = (kMadK * (double)mad4) * sqrtw[i];
        s = (double)num / den;
      } else {
        s = ((double)peak - (double)w * (double)med) /
            ((kMadK * (double)mad) * sqrtw[i]);
      }
      if (bw == 0 || s > best) {
        best = s;
        bw = w;
      }
    }
  }
  if (lane == 0) {
    *snr_out = (float)best;
    *width_out = bw;
  }
}

template <bool INT>
__device__ void score_dispatch(typename Types<INT>::T* row, int P0, int wmax,
                               const int32_t* widths, const double* sqrtw,
                               int nw, float* snr_out, int32_t* width_out) {
  if (P0 <= 64)
    score_profile<1, INT>(row, P0, wmax, widths, sqrtw, nw, snr_out, width_out);
  else if (P0 <= 128)
    score_profile<2, INT>(row, P0, wmax, widths, sqrtw, nw, snr_out, width_out);
  else if (P0 <= 256)
    score_profile<4, INT>(row, P0, wmax, widths, sqrtw, nw, snr_out, width_out);
  else if (P0 <= 512)
    score_profile<8, INT>(row, P0, wmax, widths, sqrtw, nw, snr_out, width_out);
  else if (P0 <= 1024)
    score_profile<16, INT>(row, P0, wmax, widths, sqrtw, nw, snr_out, width_out);
  else
    score_profile<32, INT>(row, P0, wmax, widths, sqrtw, nw, snr_out, width_out);
}

// ------------------------------------------------------------ pass kernel

template <bool INT>
__global__ __launch_bounds__(kThreads) void ffa_pass_kernel(
    const Tile* __restrict__ tiles, void* __restrict__ ws_raw,
    float* __restrict__ snr, int32_t* __restrict__ width,
    void* __restrict__ profiles, int64_t trial_base, int mode,
    const int32_t* __restrict__ wtab, const double* __restrict__ sqrtw) {
  using T = typename Types<INT>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  T* ws = reinterpret_cast<T*>(ws_raw);

  const Tile tl = tiles[blockIdx.x];
  const int P0 = tl.P0;
  const int d = tl.depth;
  const int R = 1 << d;
  const int S = tl.stride;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;

  // stage the group's rows (rows >= valid are zero padding, paper Sec. 2.1)
  const T* src = ws + tl.src;
  for (int r = wave; r < R; r += nwaves) {
    T* row = lds + (size_t)r * S;
    if (r < tl.valid) {
      const T* g = src + (int64_t)r * P0;
      for (int j = lane; j < P0; j += kWave) row[j] = g[j];
    } else {
      for (int j = lane; j < P0; j += kWave) row[j] = (T)0;
    }
  }
  __syncthreads();

  butterfly<T>(lds, S, P0, d);

  if (!tl.final_) {
    // Hand partial t to the next pass rotated left by t*h bins: the levels
    // above this pass then act on the rotated rows like a plain FFA tree.
    for (int t = wave; t < R; t += nwaves) {
      const T* srow = lds + (size_t)bitrev(t, d) * S;
      const int rot = (int)(((int64_t)t * tl.h) % P0);
      T* out = ws + tl.dst + (int64_t)t * tl.dst_step;
      for (int j = lane; j < P0; j += kWave) {
        int i = j + rot;
        i -= (i >= P0) ? P0 : 0;
        out[j] = srow[i];
      }
    }
    return;
  }
  if (mode == kModeProfiles) {
    T* out = reinterpret_cast<T*>(profiles);
    for (int t = wave; t < R; t += nwaves) {
      const T* srow = lds + (size_t)bitrev(t, d) * S;
      T* o = out + (tl.dst - trial_base + t) * (int64_t)P0;
      for (int j = lane; j < P0; j += kWave) o[j] = srow[j];
    }
    return;
  }
  const int32_t* widths = wtab + tl.wofs;
  const double* sw = sqrtw + tl.wofs;
  int wmax = 0;
  for (int i = 0; i < tl.nw; ++i) wmax = widths[i] > wmax ? widths[i] : wmax;
  for (int t = wave; t < R; t += nwaves) {
    T* row = lds + (size_t)bitrev(t, d) * S;
    const int64_t trial = tl.dst + t;
    score_dispatch<INT>(row, P0, wmax, widths, sw, tl.nw, snr + trial,
                        width + trial);
  }
}

// ------------------------------------------------------------- prep kernels

constexpr int kMeanBlocks = 1024;
constexpr int kMeanThreads = 256;

// Per-block partial sums of the series in double (fixed order).
__global__ __launch_bounds__(kMeanThreads) void mean_partial_kernel(
    const float* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double red[kMeanThreads];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kMeanThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kMeanThreads)
    s += (double)x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kMeanThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kMeanBlocks) void mean_final_kernel(
    const double* __restrict__ part, int64_t n, float* __restrict__ c) {
  __shared__ double red[kMeanBlocks];
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int o = kMeanBlocks / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *c = (float)(red[0] / (double)n);
}

// Octave 0 in the accumulator type: exact int32 for uint8 input, float minus
// the centring constant for float input.
__global__ void prep_u8_kernel(const uint8_t* __restrict__ in, int64_t n,
                               int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int32_t)in[i];
}

__global__ void prep_f32_kernel(const float* __restrict__ in, int64_t n,
                                const float* __restrict__ c, int center,
                                float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = center ? in[i] - *c : in[i];
}

// One halving of the time resolution (paper Sec. 2.3.1): y[i] = x[2i]+x[2i+1].
template <typename T>
__global__ void halve_kernel(const T* __restrict__ in, int64_t n_out,
                             T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_out) out[i] = in[2 * i] + in[2 * i + 1];
}

// Largest score, first index on ties (one workgroup; NaN never wins).
__global__ __launch_bounds__(1024) void best_kernel(const float* __restrict__ s,
                                                    int64_t n,
                                                    int64_t* __restrict__ best) {
  __shared__ float bv[1024];
  __shared__ int64_t bi[1024];
  float v = -INFINITY;
  int64_t idx = -1;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float x = s[i];
    if (x > v || (idx < 0 && x == v)) {
      v = x;
      idx = i;
    }
  }
  bv[threadIdx.x] = v;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const float v2 = bv[threadIdx.x + o];
      const int64_t i2 = bi[threadIdx.x + o];
      const float v1 = bv[threadIdx.x];
      const int64_t i1 = bi[threadIdx.x];
      bool take;
      if (i2 < 0) take = false;
      else if (i1 < 0) take = true;
      else take = v2 > v1 || (v2 == v1 && i2 < i1);
      if (take) {
        bv[threadIdx.x] = v2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *best = bi[0] < 0 ? 0 : bi[0];
}

}  // namespace

// --------------------------------------------------------------- launchers

// Workspace header: [0, 1024) doubles of partial sums, then the centring
// constant (one float) -- see the planner's header size.
hipError_t launch_mean(const float* x, int64_t n, void* ws, hipStream_t st) {
  double* part = reinterpret_cast<double*>(ws);
  float* c = reinterpret_cast<float*>(part + kMeanBlocks);
  mean_partial_kernel<<<kMeanBlocks, kMeanThreads, 0, st>>>(x, n, part);
  mean_final_kernel<<<1, kMeanBlocks, 0, st>>>(part, n, c);
  return hipGetLastError();
}

hipError_t launch_prep(const void* series, int is_int, int64_t n, void* ws,
                       int64_t out_off, int center, hipStream_t st) {
  const int tpb = 256;
  const int64_t blocks = (n + tpb - 1) / tpb;
  if (is_int) {
    int32_t* out = reinterpret_cast<int32_t*>(ws) + out_off;
    prep_u8_kernel<<<blocks, tpb, 0, st>>>(
        reinterpret_cast<const uint8_t*>(series), n, out);
  } else {
    const float* c = reinterpret_cast<const float*>(
        reinterpret_cast<const double*>(ws) + kMeanBlocks);
    float* out = reinterpret_cast<float*>(ws) + out_off;
    prep_f32_kernel<<<blocks, tpb, 0, st>>>(
        reinterpret_cast<const float*>(series), n, c, center, out);
  }
  return hipGetLastError();
}

hipError_t launch_halve(void* ws, int is_int, int64_t in_off,
                              int64_t n_out, int64_t out_off, hipStream_t st) {
  const int tpb = 256;
  const int64_t blocks = (n_out + tpb - 1) / tpb;
  if (n_out <= 0) return hipSuccess;
  if (is_int) {
    int32_t* w = reinterpret_cast<int32_t*>(ws);
    halve_kernel<int32_t><<<blocks, tpb, 0, st>>>(w + in_off, n_out, w + out_off);
  } else {
    float* w = reinterpret_cast<float*>(ws);
    halve_kernel<float><<<blocks, tpb, 0, st>>>(w + in_off, n_out, w + out_off);
  }
  return hipGetLastError();
}

hipError_t launch_pass(const Tile* tiles, int64_t n_tiles, int lds_bytes,
                       int is_int, void* ws, float* snr, int32_t* width,
                       void* profiles, int64_t trial_base, int mode,
                       const int32_t* wtab, const double* sqrtw,
                       hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if ((size_t)lds_bytes > kLdsBytes) return hipErrorInvalidValue;
  static hipError_t attr = [] {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ffa_pass_kernel<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ffa_pass_kernel<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    return e;
  }();
  if (attr != hipSuccess) return attr;
  if (is_int) {
    ffa_pass_kernel<true><<<(unsigned)n_tiles, kThreads, lds_bytes, st>>>(
        tiles, ws, snr, width, profiles, trial_base, mode, wtab, sqrtw);
  } else {
    ffa_pass_kernel<false><<<(unsigned)n_tiles, kThreads, lds_bytes, st>>>(
        tiles, ws, snr, width, profiles, trial_base, mode, wtab, sqrtw);
  }
  return hipGetLastError();
}

hipError_t launch_best(const float* snr, int64_t n, int64_t* best,
                       hipStream_t st) {
  best_kernel<<<1, 1024, 0, st>>>(snr, n, best);
  return hipGetLastError();
}

}  // namespace ffa
