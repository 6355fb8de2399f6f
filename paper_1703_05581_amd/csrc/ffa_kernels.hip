// HIP kernels of the FFA search for gfx950 (CDNA4, 64-wide wavefronts).
//
// Work is cut into tiles (ffa_internal.h): one workgroup stages 2^d rows of a
// step in LDS, runs d butterfly levels of the FFA tree in place, and then
// either writes the 2^d partial profiles back for the next pass or scores
// each folded profile with Algorithm 1 (paper Sec. 2.2.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

#include "ffa_internal.h"

namespace ffa {
namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// The lane index as a value the compiler cannot hoist: the scoring helpers
// take it afresh on every profile, so the lane masks derived from it are
// recomputed where they are used instead of being held for the whole tile
// (held, they overflow the scalar registers and go to vector-register lanes).
__device__ __forceinline__ int lane_fresh() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t & (kWave - 1);
}

// Index of this wave in its workgroup, as a wave-uniform (scalar) value: the
// per-wave loops and their index arithmetic then run on the scalar unit.
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// Position of partial t after d in-place levels: its d-bit reversal.
__device__ __forceinline__ int bitrev(int t, int d) {
  return d == 0 ? 0 : (int)(__brev((unsigned)t) >> (32 - d));
}

// Orders this wave's earlier LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------- wave primitives

// DPP lane patterns of GFX9 (data-parallel primitives on VALU operands).
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppRowMirror = 0x140;  // lane i <- 15-i within a row of 16
constexpr int kDppHalfMirror = 0x141; // lane i <- 7-i within 8
constexpr int kDppBcast15 = 0x142;    // lane 15 of each row -> next row
constexpr int kDppBcast31 = 0x143;    // lane 31 -> rows 2 and 3
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;
constexpr int kDppRor4 = 0x124, kDppRor8 = 0x128;  // lane i <- (i - n) mod 16 within a row

template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWMASK, 0xF, false);
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// A value the wave holds in every lane, marked as such for the compiler
// (scalar registers, uniform branches).
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ float uniform(float v) {
  return __uint_as_float((uint32_t)__builtin_amdgcn_readfirstlane((int)__float_as_uint(v)));
}

__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }

// Maximum / minimum of one value per lane; the result is wave-uniform.
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
  v = umax(v, dpp<kDppXor1>(0u, v));
  v = umax(v, dpp<kDppXor2>(0u, v));
  v = umax(v, dpp<kDppHalfMirror>(0u, v));
  v = umax(v, dpp<kDppRowMirror>(0u, v));
  v = umax(v, dpp<kDppBcast15, 0xA>(0u, v));
  v = umax(v, dpp<kDppBcast31, 0xC>(0u, v));
  return readlane(v, 63);
}

// Wave maxima of eight values at once: lane L returns the maximum over all
// lanes of v[L & 7].  Three exchange steps each halve what a lane keeps
// (partners keep opposite halves, so every value is combined once per step),
// one row rotation and two lane permutes finish the reduction, and a last
// permute moves each maximum to the lanes of its index.
__device__ __forceinline__ uint32_t bpermute(int src_lane, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}

__device__ __forceinline__ uint32_t wave_umax8(const uint32_t (&v)[8]) {
  const int lane = lane_fresh();
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  uint32_t r[4], s[2];
#pragma unroll
  for (int j = 0; j < 4; ++j)  // r[j]: index j + 4*b0, over lanes L and L^1
    r[j] = umax(b0 ? v[j + 4] : v[j], dpp<kDppXor1>(0u, b0 ? v[j] : v[j + 4]));
#pragma unroll
  for (int j = 0; j < 2; ++j)  // s[j]: index j + 2*b1 + 4*b0, over the quad
    s[j] = umax(b1 ? r[j + 2] : r[j], dpp<kDppXor2>(0u, b1 ? r[j] : r[j + 2]));
  // index b2 + 2*b1 + 4*b0 (bits of L reversed), over two quads of the row
  // (lane L - 4 mod 16 has the other b2 and the same b0, b1)
  uint32_t t = umax(b2 ? s[1] : s[0], dpp<kDppRor4>(0u, b2 ? s[0] : s[1]));
  t = umax(t, dpp<kDppRor8>(0u, t));  // the other two quads: the whole row
  t = umax(t, bpermute(lane ^ 16, t));
  t = umax(t, bpermute(lane ^ 32, t));
  const int k = lane & 7;
  return bpermute(((k & 1) << 2) | (k & 2) | (k >> 2), t);
}

__device__ __forceinline__ uint32_t wave_umin(uint32_t v) {
  v = umin(v, dpp<kDppXor1>(~0u, v));
  v = umin(v, dpp<kDppXor2>(~0u, v));
  v = umin(v, dpp<kDppHalfMirror>(~0u, v));
  v = umin(v, dpp<kDppRowMirror>(~0u, v));
  v = umin(v, dpp<kDppBcast15, 0xA>(~0u, v));
  v = umin(v, dpp<kDppBcast31, 0xC>(~0u, v));
  return readlane(v, 63);
}

// Inclusive prefix sum over the 64 lanes (modular for integers).
__device__ __forceinline__ uint32_t wave_scan(uint32_t v) {
  v += dpp<kDppShr1>(0u, v);
  v += dpp<kDppShr2>(0u, v);
  v += dpp<kDppShr4>(0u, v);
  v += dpp<kDppShr8>(0u, v);
  v += dpp<kDppBcast15, 0xA>(0u, v);
  v += dpp<kDppBcast31, 0xC>(0u, v);
  return v;
}

__device__ __forceinline__ float wave_scan(float v) {
  auto step = [](float x, uint32_t sh) { return x + __uint_as_float(sh); };
  v = step(v, dpp<kDppShr1>(0u, __float_as_uint(v)));
  v = step(v, dpp<kDppShr2>(0u, __float_as_uint(v)));
  v = step(v, dpp<kDppShr4>(0u, __float_as_uint(v)));
  v = step(v, dpp<kDppShr8>(0u, __float_as_uint(v)));
  v = step(v, dpp<kDppBcast15, 0xA>(0u, __float_as_uint(v)));
  v = step(v, dpp<kDppBcast31, 0xC>(0u, __float_as_uint(v)));
  return v;
}

__device__ __forceinline__ int wave_count(bool p) { return __popcll(__ballot(p)); }

// DPP of a 64-bit value (both halves moved the same way; masked rows give 0).
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t lo = dpp<CTRL, ROWMASK>(0u, (uint32_t)v);
  const uint32_t hi = dpp<CTRL, ROWMASK>(0u, (uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  return ((uint64_t)readlane((uint32_t)(v >> 32), l) << 32) | readlane((uint32_t)v, l);
}

// The width table of a step, held one entry per lane (lane i: width i, its
// square root and reciprocal square root), so the scoring loops read entries
// with v_readlane instead of memory loads.
struct WidthLanes {
  int32_t w;
  double sq, isq;
  __device__ __forceinline__ int32_t width(int i) const { return (int32_t)readlane((uint32_t)w, i); }
  __device__ __forceinline__ double sqrtw(int i) const {
    return __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(sq), i));
  }
  __device__ __forceinline__ double isqrtw(int i) const {
    return __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(isq), i));
  }
};

// Sums of two values per lane over the wave at once (fixed trees, so the
// results are deterministic): after the first exchange even lanes carry a
// and odd lanes b, and the remaining steps keep that parity.
__device__ __forceinline__ void wave_sum2(double a, double b, double& sa, double& sb) {
  auto bits = [](double x) { return (uint64_t)__double_as_longlong(x); };
  auto dbl = [](uint64_t u) { return __longlong_as_double((long long)u); };
  const int lane = lane_fresh();
  const bool odd = lane & 1;
  double v = (odd ? b : a) + dbl(dpp64<kDppXor1>(bits(odd ? a : b)));
  v += dbl(dpp64<kDppXor2>(bits(v)));  // the quad
  v += dbl(dpp64<kDppRor4>(bits(v)));  // two quads
  v += dbl(dpp64<kDppRor8>(bits(v)));  // the row
  auto perm = [&](int src, double x) {
    const uint64_t u = bits(x);
    return dbl(((uint64_t)bpermute(src, (uint32_t)(u >> 32)) << 32) | bpermute(src, (uint32_t)u));
  };
  v += perm(lane ^ 16, v);
  v += perm(lane ^ 32, v);
  sa = dbl(readlane64(bits(v), 0));
  sb = dbl(readlane64(bits(v), 1));
}

// Sum of one value per lane over the wave (a fixed reduction tree, so the
// result is deterministic); wave-uniform.
__device__ __forceinline__ int64_t wave_sum(int64_t v) {
  uint64_t u = (uint64_t)v;
  u += dpp64<kDppXor1>(u);
  u += dpp64<kDppXor2>(u);
  u += dpp64<kDppHalfMirror>(u);
  u += dpp64<kDppRowMirror>(u);
  u += dpp64<kDppBcast15, 0xA>(u);
  u += dpp64<kDppBcast31, 0xC>(u);
  return (int64_t)readlane64(u, 63);
}

__device__ __forceinline__ double wave_sum(double v) {
  auto add = [](double a, uint64_t b) { return a + __longlong_as_double((long long)b); };
  auto bits = [](double a) { return (uint64_t)__double_as_longlong(a); };
  v = add(v, dpp64<kDppXor1>(bits(v)));
  v = add(v, dpp64<kDppXor2>(bits(v)));
  v = add(v, dpp64<kDppHalfMirror>(bits(v)));
  v = add(v, dpp64<kDppRowMirror>(bits(v)));
  v = add(v, dpp64<kDppBcast15, 0xA>(bits(v)));
  v = add(v, dpp64<kDppBcast31, 0xC>(bits(v)));
  return __longlong_as_double((long long)readlane64(bits(v), 63));
}

// Maximum of one double per lane (no NaNs); wave-uniform.
__device__ __forceinline__ double wave_dmax(double v) {
  auto mx = [](double a, uint64_t b) { return fmax(a, __longlong_as_double((long long)b)); };
  auto bits = [](double a) { return (uint64_t)__double_as_longlong(a); };
  v = mx(v, dpp64<kDppXor1>(bits(v)));
  v = mx(v, dpp64<kDppXor2>(bits(v)));
  v = mx(v, dpp64<kDppHalfMirror>(bits(v)));
  v = mx(v, dpp64<kDppRowMirror>(bits(v)));
  v = mx(v, dpp64<kDppBcast15, 0xA>(bits(v)));
  v = mx(v, dpp64<kDppBcast31, 0xC>(bits(v)));
  return __longlong_as_double((long long)readlane64(bits(v), 63));
}

// Maximum over lanes 0..15 (the first row; other lanes are ignored), as a
// wave-uniform value: four in-row exchange steps instead of six.
__device__ __forceinline__ double row_dmax16(double v) {
  auto mx = [](double a, uint64_t b) { return fmax(a, __longlong_as_double((long long)b)); };
  auto bits = [](double a) { return (uint64_t)__double_as_longlong(a); };
  v = mx(v, dpp64<kDppXor1>(bits(v)));
  v = mx(v, dpp64<kDppXor2>(bits(v)));
  v = mx(v, dpp64<kDppHalfMirror>(bits(v)));
  v = mx(v, dpp64<kDppRowMirror>(bits(v)));
  return __longlong_as_double((long long)readlane64(bits(v), 0));
}

// Order-preserving 32-bit keys: integer sums (non-negative, < 2^31) are their
// own keys; a finite float maps to an unsigned integer with the same order.
__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t b = __float_as_uint(f);
  return b ^ ((b >> 31) ? 0xffffffffu : 0x80000000u);
}
__device__ __forceinline__ float fval(uint32_t k) {
  return __uint_as_float(k ^ ((k >> 31) ? 0x80000000u : 0xffffffffu));
}

constexpr uint32_t kPadKey = 0xffffffffu;  // above every real key

// --------------------------------------------------------------- butterfly

// All `d` levels of the FFA tree on 2^d rows held in LDS.  Row r occupies
// lds[r*S .. r*S + P0 + H): bins 0..P0-1, then H bins of halo.
//
// Level l merges the two halves A, B of each block of 2^l rows:
//   out_{2v}[j]   = A_v[j] + B_v[(j + v)     mod P0]
//   out_{2v+1}[j] = A_v[j] + B_v[(j + v + 1) mod P0]
// (paper Sec. 2.1, after Staelin 1969).  The pair is written over the slots
// of A_v and B_v, so partial t of a block ends at the bit reversal of t.
// One wave owns a pair of rows per level.  It first copies bins 0..H-1 of B
// into B's halo, so the shifted reads B[j + s], j + s < P0 + H, never wrap;
// then it walks the bins in chunks of 64.  Chunk c reads B at
// [64c + s, 64c + 64 + s] and writes B at [64c, 64c + 63], so no write lands
// where a later chunk reads, and the halo keeps the old bins.  No barrier is
// needed inside a level.  Where the row's spare bins allow a halo of
// 3*2^(l-1), levels l and l+1 run as one pass over four rows (radix 4): the
// same sums in the same order, with 10 reads and 4 writes per four outputs
// instead of 12 and 8, and one barrier instead of two.
template <typename T>
__device__ __forceinline__ void butterfly(T* lds, int S, int P0, int H, int d) {
  const int lane = lane_id();
  const int wave = wave_id();
  const int nwaves = blockDim.x / kWave;
  const int R = 1 << d;
  const int nfull = P0 / kWave;
  const bool tail = nfull * kWave + lane < P0;
  const int room = S - P0 < P0 ? S - P0 : P0;  // bins a halo may hold
  // 1, hidden from the compiler: adjacent 16-bit reads of one row would be
  // merged into one wider read that is not 4-byte aligned, which the LDS
  // serves slowly
  int one = 1;
  asm volatile("" : "+s"(one));
  int l = 1;
  while (l <= d) {
    const int half = 1 << (l - 1);
    if (l < d && 3 * half <= room) {
      // Levels l and l+1 at once (radix 4).  Unit (block b, index v < half)
      // holds partial v of the four quarters of a block of 4*half rows,
      // x0..x3 (all shifts below P0, as 3*half <= P0).  With every index
      // mod P0,
      //   t_{4v}   = (x0 + x1[+v])   + (x2[+2v]   + x3[+3v])
      //   t_{4v+1} = (x0 + x1[+v])   + (x2[+2v+1] + x3[+3v+1])
      //   t_{4v+2} = (x0 + x1[+v+1]) + (x2[+2v+1] + x3[+3v+2])
      //   t_{4v+3} = (x0 + x1[+v+1]) + (x2[+2v+2] + x3[+3v+3])
      // which are the two levels' sums in the same order, written over
      // x0, x2, x1, x3: the slots the two single levels would use.  The
      // halos hold bins 0..k*v+k of x_k, so no read wraps.
      for (int u = wave; u < (R >> 2); u += nwaves) {
        const int blk = u >> (l - 1);
        const int v = u & (half - 1);
        T* X0 = lds + (size_t)(blk * 4 * half + bitrev(v, l - 1)) * S;
        T* X1 = X0 + (size_t)half * S;
        T* X2 = X1 + (size_t)half * S;
        T* X3 = X2 + (size_t)half * S;
        for (int i = lane; i < v + 1; i += kWave) X1[P0 + i] = X1[i];
        for (int i = lane; i < 2 * v + 2; i += kWave) X2[P0 + i] = X2[i];
        for (int i = lane; i < 3 * v + 3; i += kWave) X3[P0 + i] = X3[i];
        const T* p1 = X1 + v + lane;
        const T* p2 = X2 + 2 * v + lane;
        const T* p3 = X3 + 3 * v + lane;
        const T* p3b = p3 + one;  // x3b and x3d: kept apart from x3a and x3c
        auto unit = [&](int j) {
          const T x0 = X0[j + lane];
          const T x1a = p1[j], x1b = p1[j + 1];
          const T x2a = p2[j], x2b = p2[j + 1], x2c = p2[j + 2];
          const T x3a = p3[j], x3b = p3b[j], x3c = p3[j + 2], x3d = p3b[j + 2];
          const T a0 = x0 + x1a, a1 = x0 + x1b;
          X0[j + lane] = a0 + (x2a + x3a);
          X2[j + lane] = a0 + (x2b + x3b);
          X1[j + lane] = a1 + (x2b + x3c);
          X3[j + lane] = a1 + (x2c + x3d);
        };
        for (int c = 0; c < nfull; ++c) unit(c * kWave);
        if (tail) unit(nfull * kWave);
      }
      l += 2;
    } else {
      // One level: pair (A_v, B_v) of each block of 2*half rows gives
      //   out_{2v}[j] = A_v[j] + B_v[(j + v) mod P0]
      //   out_{2v+1}[j] = A_v[j] + B_v[(j + v + 1) mod P0]
      // written over A_v and B_v.  B's halo holds its bins 0..v.
      for (int p = wave; p < (R >> 1); p += nwaves) {
        const int beta = p >> (l - 1);
        const int v = p & (half - 1);
        T* A = lds + (size_t)(beta * 2 * half + bitrev(v, l - 1)) * S;
        T* B = A + (size_t)half * S;
        const int sh = v < P0 ? v : v % P0;
        const int hn = sh + 1 < H ? sh + 1 : H;  // halo bins this pair reads
        for (int i = lane; i < hn; i += kWave) B[P0 + i] = B[i];
        T* pa = A + lane;
        T* pb = B + lane;
        const T* pb0 = B + sh + lane;
        int c = 0;
        for (; c + 2 <= nfull; c += 2) {
          const T a0 = pa[0], a1 = pa[kWave];
          const T x0 = pb0[0], y0 = pb0[1], x1 = pb0[kWave], y1 = pb0[kWave + 1];
          pa[0] = a0 + x0;
          pb[0] = a0 + y0;
          pa[kWave] = a1 + x1;
          pb[kWave] = a1 + y1;
          pa += 2 * kWave;
          pb += 2 * kWave;
          pb0 += 2 * kWave;
        }
        if (c < nfull) {
          const T a0 = pa[0], x0 = pb0[0], y0 = pb0[1];
          pa[0] = a0 + x0;
          pb[0] = a0 + y0;
          pa += kWave;
          pb += kWave;
          pb0 += kWave;
        }
        if (tail) {
          const T a0 = pa[0], x0 = pb0[0], y0 = pb0[1];
          pa[0] = a0 + x0;
          pb[0] = a0 + y0;
        }
      }
      l += 1;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- selection

template <int E>
__device__ __forceinline__ int count_lt(const uint32_t (&key)[E], uint32_t T) {
  int c = 0;
#pragma unroll
  for (int r = 0; r < E; ++r) c += wave_count(key[r] < T);
  return c;
}

// t-th smallest (0-based) of the `cnt` keys held one per lane in lanes
// 0..cnt-1: quickselect with the first remaining lane as pivot.  Each round
// removes at least the pivot, so it ends within cnt rounds.
__device__ __forceinline__ uint32_t lane_select(uint32_t c, int cnt, int t) {
  const int lane = lane_fresh();
  uint64_t active = __ballot(lane < cnt);
  for (int it = 0; it < kWave; ++it) {
    const int src = __ffsll((unsigned long long)active) - 1;
    const uint32_t p = readlane(c, src);
    const uint64_t lt = active & __ballot(c < p);
    const uint64_t eq = active & __ballot(c == p);
    const int nlt = __popcll(lt), neq = __popcll(eq);
    if (t < nlt) {
      active = lt;
    } else if (t < nlt + neq) {
      return p;
    } else {
      t -= nlt + neq;
      active &= ~(lt | eq);
    }
  }
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)c);  // not reached: the loop returns
}

// Counts of the keys below three pivots: one compare per key and pivot, the
// ballots counted on the scalar unit (the vector unit is the busier one).
template <int E>
__device__ __forceinline__ void count_lt3(const uint32_t (&key)[E], const uint32_t (&t)[3], int (&c)[3]) {
  int c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    c0 += wave_count(key[r] < t[0]);
    c1 += wave_count(key[r] < t[1]);
    c2 += wave_count(key[r] < t[2]);
  }
  c[0] = c0;
  c[1] = c1;
  c[2] = c2;
}

// Three ascending first pivots for a selection (a guess from the profile's
// moments); any pivots keep it exact.
struct Prior {
  bool on;
  uint32_t t[3];
};

// What a wave carries from one profile to the next for the first pivots:
// the profiles' common mean and the spread of the last one (0: unknown).
struct WavePrior {
  float mean;
  float sd;
};

struct SelectKnobs {
  int max_iters;  // counting rounds before the full-sort fallback
  int max_cand;   // candidates small enough for lane_select (<= 64)
};

// Exact order statistics v1 = key_(k1) and v2 = key_(k2), k2 in {k1, k1+1},
// of the n real keys in key[E] (pads are kPadKey), given a bracket [lo0, hi0)
// of the real keys.  An end given as 0 (lo0) or kPadKey (hi0) is open: if the
// first round leaves it so, it becomes the keys' minimum (maximum + 1), so
// the extremes are reduced across the wave only when the pivots miss.  A bracket [lo, hi) holding both targets is narrowed by counting
// keys below a pivot (one ballot per register).  With a prior (E <= 8) the
// first round counts its three pivots at once; later pivots interpolate the
// ranks inside the bracket, falling back to halving it when a round gains
// little.
// Once at most max_cand keys remain in the bracket they are compacted into
// the wave's LDS scratch and selected exactly.  FKEY: keys encode floats, so
// interpolation happens on the float values.  Every exit is exact.
template <int E, bool FKEY>
__device__ __forceinline__ void select_pair(const uint32_t (&key)[E], int n, int k1, int k2, uint32_t lo0,
                            uint32_t hi0, uint32_t* scratch, SelectKnobs kn, const Prior& pr,
                            uint32_t& v1, uint32_t& v2) {
  const int lane = lane_fresh();
  uint32_t lo = lo0, hi = hi0;
  int c_lo = 0, c_hi = n;              // keys below lo / below hi
  bool halve = false;
  int side = 0;         // +1: hi moved last round, -1: lo moved
  float wlo = 1.0f, whi = 1.0f;  // Illinois weights of the bracket ends
  // the straddle exit: k1 < count(keys < T) <= k2 puts v1 below T, v2 above
  auto straddle = [&](uint32_t T) {
    uint32_t mx = 0u, mn = kPadKey;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      if (key[r] < T) mx = umax(mx, key[r]);
      else mn = umin(mn, key[r]);
    }
    v1 = wave_umax(mx);
    v2 = wave_umin(mn);
  };
  if constexpr (E <= 8) {
    if (pr.on) {  // first round: the three guessed pivots at once
      int c[3];
      count_lt3(key, pr.t, c);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const uint32_t T = pr.t[j];
        if (T <= lo || T >= hi) continue;
        if (c[j] <= k1) {
          lo = T;
          c_lo = c[j];
        } else if (c[j] > k2) {
          hi = T;
          c_hi = c[j];
        } else {
          straddle(T);
          return;
        }
      }
    }
  }
  if (lo == 0u) {  // open lower end: the smallest key (count below it is 0)
    uint32_t mn = kPadKey;
#pragma unroll
    for (int r = 0; r < E; ++r) mn = umin(mn, key[r]);
    lo = wave_umin(mn);
  }
  if (hi == kPadKey) {  // open upper end: just above the largest real key (real keys < kPadKey)
    uint32_t mx = 0u;
#pragma unroll
    for (int r = 0; r < E; ++r) mx = umax(mx, key[r] != kPadKey ? key[r] : 0u);
    hi = wave_umax(mx) + 1u;
  }
  // Rounds past max_iters only halve the key range, which ends the loop
  // within 33 more rounds (the range is at most 2^32).
  for (int it = 0; it < kn.max_iters + 34; ++it) {
    if (it >= kn.max_iters) halve = true;
    if (hi - lo <= 1u) {  // only the value lo lies in the bracket
      v1 = v2 = lo;
      return;
    }
    const int cand = c_hi - c_lo;
    if (cand <= kn.max_cand) {
      int base = 0;
      const uint32_t span = hi - lo;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const bool in = key[r] - lo < span;  // lo <= key < hi, one compare
        const uint64_t m = __ballot(in);
        const int pos = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (in) scratch[pos] = key[r];
        base += __popcll(m);
      }
      wave_lds_sync();
      const uint32_t c = lane < cand ? scratch[lane] : kPadKey;
      wave_lds_sync();
      const int t1 = k1 - c_lo;
      v1 = lane_select(c, cand, t1);
      if (k2 == k1) {
        v2 = v1;
      } else {
        const int le = wave_count(lane < cand && c <= v1);
        v2 = le > t1 + 1 ? v1 : wave_umin(lane < cand && c > v1 ? c : kPadKey);
      }
      return;
    }
    // pivot T in (lo, hi): regula falsi on rank (target k1 + 1), with the
    // end that stayed put twice in a row down-weighted (Illinois rule)
    const float flo = wlo * ((float)(k1 - c_lo) + 1.0f);
    const float fhi = whi * ((float)(c_hi - k1) - 1.0f);
    const float frac = halve ? 0.5f : (flo + fhi > 0.0f ? flo * __builtin_amdgcn_rcpf(flo + fhi) : 0.5f);
    uint32_t T;
    if (FKEY && it < kn.max_iters) {  // float keys: interpolate / halve the values
      const float a = fval(lo), b = fval(hi - 1u);
      T = fkey(fmaf(frac, b - a, a));
    } else {
      T = lo + (uint32_t)(frac * (float)(hi - lo));
    }
    T = T <= lo ? lo + 1u : (T >= hi ? hi - 1u : T);
    const int c = count_lt(key, T);
    const int before = cand;
    if (c <= k1) {
      lo = T;
      c_lo = c;
      whi = side < 0 ? whi * 0.5f : 1.0f;
      wlo = 1.0f;
      side = -1;
    } else if (c > k2) {
      hi = T;
      c_hi = c;
      wlo = side > 0 ? wlo * 0.5f : 1.0f;
      whi = 1.0f;
      side = 1;
    } else {  // k1 < c <= k2: the two targets straddle T
      straddle(T);
      return;
    }
    halve = (c_hi - c_lo) * 4 > before * 3;
  }
  v1 = lo;  // not reached: the halving rounds end the loop by returning
  v2 = lo;
}

// ----------------------------------------------------------- Algorithm 1

template <bool INT>
struct Types;
template <>
struct Types<true> {
  using T = int32_t;   // stored sums (non-negative, < 2^31)
  using A = uint32_t;  // modular prefix-sum type
};
template <>
struct Types<false> {
  using T = float;
  using A = float;
};

// Registers of a profile's lane layout (bin j in register j/64) that hold 64
// real bins for every P0 that score_dispatch sends to an E-register scorer:
// P0 > 64(E-1) for E <= 8, and above the previous case's bound for the
// larger E.  Their bounds checks then fold away at compile time.
template <int E>
constexpr int kFullRegs = E <= 8 ? E - 1 : (E == 12 ? 8 : (E == 16 ? 12 : (E == 24 ? 16 : 24)));

// Circular prefix sums of the profile in `row`, in place: afterwards row[k] =
// C[k] = sum_{i<k} F[i mod P0] for k <= P0 + wmax, and cex[r] holds C[j] of
// the lane's bin j = 64r + lane.  A box of width w starting at j is then
// C[j + w] - C[j] (modular arithmetic is exact for the integer sums).
template <int E, bool INT>
__device__ __forceinline__ void circular_prefix(typename Types<INT>::T* row, int P0, int wmax,
                                                typename Types<INT>::A (&cex)[E],
                                                typename Types<INT>::T shift = 0) {
  using T = typename Types<INT>::T;
  using A = typename Types<INT>::A;
  const int lane = lane_fresh();
  A xv[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = r * kWave + lane;
    xv[r] = (r < kFullRegs<E> || e < P0) ? (A)(T)(row[e] - shift) : (A)0;
  }
  wave_lds_sync();
  A carry = (A)0;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = r * kWave + lane;
    const A s = wave_scan(xv[r]);
    cex[r] = carry + s - xv[r];
    if (r < kFullRegs<E> || e < P0) row[e + 1] = (T)(carry + s);
    if constexpr (INT) carry += readlane(s, 63);
    else carry += __uint_as_float(readlane(__float_as_uint(s), 63));
  }
  if (lane == 0) row[0] = (T)0;
  wave_lds_sync();
  const A total = carry;
  for (int i = lane; i < wmax; i += kWave) row[P0 + 1 + i] = (T)(total + (A)row[1 + i]);
  wave_lds_sync();
}

// Score one folded profile with Algorithm 2 (paper Sec. 2.2.2, Eq. 5): for
// each width w, the circular boxcar of the profile, its maximum I_max at the
// first position j*; an on-pulse window of L = max(round(P0/5), w) profile
// bins centred on that box (starting at j* + floor((w - L)/2), wrapping); the
// mean I_av and population sigma of the c = P0 - L profile bins outside it
// (themselves a circular run, taken from the lane's own bins in registers,
// mean first, then the squared deviations); and
// A_w = (I_max - w*I_av) / (sigma*sqrt(w)).  Score = max_w A_w, the first
// width on ties, 0 where sigma = 0.  Integer profiles are scored from exact
// integers: with s1 and s2 the kept bins' sum and sum of squares,
// A_w = (c*I_max - w*s1) / (sqrt(c*s2 - s1^2)*sqrt(w)).
template <int E, bool INT>
__device__ __forceinline__ void score_alg2(typename Types<INT>::T* row, int P0, int wmax,
                                           const WidthLanes& wt, int nw, float* snr_out,
                                           int32_t* width_out) {
  using T = typename Types<INT>::T;
  using A = typename Types<INT>::A;
  const int lane = lane_id();
  // Up to 16 boxes per lane are held in registers; longer profiles re-read
  // them from the prefix sums in LDS in each sweep, in a plain loop.
  constexpr bool kRegs = E <= 16;
  constexpr int ER = kRegs ? E : 1;
  T fv[E];  // the lane's profile bins, kept for the off-pulse statistics
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = r * kWave + lane;
    fv[r] = (r < kFullRegs<E> || e < P0) ? row[e] : (T)0;
  }
  // Float profiles: the boxes come from prefix sums of the profile shifted by
  // its bin nearest the mean, which keeps them as precise as their own bins
  // whatever the profile's offset (and exact where the bins are exact small
  // multiples of a power of two, so exact ties stay ties); the shift is added
  // back in double.
  float shift = 0.f;
  if constexpr (!INT) {
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < E; ++r) t += (double)fv[r];  // pads hold 0
    const double mean_all = wave_sum(t) / (double)P0;
    float bd = INFINITY, bv = 0.f;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = r * kWave + lane;
      const float d = (float)fabs((double)fv[r] - mean_all);
      if ((r < kFullRegs<E> || e < P0) && d < bd) {
        bd = d;
        bv = fv[r];
      }
    }
    const uint32_t kd = fkey(bd), kmin = wave_umin(kd);
    const int src = __ffsll((unsigned long long)__ballot(kd == kmin)) - 1;
    shift = __uint_as_float(readlane(__float_as_uint(bv), src));
  }
  A cex[ER];
  {
    A cex_all[E];
    if constexpr (!INT) circular_prefix<E, INT>(row, P0, wmax, cex_all, shift);
    else circular_prefix<E, INT>(row, P0, wmax, cex_all);
    if constexpr (kRegs) {
#pragma unroll
      for (int r = 0; r < E; ++r) cex[r] = cex_all[r];
    }
  }
  const int n_ex = (2 * P0 + 5) / 10;  // round(P0/5)
  auto key_of = [](A v) -> uint32_t {
    if constexpr (INT) return (uint32_t)v;
    else return fkey(v);
  };
  double best = 0.0;
  int32_t bw = 0;
  for (int i = 0; i < nw; ++i) {
    const int32_t w = wt.width(i);
    A breg[ER];
    if constexpr (kRegs) {
#pragma unroll
      for (int r = 0; r < E; ++r) breg[r] = (A)row[r * kWave + lane + w] - cex[r];
    }
    // maximum and its first position
    uint32_t mk = 0u, jf = 0xffffffffu;
    auto visit = [&](auto&& f) {
      if constexpr (kRegs) {
#pragma unroll
        for (int r = 0; r < E; ++r)
          if (r < kFullRegs<E> || r * kWave + lane < P0) f(r * kWave + lane, breg[r]);
      } else {
        for (int e = lane; e < P0; e += kWave) f(e, (A)row[e + w] - (A)row[e]);
      }
    };
    visit([&](int e, A b) {
      const uint32_t kv = key_of(b);
      if (kv > mk) {
        mk = kv;
        jf = (uint32_t)e;
      }
    });
    const uint32_t pk = wave_umax(mk);
    const int jstar = (int)wave_umin(mk == pk ? jf : 0xffffffffu);
    // the on-pulse window [start, start + L) and the kept run after it
    const int L = w > n_ex ? w : n_ex;
    int kb = jstar + ((w - L) >> 1) + L;  // start + L, start = j* + floor((w - L)/2)
    kb += kb < 0 ? P0 : 0;
    kb -= kb >= P0 ? P0 : 0;
    const int c = P0 - L;
    auto kept = [&](int r) {  // bin r*64 + lane is real and outside the window
      const int e = r * kWave + lane;
      int d = e - kb;
      d += d < 0 ? P0 : 0;
      return (r < kFullRegs<E> || e < P0) && d < c;
    };
    double a = 0.0;
    if constexpr (INT) {
      int64_t s1 = 0, s2 = 0;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int64_t v = kept(r) ? (int64_t)fv[r] : 0;
        s1 += v;
        s2 += v * v;
      }
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      const int64_t D = (int64_t)c * s2 - s1 * s1;
      const int64_t num = (int64_t)c * (int64_t)pk - (int64_t)w * s1;
      a = (c > 1 && D > 0) ? (double)num / (sqrt((double)D) * wt.sqrtw(i)) : 0.0;
    } else if (c > 1) {
      double s1 = 0.0;
#pragma unroll
      for (int r = 0; r < E; ++r) s1 += kept(r) ? (double)fv[r] : 0.0;
      const double mean = wave_sum(s1) / (double)c;
      double s2 = 0.0;
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const double dv = kept(r) ? (double)fv[r] - mean : 0.0;
        s2 = fma(dv, dv, s2);
      }
      const double var = wave_sum(s2) / (double)c;
      // the box maximum is of the shifted profile: I_max - w*I_av is
      // max_c - w*(I_av - shift)
      a = var > 0.0 ? ((double)fval(pk) - (double)w * (mean - (double)shift)) / (sqrt(var) * wt.sqrtw(i)) : 0.0;
    }
    if (i == 0 || a > best) {
      best = a;
      bw = w;
    }
  }
  if (lane == 0) {
    *snr_out = (float)best;
    *width_out = bw;
  }
}

// Score one folded profile with Algorithm 1 (paper Sec. 2.2.1): median and
// MAD of the profile (Eqs. 3-4), circular boxcars of every width, score =
// max_w (max_j box_w[j] - w*median) / (K*MAD*sqrt(w)).  The wave works on one
// profile held in LDS `row` (room for P0 + wmax + 1 entries); the row is
// overwritten with circular prefix sums.  Bin j of the profile sits in
// register j/64 of lane j%64.
//
// Integer profiles are scored exactly: med2 = 2*median, mad4 = 4*MAD, and
// S/N = 2*(2*peak - w*med2) / ((K*mad4)*sqrt(w)) in double with sqrt(w) from
// a host table, so every rounding is a correctly rounded IEEE operation.
template <int E, bool INT>
__device__ __forceinline__ void score_profile(typename Types<INT>::T* row, uint32_t* scratch, int P0, int wmax,
                              const WidthLanes& wt, int nw, SelectKnobs kn, WavePrior& wp, float* snr_out,
                              int32_t* width_out) {
  using T = typename Types<INT>::T;
  using A = typename Types<INT>::A;
  const int lane = lane_fresh();
  const int k1 = (P0 - 1) / 2;
  const int k2 = P0 / 2;

  uint32_t key[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int e = r * kWave + lane;
    const bool real = r < kFullRegs<E> || e < P0;
    if constexpr (INT) key[r] = real ? (uint32_t)row[e] : kPadKey;
    else key[r] = real ? fkey(row[e]) : kPadKey;
  }
  // Mean and spread of the profile in float: they only place the selections'
  // first pivots (about 2.5 standard errors either side of the expected
  // median and MAD of normal noise).  Every profile of an FFA execution sums
  // the same samples, so the mean is shared; the spread is taken from the
  // previous profile's MAD.  The wave's first profile, and any after a zero
  // MAD, computes both from its moments.
  Prior pm{false, {0u, 0u, 0u}}, pd{false, {0u, 0u, 0u}};
  float sd = 0.f;
  if constexpr (E <= 8) {
    if (__builtin_amdgcn_readfirstlane(wp.sd > 0.f ? 1 : 0) == 0) {
      float s1 = 0.f, s2 = 0.f;
      uint32_t kmin = kPadKey;  // moments about the smallest value, for their precision
#pragma unroll
      for (int r = 0; r < E; ++r) kmin = umin(kmin, key[r]);
      kmin = wave_umin(kmin);
      const float base = INT ? (float)kmin : fval(kmin);
#pragma unroll
      for (int r = 0; r < E; ++r) {
        if (r < kFullRegs<E> || r * kWave + lane < P0) {
          const float y = INT ? (float)(key[r] - kmin) : fval(key[r]) - base;
          s1 += y;
          s2 += y * y;
        }
      }
      s1 = __uint_as_float(readlane(__float_as_uint(wave_scan(s1)), 63));
      s2 = __uint_as_float(readlane(__float_as_uint(wave_scan(s2)), 63));
      const float inv = __builtin_amdgcn_rcpf((float)P0);
      const float mu_y = s1 * inv;
      const float var = s2 * inv - mu_y * mu_y;
      wp.mean = uniform(base + mu_y);
      wp.sd = uniform(var > 0.f ? __builtin_sqrtf(var) : 0.f);
    }
    sd = wp.sd;
    const float h = 2.5f * sd * __builtin_amdgcn_rsqf((float)P0);
    pm.on = __builtin_amdgcn_readfirstlane(sd > 0.f ? 1 : 0) != 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float u = wp.mean + (float)(j - 1) * h;
      if constexpr (INT) pm.t[j] = uniform_u32((uint32_t)fminf(fmaxf(u, 0.f), 4294967040.f));
      else pm.t[j] = uniform_u32(fkey(u));
    }
  }

  // median (even P0: mean of the two middle order statistics)
  uint32_t m1, m2;
  select_pair<E, !INT>(key, P0, k1, k2, 0u, kPadKey, scratch, kn, pm, m1, m2);
  uint64_t med2 = 0;
  float med = 0.f;
  double med_d = 0.0;
  if constexpr (INT) {
    med2 = (uint64_t)m1 + (uint64_t)m2;
  } else {
    med_d = 0.5 * ((double)fval(m1) + (double)fval(m2));
    med = (float)med_d;
  }
  // MAD: the same selection on |x - median| (doubled for integers)
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const bool real = r < kFullRegs<E> || r * kWave + lane < P0;
    if constexpr (INT) {  // 2*x and med2 are below 2^32 (sums below 2^31)
      const uint32_t tx = 2u * key[r], m2 = (uint32_t)med2;
      key[r] = real ? (tx >= m2 ? tx - m2 : m2 - tx) : kPadKey;
    } else {  // from the profile in LDS: the key of a value >= 0 is its bits with the top bit set
      key[r] = real ? (__float_as_uint(fabsf(row[r * kWave + lane] - med)) | 0x80000000u) : kPadKey;
    }
  }
  const uint32_t dmin = INT ? 0u : fkey(0.f);
  if constexpr (E <= 8) {
    // the MAD of normal noise is 0.6745 sd (doubled for integers)
    const float m = (INT ? 2.f : 1.f) * 0.6745f * sd;
    const float e = 2.4f * __builtin_amdgcn_rsqf((float)P0);
    pd.on = __builtin_amdgcn_readfirstlane(sd > 0.f ? 1 : 0) != 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float v = m * (1.f + (float)(j - 1) * e);
      if constexpr (INT) pd.t[j] = uniform_u32((uint32_t)fminf(fmaxf(v, 0.f), 4294967040.f));
      else pd.t[j] = uniform_u32(fkey(fmaxf(v, 0.f)));
    }
  }
  uint32_t d1, d2;
  select_pair<E, !INT>(key, P0, k1, k2, dmin, kPadKey, scratch, kn, pd, d1, d2);
  uint64_t mad4 = 0;
  float mad = 0.f;
  bool mad_zero;
  if constexpr (INT) {
    mad4 = (uint64_t)d1 + (uint64_t)d2;
    mad_zero = mad4 == 0;
  } else {
    mad = (float)(0.5 * ((double)fval(d1) + (double)fval(d2)));
    mad_zero = mad == 0.f;
  }
  // the spread of normal noise with this MAD, for the next profile's pivots
  if constexpr (INT) wp.sd = uniform((float)(0.25 * kMadK) * (float)mad4);
  else wp.sd = uniform((float)kMadK * mad);
  if (mad_zero) {
    if (lane == 0) {
      *snr_out = 0.f;
      *width_out = 0;
    }
    return;
  }

  // Float profiles are shifted by their median before the prefix sums, so a
  // box C[j+w] - C[j] keeps the precision of its own bins whatever the
  // profile's offset; the shift is added back exactly in double below.  On a
  // skewed profile, whose mean lies more than 3 K*MAD/sqrt(P0) from its median
  // (about a 4-sigma event for normal noise), the running sum of x - median
  // drifts to P0 * (mean - median), and its float32 rounding grows large
  // against the MAD; such a profile is shifted by the profiles' shared mean
  // instead (where the wave holds it, E <= 8), about which the running sum
  // returns to zero.
  float cshift = med;
  if constexpr (E <= 8) {
    const float dm = wp.mean - med;  // compared squared: no square root
    if (__builtin_amdgcn_readfirstlane(dm * dm * (float)P0 > 9.f * wp.sd * wp.sd ? 1 : 0)) cshift = wp.mean;
  }
  A cex[E];  // C[j] (exclusive prefix) of this lane's bins
  if constexpr (!INT) circular_prefix<E, INT>(row, P0, wmax, cex, cshift);
  else circular_prefix<E, INT>(row, P0, wmax, cex);

  // Each width's score is num_w / ((K*MAD)*sqrt(w)), the box maximum taken
  // over all positions.
  const double scale = INT ? kMadK * (double)mad4 : kMadK * (double)mad;
  // Pass 1: the largest box of each width (wave-uniform), kept in lane i for
  // width i (as a key for floats).  Two widths per iteration for ILP.
  const int nfull = P0 / kWave;  // registers holding 64 real bins
  auto lane_max = [&](int32_t w) -> A {
    A mx;  // box sums are >= 0 for integers
    if constexpr (INT) mx = 0u;
    else mx = -INFINITY;
    const T* rw = row + w + lane;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      if (r < kFullRegs<E> || r < nfull) {  // wave-uniform branch
        const A b = (A)rw[r * kWave] - cex[r];
        if constexpr (INT) mx = umax(mx, b);
        else mx = fmaxf(mx, b);
      } else if (r == nfull && lane < P0 - r * kWave) {
        const A b = (A)rw[r * kWave] - cex[r];
        if constexpr (INT) mx = umax(mx, b);
        else mx = fmaxf(mx, b);
      }
    }
    return mx;
  };
  auto as_key = [](A v) -> uint32_t {
    if constexpr (INT) return v;
    else return fkey(v);
  };
  uint32_t pk_l = 0;
  int i = 0;
  for (; i + 8 <= nw; i += 8) {  // eight widths reduced together
    uint32_t m8[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) m8[k] = as_key(lane_max(wt.width(i + k)));
    const uint32_t p8 = wave_umax8(m8);
    pk_l = (uint32_t)(lane - i) < 8u ? p8 : pk_l;
  }
  for (; i + 2 <= nw; i += 2) {
    const A m0 = lane_max(wt.width(i)), m1 = lane_max(wt.width(i + 1));
    const uint32_t p0 = wave_umax(as_key(m0)), p1 = wave_umax(as_key(m1));
    pk_l = lane == i ? p0 : (lane == i + 1 ? p1 : pk_l);
  }
  if (i < nw) {
    const uint32_t p0 = wave_umax(as_key(lane_max(wt.width(i))));
    pk_l = lane == i ? p0 : pk_l;
  }
  // Pass 2, lane i = width i: num_i, and the ranking value num_i / sqrt(w_i)
  // up to the common factor.  The exact score num / (scale * sqrt(w)) is
  // computed for the widths within 1e-12 of the largest ranking value only;
  // any other width scores strictly lower, so the maximum and the first-width
  // tie rule are those of scoring every width.
  const bool live = lane < nw;
  double num;
  if constexpr (INT) num = (double)(2 * (2 * (int64_t)pk_l - (int64_t)wt.w * (int64_t)med2));
  else num = (double)fval(pk_l) - (double)wt.w * (med_d - (double)cshift);
  const double a = live ? num * wt.isq : -INFINITY;
  const bool row0 = nw <= 16;  // every width's lane is in the first row
  const double amax = row0 ? row_dmax16(a) : wave_dmax(a);
  const bool cand = live && a >= amax - 1e-12 * fabs(amax);
  const double sc = cand ? num / (scale * wt.sq) : -INFINITY;
  const double best = row0 ? row_dmax16(sc) : wave_dmax(sc);
  const uint64_t hit = __ballot(cand && sc == best);
  const int first = __ffsll((unsigned long long)hit) - 1;
  const int32_t bw = wt.width(first);
  if (lane == 0) {
    *snr_out = (float)best;
    *width_out = bw;
  }
}

// EMAX bounds the registers per lane the kernel is compiled for; profiles of
// P0 <= 64*EMAX are scored (the launcher picks EMAX from the largest P0).
template <bool INT, int EMAX, int ALG>
__device__ __forceinline__ void score_dispatch(typename Types<INT>::T* row, uint32_t* scratch, int P0, int wmax,
                               const WidthLanes& wt, int nw, SelectKnobs kn, WavePrior& wp, float* snr_out,
                               int32_t* width_out) {
  // P0, the width count and the widest width are fixed for a tile, so the
  // compiler would hoist everything derived from them (the per-register bounds
  // masks above all) out of the loop over a wave's profiles. Held across that
  // loop they overflow the 80 scalar registers a wave has at 8 waves per SIMD,
  // and the spills to vector-register lanes cost two readlanes per use. Marked
  // as redefined here, they are derived again for each profile.
  asm volatile("" : "+s"(P0), "+s"(nw), "+s"(wmax));
#define FFA_SCORE(EE)                                                                              \
  do {                                                                                             \
    if constexpr (ALG == 2)                                                                        \
      score_alg2<EE, INT>(row, P0, wmax, wt, nw, snr_out, width_out);                              \
    else                                                                                           \
      score_profile<EE, INT>(row, scratch, P0, wmax, wt, nw, kn, wp, snr_out, width_out);         \
  } while (0)
  if (P0 <= 64) FFA_SCORE(1);
  else if (P0 <= 128) FFA_SCORE(2);
  else if (P0 <= 192) FFA_SCORE(3);
  else if (P0 <= 256) FFA_SCORE(4);
  else if (P0 <= 320) FFA_SCORE(5);
  else if (P0 <= 384) FFA_SCORE(6);
  else if (P0 <= 448) FFA_SCORE(7);
  else if (P0 <= 512) FFA_SCORE(8);
  else if constexpr (EMAX >= 16) {
    if (P0 <= 768) FFA_SCORE(12);
    else if (P0 <= 1024) FFA_SCORE(16);
    else if constexpr (EMAX >= 32) {
      if (P0 <= 1536) FFA_SCORE(24);
      else FFA_SCORE(32);
    }
  }
#undef FFA_SCORE
}

// Copy a tile's 2^d rows (R rows of P0 bins, contiguous at src) into LDS
// rows of stride S; rows >= valid are zero padding (paper Sec. 2.1).  Each
// wave copies two whole rows at a time, its lanes walking the bins in chunks
// of 64: up to 16 loads in flight per lane, addressed by immediate offsets
// from one base per row and group of 8 chunks.  TL may be narrower than TS
// when the caller knows the values fit.
template <typename TL, typename TS>
__device__ __forceinline__ void stage_rows(TL* lds, const TS* src, int R, int valid, int P0, int S) {
  const int lane = lane_id();
  const int wave = wave_id();
  const int nwaves = blockDim.x / kWave;
  const int nfull = P0 / kWave;
  const bool tail = nfull * kWave + lane < P0;
  for (int r0 = wave; r0 < R; r0 += 2 * nwaves) {
    const int r1 = r0 + nwaves;
    const bool has1 = r1 < R;
    const bool in0 = r0 < valid, in1 = r1 < valid;
    const TS* s0 = src + (size_t)r0 * P0 + lane;
    const TS* s1 = src + (size_t)r1 * P0 + lane;
    TL* d0 = lds + (size_t)r0 * S + lane;
    TL* d1 = lds + (size_t)r1 * S + lane;
    for (int c0 = 0; c0 < nfull; c0 += 8) {
      TS a[8], b[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c0 + c < nfull) {
          a[c] = in0 ? s0[(c0 + c) * kWave] : (TS)0;
          b[c] = in1 ? s1[(c0 + c) * kWave] : (TS)0;
        }
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c0 + c < nfull) {
          d0[(c0 + c) * kWave] = (TL)a[c];
          if (has1) d1[(c0 + c) * kWave] = (TL)b[c];
        }
      }
    }
    if (tail) {
      const TS a = in0 ? s0[nfull * kWave] : (TS)0;
      const TS b = in1 ? s1[nfull * kWave] : (TS)0;
      d0[nfull * kWave] = (TL)a;
      if (has1) d1[nfull * kWave] = (TL)b;
    }
  }
}

// stage_rows for 4-byte rows through the LDS DMA path: every whole chunk of
// 64 bins of a row with data goes from global memory straight into LDS
// (global_load_lds_dword, no registers), all of a wave's chunks in flight at
// once; the row tails and the zero rows take ordinary stores.  The caller's
// barrier follows the wait for the DMA below.
template <typename T>
__device__ __forceinline__ void stage_rows_dma(T* lds, const T* src, int R, int valid, int P0, int S) {
  static_assert(sizeof(T) == 4, "4-byte rows");
  const int lane = lane_id();
  const int wave = wave_id();
  const int nwaves = blockDim.x / kWave;
  const int nfull = P0 / kWave;
  const bool tail = nfull * kWave + lane < P0;
  for (int r = wave; r < R; r += nwaves) {
    T* d = lds + (size_t)r * S;
    if (r < valid) {
      const T* g = src + (size_t)r * P0 + lane;
      for (int c = 0; c < nfull; ++c)
        __builtin_amdgcn_global_load_lds(g + c * kWave, d + c * kWave, 4, 0, 0);
      if (tail) d[nfull * kWave + lane] = g[nfull * kWave];
    } else {
      for (int c = 0; c < nfull; ++c) d[c * kWave + lane] = (T)0;
      if (tail) d[nfull * kWave + lane] = (T)0;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
}

// Hand partial t of a first-pass tile (LDS row bitrev(t, d)) to the next
// pass, rotated left by t*h bins, at out0 + t*dst_step: the levels above
// this pass then act on the rotated rows like a plain FFA tree.
template <typename TL, typename TO>
__device__ __forceinline__ void write_partials(const TL* lds, TO* out0, int R, int d, int S, int P0,
                                               int64_t dst_step, int h) {
  const int lane = lane_id();
  const int wave = wave_id();
  const int nwaves = blockDim.x / kWave;
  for (int tt = wave; tt < R; tt += nwaves) {
    const TL* srow = lds + (size_t)bitrev(tt, d) * S;
    const int rot = (int)(((int64_t)tt * h) % P0);
    TO* out = out0 + (int64_t)tt * dst_step;
    for (int j = lane; j < P0; j += kWave) {
      int i = j + rot;
      i -= (i >= P0) ? P0 : 0;
      out[j] = (TO)srow[i];
    }
  }
}

// ------------------------------------------------------------- tile kernel

// One workgroup per tile.  A launch covers tiles whose inputs were all
// written by earlier launches on the stream (the planner's windows), so
// workgroups never wait on one another.  For profiles of up to 512 bins the
// registers are held to 8 waves per SIMD, so two workgroups share a CU when
// their tiles' LDS allows it.
template <bool INT, int EMAX, int ALG>
__global__ __launch_bounds__(kThreads, EMAX <= 8 ? 8 : 4) void ffa_tile_kernel(TileArgs a, void* __restrict__ ws_raw) {
  using T = typename Types<INT>::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  T* ws = reinterpret_cast<T*>(ws_raw);
  const SelectKnobs kn{a.select_iters, a.select_cand};
  const int lane = lane_id();
  const int wave = wave_id();
  const int nwaves = blockDim.x / kWave;

  const int64_t t = a.tile0 + blockIdx.x;
  const Phase ph = a.phases[a.tile_phase ? a.tile_phase[t] : 0];
  const int32_t k = (int32_t)(t - ph.tile0);
  const int32_t q = k / ph.ng;
  const int32_t h = k - q * ph.ng;
  const int64_t buf0 = a.ring_off + (int64_t)ph.ring64 * 64;
  const int64_t buf1 = buf0 + (int64_t)ph.M * ph.P0;

  // geometry of this tile
  const int d = ph.depth;
  const int R = 1 << d;
  const int P0 = ph.P0;
  const int S = ph.stride;
  const int H = ph.halo;
  const int64_t Gin = (int64_t)ph.M >> ph.D;
  const int64_t in_base = ph.pass == 0 ? a.oct_base + ph.oct_off : ((ph.pass - 1) & 1 ? buf1 : buf0);
  const int64_t src_off = in_base + ((int64_t)q * Gin + ((int64_t)h << d)) * P0;
  const int valid = min(R, ph.vin - (h << d));

  if constexpr (INT) {
    if (ph.u16) {  // a first pass whose sums stay below 2^16 (the planner checks)
      uint16_t* l16 = reinterpret_cast<uint16_t*>(lds_raw);
      stage_rows(l16, ws + src_off, R, valid, P0, S);
      __syncthreads();
      butterfly<uint16_t>(l16, S, P0, H, d);
      const int64_t Gout = Gin >> d;
      write_partials(l16, ws + ((ph.pass & 1) ? buf1 : buf0) + (((int64_t)q << d) * Gout + h) * P0, R, d, S, P0,
                     Gout * P0, h);
      return;
    }
  }
  // The DMA loads are issued at raised wave priority, so a workgroup that is
  // staging gets its loads in flight ahead of the other workgroup's scoring
  // on the same SIMDs.
  __builtin_amdgcn_s_setprio(3);
  stage_rows_dma(lds, ws + src_off, R, valid, P0, S);
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();

  butterfly<T>(lds, S, P0, H, d);

  if (!ph.last) {
    // Hand partial t to the next pass rotated left by t*h bins: the levels
    // above this pass then act on the rotated rows like a plain FFA tree.
    const int64_t Gout = Gin >> d;
    write_partials(lds, ws + ((ph.pass & 1) ? buf1 : buf0) + (((int64_t)q << d) * Gout + h) * P0, R, d, S, P0,
                   Gout * P0, h);
  } else if (a.mode == kModeProfiles) {
    T* out = reinterpret_cast<T*>(a.profiles) +
             (ph.first_trial + ((int64_t)q << d) - a.trial_base) * (int64_t)P0;
    for (int tt = wave; tt < R; tt += nwaves) {
      const T* srow = lds + (size_t)bitrev(tt, d) * S;
      T* o = out + (int64_t)tt * P0;
      for (int j = lane; j < P0; j += kWave) o[j] = srow[j];
    }
  } else {
    uint32_t* scratch = reinterpret_cast<uint32_t*>(lds + (size_t)R * S) + wave * kWave;
    const int32_t* widths = a.widths + ph.wofs;
    const double* sw = a.sqrtw + ph.wofs;
    const double* isw = a.sqrtw + ph.isqrt_ofs;
    WidthLanes wt;
    wt.w = lane < ph.nw ? widths[lane] : 0;
    wt.sq = lane < ph.nw ? sw[lane] : 1.0;
    wt.isq = lane < ph.nw ? isw[lane] : 1.0;
    const int wmax = (int)wave_umax((uint32_t)wt.w);
    const int64_t trial0 = ph.first_trial + ((int64_t)q << d);
    // a batch's tiles write their own series' periodogram
    float* snr_out = a.snr;
    int32_t* width_out = a.width;
    if (a.outs) {
      const SeriesOut so = a.outs[ph.series];
      snr_out = so.snr;
      width_out = so.width;
    }
    WavePrior wp{0.f, 0.f};
    for (int tt = wave; tt < R; tt += nwaves) {
      T* row = lds + (size_t)bitrev(tt, d) * S;
      const int64_t trial = trial0 + tt;
      score_dispatch<INT, EMAX, ALG>(row, scratch, P0, wmax, wt, ph.nw, kn, wp, snr_out + trial, width_out + trial);
    }
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

// ------------------------------------------------------------ dereddening
//
// Running-median dereddening (paper Sec. 2.3.1): the median of the window at
// every knot t_c = c*stride, then the linearly interpolated baseline is
// subtracted.  One workgroup per knot finds the median by radix selection on
// order-preserving keys (staged in LDS when the window fits): one pass per
// 8-bit digit counts the keys that share the digits found so far into an
// LDS histogram, and a block-wide scan of the 256 bins finds the digit that
// holds the target rank.  For an even count the upper middle value is the
// lower one again if it repeats, else the smallest key above it.  The
// medians are kept in double and the baseline is subtracted in double, so
// the series (exact int32 sums for uint8 input, float otherwise) is rounded
// once, to the float32 output written over it.

constexpr int kKnotThreads = 256;   // one thread per histogram bin
constexpr int kKnotStage = 4096;    // window keys staged in LDS

__device__ __forceinline__ uint32_t series_key(int32_t v) { return (uint32_t)v; }  // sums are >= 0
__device__ __forceinline__ uint32_t series_key(float v) { return fkey(v); }
__device__ __forceinline__ uint64_t series_key(double v) {  // order-preserving, like fkey
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return b ^ ((b >> 63) ? ~0ull : 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(uint32_t k, int32_t) { return (double)k; }
__device__ __forceinline__ double key_value(uint32_t k, float) { return (double)fval(k); }
__device__ __forceinline__ double key_value(uint64_t k, double) {
  return __longlong_as_double((long long)(k ^ ((k >> 63) ? 0x8000000000000000ull : ~0ull)));
}

// k-th smallest (0-based) key of x[lo..hi) (all threads return it).
template <typename T>
__global__ __launch_bounds__(kKnotThreads) void knot_median_kernel(const T* __restrict__ x, int64_t n,
                                                                   int32_t window, int32_t stride,
                                                                   double* __restrict__ med) {
  using K = decltype(series_key(T()));
  constexpr int kBits = 8 * (int)sizeof(K);
  __shared__ K skeys[kKnotStage];
  __shared__ uint32_t hist[kKnotThreads];
  __shared__ uint32_t wsum[kKnotThreads / kWave];
  __shared__ uint32_t s_digit, s_eq;
  __shared__ int64_t s_below;
  __shared__ K s_min;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = wave_id();
  const int64_t c = blockIdx.x;
  const int64_t t = c * stride;
  int64_t lo = t - window / 2, hi = lo + window;
  lo = lo < 0 ? 0 : lo;
  hi = hi > n ? n : hi;
  const int64_t cnt = hi - lo;
  if (cnt <= 0) {  // not reached for knots inside the series
    if (tid == 0) med[c] = 0.0;
    return;
  }
  const bool staged = cnt <= kKnotStage;
  if (staged)
    for (int64_t i = tid; i < cnt; i += kKnotThreads) skeys[i] = series_key(x[lo + i]);
  auto key_at = [&](int64_t i) -> K { return staged ? skeys[i] : series_key(x[lo + i]); };
  // rank (cnt - 1) / 2, one 8-bit digit per pass, most significant first
  int64_t k = (cnt - 1) / 2;
  K prefix = 0;
  uint32_t eq = 0;  // keys equal to the result, after the last pass
  for (int shift = kBits - 8; shift >= 0; shift -= 8) {
    hist[tid] = 0u;
    __syncthreads();
    const K hmask = shift == kBits - 8 ? (K)0 : (K)(~(K)0 << (shift + 8));
    for (int64_t i = tid; i < cnt; i += kKnotThreads) {
      const K key = key_at(i);
      if ((key & hmask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    // thread b owns bin b: keys below the bin = exclusive prefix over bins
    const uint32_t h = hist[tid];
    const uint32_t incl = wave_scan(h);
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    const int64_t below = (int64_t)(base + incl - h);
    if (k >= below && k < below + (int64_t)h) {  // exactly one bin holds rank k
      s_digit = (uint32_t)tid;
      s_below = below;
      s_eq = h;
    }
    __syncthreads();
    prefix |= (K)s_digit << shift;
    k -= s_below;
    eq = s_eq;
    __syncthreads();
  }
  double m = key_value(prefix, T());
  if (cnt % 2 == 0) {
    K v2 = prefix;
    if (k + 1 >= (int64_t)eq) {  // rank cnt/2 is the smallest key above
      if (tid == 0) s_min = ~(K)0;
      __syncthreads();
      K mn = ~(K)0;
      for (int64_t i = tid; i < cnt; i += kKnotThreads) {
        const K key = key_at(i);
        if (key > prefix && key < mn) mn = key;
      }
      if constexpr (sizeof(K) == 8)
        atomicMin(reinterpret_cast<unsigned long long*>(&s_min), (unsigned long long)mn);
      else
        atomicMin(reinterpret_cast<unsigned int*>(&s_min), (unsigned int)mn);
      __syncthreads();
      v2 = s_min;
    }
    m = 0.5 * (m + key_value(v2, T()));
  }
  if (tid == 0) med[c] = m;
}

// ------------------------------------------- exact running median (stride 1)
//
// The median of the window at every sample, in blocks of kRmBlock
// consecutive outputs per workgroup.  The windows of a block overlap in a
// core C (the samples every one of them holds); output i's window is C plus
// at most kRmBlock - 1 fringe samples.  So the rank-k value of window i lies
// between the core's values of rank k - f_i and k (f_i its fringe count),
// and every median of the block lies between the core's values of the
// smallest and largest such ranks.  With the core's values in equal buckets,
// the union's values in the buckets qa..qb holding those two ranks form a
// small pool, sorted once; output i's median is the value of rank
// k - below_i among the pool entries inside its window, below_i being the
// count of its window's values in buckets below qa.  Each selection is exact; blocks
// whose pool would overflow (many equal values), whose windows share no core
// (windows shorter than the block) or that are too long to stage in LDS
// select every output's median directly instead.

constexpr int kRmBlock = 256;     // outputs per workgroup
constexpr int kRmThreads = 1024;  // threads per workgroup (the passes over a window use all)
constexpr int kRmPool = 1024;     // pool entries
constexpr int kRmStageMax = 16384;  // window values staged in LDS (doubles)
constexpr int kRmBins = 1024;      // buckets of the pass that bounds the medians

struct RmShared {
  double pool_v[kRmPool];
  int16_t pool_p[kRmPool];    // union index of each pool entry
  int16_t core_at[kRmPool];   // pool index of the r-th core entry, in value order
  int16_t fr_at[kRmPool];     // pool index of the j-th fringe entry, in value order
  int16_t fr_p[kRmPool];      // its union index
  double cand[kRmBlock];
  int32_t scanL[kRmBlock], scanR[kRmBlock];
  int32_t wred[kRmThreads / kWave], wred2[kRmThreads / kWave];
  int64_t wred64[kRmThreads / kWave], wred64b[kRmThreads / kWave];
  double dred[kRmThreads / kWave];
  double dred4[4][kRmThreads / kWave];
  uint32_t hist[kRmBins];
  int32_t pool_n, n_core, n_fr, qa, qb;
  double res;
};
static_assert(kRmStageMax <= 32767 && kRmPool <= 32767, "16-bit indices of the running median");
static_assert(kRmThreads >= kRmBlock && kRmBins % kRmThreads == 0 && kRmPool % kRmThreads == 0,
              "threads of the running median");

// Block-wide reductions (every thread returns the result).
__device__ __forceinline__ int64_t rm_sum(RmShared& sh, int64_t v) {
  v = wave_sum(v);
  if (lane_id() == 0) sh.wred64[wave_id()] = v;
  __syncthreads();
  int64_t t = 0;
  for (int w = 0; w < kRmThreads / kWave; ++w) t += sh.wred64[w];
  __syncthreads();
  return t;
}
__device__ __forceinline__ void rm_sum2(RmShared& sh, int64_t& a, int64_t& b) {
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane_id() == 0) {
    sh.wred64[wave_id()] = a;
    sh.wred64b[wave_id()] = b;
  }
  __syncthreads();
  int64_t ta = 0, tb = 0;
  for (int w = 0; w < kRmThreads / kWave; ++w) {
    ta += sh.wred64[w];
    tb += sh.wred64b[w];
  }
  __syncthreads();
  a = ta;
  b = tb;
}
__device__ __forceinline__ double rm_min(RmShared& sh, double v) {
  v = -wave_dmax(-v);
  if (lane_id() == 0) sh.dred[wave_id()] = v;
  __syncthreads();
  double t = sh.dred[0];
  for (int w = 1; w < kRmThreads / kWave; ++w) t = fmin(t, sh.dred[w]);
  __syncthreads();
  return t;
}
__device__ __forceinline__ double rm_max(RmShared& sh, double v) {
  v = wave_dmax(v);
  if (lane_id() == 0) sh.dred[wave_id()] = v;
  __syncthreads();
  double t = sh.dred[0];
  for (int w = 1; w < kRmThreads / kWave; ++w) t = fmax(t, sh.dred[w]);
  __syncthreads();
  return t;
}
// Two minima (a, c) and two maxima (b, d) in one exchange.
__device__ __forceinline__ void rm_ext4(RmShared& sh, double& a, double& b, double& c, double& d) {
  a = -wave_dmax(-a);
  b = wave_dmax(b);
  c = -wave_dmax(-c);
  d = wave_dmax(d);
  if (lane_id() == 0) {
    const int w = wave_id();
    sh.dred4[0][w] = a;
    sh.dred4[1][w] = b;
    sh.dred4[2][w] = c;
    sh.dred4[3][w] = d;
  }
  __syncthreads();
  a = sh.dred4[0][0];
  b = sh.dred4[1][0];
  c = sh.dred4[2][0];
  d = sh.dred4[3][0];
  for (int w = 1; w < kRmThreads / kWave; ++w) {
    a = fmin(a, sh.dred4[0][w]);
    b = fmax(b, sh.dred4[1][w]);
    c = fmin(c, sh.dred4[2][w]);
    d = fmax(d, sh.dred4[3][w]);
  }
  __syncthreads();
}

// The rank-r (0-based) value of the `cnt` values get(0 .. cnt-1), exact.  A
// value bracket [a, b] with count(< a) = ca <= r < count(<= b) = cb is halved
// until at most kRmBlock values lie in it (or no double lies strictly inside
// it); those are then ranked directly.  Every thread returns the result.
template <typename Get>
__device__ double rm_kth(RmShared& sh, Get get, int64_t cnt, int64_t r) {
  const int tid = threadIdx.x;
  double mn = INFINITY, mx = -INFINITY;
  for (int64_t j = tid; j < cnt; j += kRmThreads) {
    const double v = get(j);
    mn = fmin(mn, v);
    mx = fmax(mx, v);
  }
  double a = rm_min(sh, mn), b = rm_max(sh, mx);
  int64_t ca = 0, cb = cnt;
  for (int it = 0; it < 2200; ++it) {
    if (a == b) return a;
    const double mid = a + 0.5 * (b - a);
    if (cb - ca <= kRmBlock || !(mid > a && mid < b)) {
      // gather the values in [a, b] and rank them
      if (tid == 0) sh.pool_n = 0;
      __syncthreads();
      for (int64_t j = tid; j < cnt; j += kRmThreads) {
        const double v = get(j);
        if (v >= a && v <= b) {
          const int at = atomicAdd(&sh.pool_n, 1);
          if (at < kRmBlock) sh.cand[at] = v;
        }
      }
      __syncthreads();
      const int m = sh.pool_n;
      if (m <= kRmBlock) {
        const int64_t want = r - ca;  // rank inside the bracket
        if (tid < m) {
          const double v = sh.cand[tid];
          int less = 0, eq = 0;
          for (int q = 0; q < m; ++q) {
            less += sh.cand[q] < v;
            eq += sh.cand[q] == v;
          }
          if (less <= want && want < less + eq) sh.res = v;  // equal values write the same
        }
        __syncthreads();
        const double res = sh.res;
        __syncthreads();
        return res;
      }
      // more than kRmBlock values, no double strictly between a and b: the
      // bracket holds only the values a and b
      __syncthreads();
      int64_t le = 0;
      for (int64_t j = tid; j < cnt; j += kRmThreads) le += get(j) <= a;
      le = rm_sum(sh, le);
      return le > r ? a : b;
    }
    int64_t c = 0;  // count(<= mid)
    for (int64_t j = tid; j < cnt; j += kRmThreads) c += get(j) <= mid;
    c = rm_sum(sh, c);
    if (c > r) {
      b = mid;
      cb = c;
    } else {
      a = nextafter(mid, INFINITY);
      ca = c;
    }
  }
  return a;  // not reached: each round narrows the bracket to a finite set of doubles
}

// One block of outputs: med[i] for i in [blockIdx.x * kRmBlock, ...).
// use_stage: the launch gave the workgroup LDS for kRmStageMax values.
// Block `blk` of the running median of x[0..n): its outputs' medians go to
// sink(i, median).
template <typename T, typename Sink>
__device__ __forceinline__ void rm_block(const T* __restrict__ x, int64_t n, int32_t window, int use_stage,
                                         int64_t blk, unsigned char* rm_lds, Sink sink) {
  RmShared& sh = *reinterpret_cast<RmShared*>(rm_lds);
  double* stage = reinterpret_cast<double*>(rm_lds + ((sizeof(RmShared) + 15) & ~(size_t)15));
  const int tid = threadIdx.x;
  const int64_t i0 = blk * kRmBlock;
  const int64_t i1 = i0 + kRmBlock < n ? i0 + kRmBlock : n;
  const int64_t h = window / 2;
  auto wlo = [&](int64_t i) { const int64_t v = i - h; return v < 0 ? (int64_t)0 : v; };
  auto whi = [&](int64_t i) { const int64_t v = i - h + window; return v > n ? n : v; };
  const int64_t Ulo = wlo(i0), Uhi = whi(i1 - 1);  // the union of the block's windows
  const int64_t Clo = wlo(i1 - 1), Chi = whi(i0);  // their common core
  const int64_t nU = Uhi - Ulo;
  const bool staged = use_stage && nU <= kRmStageMax;
  double cmn = INFINITY, cmx = -INFINITY;  // the core's extremes, taken while staging
  if (staged) {
    const int64_t cb = Clo - Ulo, ce = Chi - Ulo;
    for (int64_t j = tid; j < nU; j += kRmThreads) {
      const double v = (double)x[Ulo + j];
      stage[j] = v;
      if (j >= cb && j < ce) {
        cmn = fmin(cmn, v);
        cmx = fmax(cmx, v);
      }
    }
  }
  __syncthreads();
  auto val = [&](int64_t pos) -> double { return staged ? stage[pos - Ulo] : (double)x[pos]; };
  const int64_t i = i0 + tid;
  const bool live = tid < kRmBlock && i < i1;
  const int64_t lo_i = live ? wlo(i) : 0, hi_i = live ? whi(i) : 1;
  const int64_t cnt_i = hi_i - lo_i;
  const int64_t k1 = (cnt_i - 1) / 2, k2 = cnt_i / 2;
  const int64_t nC = Chi - Clo;
  bool direct = !staged || nC < 1;
  int64_t below = 0;
  if (!direct) {
    // ranks of the core that bound every median of the block: the rank-k
    // value of window i lies between the core's values of rank k - f_i and
    // k (f_i fringe samples), so the buckets from the one holding rank ra to
    // the one holding rank rb below hold every median; with a rank k - f_i
    // below 0 (a core under half the window) there is no lower bound, and
    // with k past the core none above
    const int64_t f_i = cnt_i - nC;
    double ra_d = live ? (double)(k1 - f_i) : INFINITY;
    double rb_d = live ? (double)k2 : -INFINITY;
    double mn = cmn, mx = cmx;
    rm_ext4(sh, ra_d, rb_d, mn, mx);
    // Buckets: kRmBins equal ones between the core's minimum and maximum,
    // -1 below the minimum, the top one at and above the maximum.  The
    // bucket is monotone in the value, so equal values share a bucket and
    // every bucket lies above the ones below it; the buckets qa..qb holding
    // ranks ra and rb then contain every value between those two ranks.
    const double* core = stage + (Clo - Ulo);
    const bool skip1 = !(ra_d >= 0.0), skip2 = !(rb_d < (double)nC);
    const int64_t ra = skip1 ? 0 : (int64_t)ra_d, rb = skip2 ? 0 : (int64_t)rb_d;
    const bool spread = mx > mn;
    const double scale = spread ? (double)kRmBins / (mx - mn) : 0.0;
    auto bucket = [&](double v) -> int {
      if (v < mn) return -1;
      if (!spread) return v > mn ? 1 : 0;  // one value in the core: its own bucket
      const double t = (v - mn) * scale;
      return t < (double)(kRmBins - 1) ? (int)t : kRmBins - 1;
    };
    int qa = 0, qb = 0;
    if (spread) {
      for (int q = tid; q < kRmBins; q += kRmThreads) sh.hist[q] = 0u;
      __syncthreads();
      for (int64_t j = tid; j < nC; j += kRmThreads) atomicAdd(&sh.hist[bucket(core[j])], 1u);
      __syncthreads();
      // exclusive prefix counts of the buckets, kRmBins / kRmThreads per thread
      constexpr int kPerB = kRmBins / kRmThreads;
      uint32_t hv[kPerB], own = 0;
#pragma unroll
      for (int q = 0; q < kPerB; ++q) {
        hv[q] = sh.hist[tid * kPerB + q];
        own += hv[q];
      }
      const uint32_t inc = wave_scan(own);
      if (lane_id() == kWave - 1) sh.wred[wave_id()] = (int32_t)inc;
      __syncthreads();
      int64_t run = (int64_t)inc - own;
      for (int w = 0; w < wave_id(); ++w) run += sh.wred[w];
      if (tid == 0) {
        sh.qa = 0;
        sh.qb = kRmBins - 1;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kPerB; ++q) {
        if (!skip1 && run <= ra && ra < run + (int64_t)hv[q]) sh.qa = tid * kPerB + q;
        if (!skip2 && run <= rb && rb < run + (int64_t)hv[q]) sh.qb = tid * kPerB + q;
        run += hv[q];
      }
      __syncthreads();
      qa = sh.qa;
      qb = sh.qb;
    }
    // below the pool: a bucket under qa (never, without a lower bound)
    auto under = [&](double v) { return !skip1 && bucket(v) < qa; };
    // the pool: the union's values in buckets qa..qb; and the core's values below them
    if (tid == 0) sh.pool_n = 0;
    __syncthreads();
    int64_t core_below = 0;
    for (int64_t j = tid; j < nU; j += kRmThreads) {
      const double v = stage[j];
      const int64_t pos = Ulo + j;
      const int q = bucket(v);
      const bool lo_ok = skip1 || q >= qa;
      if (lo_ok && (skip2 || q <= qb)) {
        const int at = atomicAdd(&sh.pool_n, 1);
        if (at < kRmPool) {
          sh.pool_v[at] = v;
          sh.pool_p[at] = (int16_t)j;
        }
      }
      if (pos >= Clo && pos < Chi) core_below += !lo_ok;
    }
    core_below = rm_sum(sh, core_below);
    // values below the pool in the left fringe [Ulo, Clo) and the right one
    // [Chi, Uhi), each at most kRmBlock - 1 samples: exclusive prefix counts
    const int64_t nL = Clo - Ulo, nR = Uhi - Chi;
    const uint32_t bl = tid < nL ? (under(stage[tid]) ? 1u : 0u) : 0u;
    const uint32_t br = tid < nR ? (under(stage[Chi - Ulo + tid]) ? 1u : 0u) : 0u;
    const uint32_t sl = wave_scan(bl), sr = wave_scan(br);
    if (lane_id() == kWave - 1) {
      sh.wred[wave_id()] = (int32_t)sl;
      sh.wred2[wave_id()] = (int32_t)sr;
    }
    __syncthreads();
    int32_t baseL = 0, baseR = 0;
    for (int w = 0; w < wave_id(); ++w) {
      baseL += sh.wred[w];
      baseR += sh.wred2[w];
    }
    int32_t totalL = 0;
    for (int w = 0; w < kRmThreads / kWave; ++w) totalL += sh.wred[w];
    __syncthreads();
    if (tid < kRmBlock) {
      sh.scanL[tid] = baseL + (int32_t)sl - (int32_t)bl;  // exclusive prefix
      sh.scanR[tid] = baseR + (int32_t)sr - (int32_t)br;
    }
    __syncthreads();
    const int pn = sh.pool_n;
    if (pn > kRmPool) {
      direct = true;
    } else {
      if (live) {
        const int64_t left = lo_i < Clo ? (int64_t)(totalL - sh.scanL[lo_i - Ulo]) : 0;
        const int64_t right = hi_i > Chi ? (int64_t)sh.scanR[hi_i - Chi] : 0;
        below = core_below + left + right;
      }
      // bitonic sort of the pool by (value, position), padded to a power of two
      int np2 = 1;
      while (np2 < pn) np2 <<= 1;
      for (int j = pn + tid; j < np2; j += kRmThreads) {
        sh.pool_v[j] = INFINITY;
        sh.pool_p[j] = 0x7fff;
      }
      __syncthreads();
      // One thread per compare pair: pair p compares entries t and t + jj,
      // t being p with a zero bit inserted at jj.  For distances up to 64 the
      // 64 pairs of a wave are the entries [128w, 128w + 128), the same at
      // every such distance, so those compares need no workgroup barrier
      // before or after.
      static_assert(kRmPool <= 2 * kRmThreads, "one compare pair per thread");
      for (int k = 2; k <= np2; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
          const int p = tid;
          if (p < (np2 >> 1)) {
            const int t = ((p & ~(jj - 1)) << 1) | (p & (jj - 1));
            const int u = t + jj;
            const bool up = (t & k) == 0;
            const double va = sh.pool_v[t], vb = sh.pool_v[u];
            const int16_t pa = sh.pool_p[t], pb = sh.pool_p[u];
            const bool gt = va > vb || (va == vb && pa > pb);
            if (gt == up) {
              sh.pool_v[t] = vb;
              sh.pool_v[u] = va;
              sh.pool_p[t] = pb;
              sh.pool_p[u] = pa;
            }
          }
          const int jn = jj > 1 ? jj >> 1 : (k < np2 ? k : 0);  // the next compare distance (0: sorted)
          if (jj >= kWave || jn >= kWave || jn == 0) __syncthreads();
          else wave_lds_sync();
        }
      }
      // split the sorted pool into its core entries (in every window of the
      // block) and its fringe entries, each list in value order
      {
        constexpr int kPer = kRmPool / kRmThreads;  // entries per thread
        const int cbeg = (int)(Clo - Ulo), cend = (int)(Chi - Ulo);
        int ncore = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
          const int t = tid * kPer + q;
          ncore += (t < pn && sh.pool_p[t] >= cbeg && sh.pool_p[t] < cend) ? 1 : 0;
        }
        const uint32_t inc = wave_scan((uint32_t)ncore);
        if (lane_id() == kWave - 1) sh.wred[wave_id()] = (int32_t)inc;
        __syncthreads();
        int cbase = 0;
        for (int w = 0; w < wave_id(); ++w) cbase += sh.wred[w];
        int ctot = 0;
        for (int w = 0; w < kRmThreads / kWave; ++w) ctot += sh.wred[w];
        int c = cbase + (int)inc - ncore;          // core entries before this thread's
        int f = tid * kPer - c;                    // fringe entries before them
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
          const int t = tid * kPer + q;
          if (t < pn) {
            const int16_t pp = sh.pool_p[t];
            if (pp >= cbeg && pp < cend) {
              sh.core_at[c++] = (int16_t)t;
            } else {
              sh.fr_at[f] = (int16_t)t;
              sh.fr_p[f++] = pp;
            }
          }
        }
        if (tid == 0) {
          sh.n_core = ctot;
          sh.n_fr = pn - ctot;
        }
        __syncthreads();
      }
      // each output: the in-window entries in value order are the core
      // entries with this output's in-window fringe entries merged in; walk
      // the fringe list and take the targets' ranks
      if (live) {
        const int64_t t1 = k1 - below, t2 = k2 - below;
        const int32_t plo = (int32_t)(lo_i - Ulo), phi = (int32_t)(hi_i - Ulo);
        const int nf = sh.n_fr, ncr = sh.n_core;
        auto core_val = [&](int64_t r) {  // the r-th core entry (clamped: r is in range)
          r = r < 0 ? 0 : (r >= ncr ? ncr - 1 : r);
          return sh.pool_v[sh.core_at[r]];
        };
        double m1 = 0.0, m2 = 0.0;
        bool got1 = false, got2 = false;
        int64_t jin = 0;  // in-window fringe entries so far
        for (int j = 0; j < nf && !got2; ++j) {
          const int32_t pp = sh.fr_p[j];
          if (pp < plo || pp >= phi) continue;
          const int64_t before = (int64_t)(sh.fr_at[j] - j) + jin;  // in-window entries before it
          if (!got1) {
            if (t1 < before) {
              m1 = core_val(t1 - jin);
              got1 = true;
            } else if (t1 == before) {
              m1 = sh.pool_v[sh.fr_at[j]];
              got1 = true;
            }
          }
          if (t2 < before) {
            m2 = core_val(t2 - jin);
            got2 = true;
          } else if (t2 == before) {
            m2 = sh.pool_v[sh.fr_at[j]];
            got2 = true;
          }
          ++jin;
        }
        if (!got1) m1 = core_val(t1 - jin);
        if (!got2) m2 = core_val(t2 - jin);
        sink(i, (cnt_i % 2) ? m1 : 0.5 * (m1 + m2));
      }
    }
  }
  if (direct) {
    // every output of the block selected on its own, cooperatively
    for (int64_t u = i0; u < i1; ++u) {
      const int64_t lo = wlo(u), hi = whi(u), c = hi - lo;
      auto win = [&](int64_t j) { return val(lo + j); };
      const double m1 = rm_kth(sh, win, c, (c - 1) / 2);
      const double m = (c % 2) ? m1 : 0.5 * (m1 + rm_kth(sh, win, c, c / 2));
      if (tid == 0) sink(u, m);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kRmThreads, 8) void running_median_kernel(const T* __restrict__ x, int64_t n,
                                                                  int32_t window, int use_stage,
                                                                  double* __restrict__ med) {
  extern __shared__ __align__(16) unsigned char rm_lds[];
  rm_block(x, n, window, use_stage, (int64_t)blockIdx.x, rm_lds, [&](int64_t i, double m) { med[i] = m; });
}

// The exact dereddening of many series in one launch: block b runs block
// b - block0 of its segment's running median (the segment from a per-block
// map) and writes x[i] - median, in double, rounded once to float32.  Input
// (double) and output (float32) never overlap.
__global__ __launch_bounds__(kRmThreads, 8) void dered_batch_kernel(const DeredSeg* __restrict__ segs,
                                                               const int32_t* __restrict__ block_seg,
                                                               int64_t block_base, float* __restrict__ ws) {
  extern __shared__ __align__(16) unsigned char rm_lds[];
  const int64_t b = block_base + blockIdx.x;
  const DeredSeg sg = segs[block_seg[b]];
  const double* x = reinterpret_cast<const double*>(ws + sg.x_off);
  float* out = ws + sg.out_off;
  rm_block(x, sg.n, sg.window, sg.use_stage, b - sg.block0, rm_lds,
           [&](int64_t i, double m) { out[i] = (float)(x[i] - m); });
}

// out[i] = x[i] - med[i], in double, rounded once to float32 (`out` may alias
// `x` for a 4-byte type: each thread reads its element first).
template <typename T>
__global__ void median_subtract_kernel(const T* x, int64_t n, const double* __restrict__ med, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = (float)((double)x[i] - med[i]);
}

// out[i] = x[i] - baseline(i), in double, rounded once to float32.  `out` may
// alias `x` when both are 4-byte types (each thread reads its element first).
template <typename T>
__global__ void dered_subtract_kernel(const T* x, int64_t n, int32_t stride, int64_t nk,
                                      const double* __restrict__ med, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c = i / stride;
  double b = med[c];
  if (c + 1 < nk) b += (med[c + 1] - med[c]) * (double)(i - c * stride) / (double)stride;
  const double v = (double)x[i] - b;
  out[i] = (float)v;
}

// float input for a dereddened search: double copy, so the octave sums keep
// the precision the baseline subtraction needs
__global__ void prep_f64_kernel(const float* __restrict__ in, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

// One halving of the time resolution (paper Sec. 2.3.1): y[i] = x[2i]+x[2i+1].
template <typename T>
__global__ void halve_kernel(const T* __restrict__ in, int64_t n_out,
                             T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_out) out[i] = in[2 * i] + in[2 * i + 1];
}

// Best trial: the largest score, the first index on ties, NaN never wins.
// Each score and index pack into one 64-bit key, larger for a better trial:
// the score's order-preserving key above (2^32 - 1 - index), so one atomic
// maximum per wave finds it.  The key accumulates in the output word itself.
__device__ __forceinline__ uint64_t best_key(float v, int64_t i) {
  const uint32_t k = v != v ? 0u : fkey(v + 0.0f);  // NaN lowest; -0 counts as +0
  return ((uint64_t)k << 32) | (uint64_t)(0xffffffffu - (uint32_t)i);
}

__global__ void best_init_kernel(unsigned long long* __restrict__ acc) { *acc = 0ull; }

// Output table of a batch, carried in the kernel arguments.
constexpr int kOutsPerLaunch = 128;
struct OutsChunk {
  SeriesOut e[kOutsPerLaunch];
};

__global__ void set_outs_kernel(OutsChunk c, int32_t n, SeriesOut* __restrict__ dst) {
  const int i = (int)threadIdx.x;
  if (i < n) dst[i] = c.e[i];
}

__global__ __launch_bounds__(256) void best_max_kernel(const float* __restrict__ s, int64_t n,
                                                       unsigned long long* __restrict__ acc) {
  uint64_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = best_key(s[i], i);
    m = k > m ? k : m;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const uint64_t other = __shfl_xor(m, o, kWave);
    m = other > m ? other : m;
  }
  if (lane_id() == 0 && m != 0) atomicMax(acc, (unsigned long long)m);
}

__global__ void best_final_kernel(int64_t* __restrict__ best) {
  const uint64_t k = (uint64_t)*best;
  *best = (int64_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
}

// ------------------------------------------------------ candidate sifting
//
// After the paper's ffa2best (Sec. 2.3.3), with the rules stated in ffa.h:
// the trials at or above min_snr are compacted in order (count, scan, write),
// one workgroup scans them for peaks, then one workgroup ranks the peaks and
// applies grouping and harmonic matching.  Periods and limits are computed in
// double with the operations in a fixed order (no contraction), so the
// decisions do not depend on the compiler.

__global__ __launch_bounds__(kSiftBlock) void sift_count_kernel(const float* __restrict__ snr, int64_t n,
                                                                float min_snr, int32_t* __restrict__ counts) {
  const int64_t t = (int64_t)blockIdx.x * kSiftBlock + threadIdx.x;
  const bool keep = t < n && snr[t] >= min_snr;
  const int c = __syncthreads_count(keep);
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// exclusive prefix of counts[0..nb) into offs[0..nb], offs[nb] = total
__global__ __launch_bounds__(1024) void sift_scan_kernel(const int32_t* __restrict__ counts, int64_t nb,
                                                         int32_t* __restrict__ offs) {
  __shared__ int32_t buf[1024];
  int32_t carry = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int32_t v = i < nb ? counts[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int32_t a = threadIdx.x >= (unsigned)o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nb) offs[i] = carry + buf[threadIdx.x] - v;
    carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) offs[nb] = carry;
}

__global__ __launch_bounds__(kSiftBlock) void sift_write_kernel(const float* __restrict__ snr, int64_t n,
                                                                float min_snr, const int32_t* __restrict__ offs,
                                                                int32_t* __restrict__ ctrial,
                                                                float* __restrict__ csnr) {
  __shared__ int32_t wsum[kSiftBlock / kWave];
  const int64_t t = (int64_t)blockIdx.x * kSiftBlock + threadIdx.x;
  const float v = t < n ? snr[t] : 0.0f;
  const bool keep = t < n && v >= min_snr;
  const uint64_t m = __ballot(keep);
  const int w = threadIdx.x / kWave;
  const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  if (lane_id() == 0) wsum[w] = __popcll(m);
  __syncthreads();
  int before = offs[blockIdx.x];
  for (int i = 0; i < w; ++i) before += wsum[i];
  if (keep) {
    ctrial[before + rank] = (int32_t)t;
    csnr[before + rank] = v;
  }
}

// Peaks of the compacted list (one workgroup; thread 0 scans chunks staged in
// LDS).  info[0] = peaks found (more than kSiftMaxPeaks: -1).
__global__ __launch_bounds__(1024) void sift_peaks_kernel(const int32_t* __restrict__ ctrial,
                                                          const float* __restrict__ csnr,
                                                          const int32_t* __restrict__ total_p, float frac_fall,
                                                          float abs_fall, int32_t* __restrict__ ptrial,
                                                          float* __restrict__ psnr, int32_t* __restrict__ info) {
#pragma clang fp contract(off)
  constexpr int kChunk = 4096;
  __shared__ int32_t st[kChunk];
  __shared__ float ss[kChunk];
  const int32_t total = *total_p;
  int32_t np = 0, prev = -2;
  bool open = false, over = false;
  int32_t cur_t = 0;
  float cur_s = 0.0f;
  for (int32_t base = 0; base < total; base += kChunk) {
    const int32_t cnt = total - base < kChunk ? total - base : kChunk;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
      st[i] = ctrial[base + i];
      ss[i] = csnr[base + i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = 0; i < cnt; ++i) {
        const int32_t t = st[i];
        const float s = ss[i];
        if (t != prev + 1) {  // a trial below min_snr lies in between: close
          if (open) {
            if (np < kSiftMaxPeaks) {
              ptrial[np] = cur_t;
              psnr[np] = cur_s;
            }
            ++np;
          }
          open = false;
        }
        prev = t;
        if (!open) {
          open = true;
          cur_t = t;
          cur_s = s;
        } else if (s > cur_s) {
          cur_t = t;
          cur_s = s;
        } else {
          const float fall = cur_s - s;
          if (fall >= frac_fall * cur_s && fall >= abs_fall) {
            if (np < kSiftMaxPeaks) {
              ptrial[np] = cur_t;
              psnr[np] = cur_s;
            }
            ++np;
            open = false;
          }
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (open) {
      if (np < kSiftMaxPeaks) {
        ptrial[np] = cur_t;
        psnr[np] = cur_s;
      }
      ++np;
    }
    over = np > kSiftMaxPeaks;
    info[0] = over ? -1 : np;
  }
}

__device__ __forceinline__ bool is_prime(int32_t x) {
  if (x < 2) return false;
  for (int32_t q = 2; q * q <= x; ++q)
    if (x % q == 0) return false;
  return true;
}

// Rank, group, match harmonics, write the survivors (one workgroup).
__global__ __launch_bounds__(1024) void sift_final_kernel(
    const int32_t* __restrict__ ptrial, const float* __restrict__ psnr, const int32_t* __restrict__ info,
    const int32_t* __restrict__ width, const StepDev* __restrict__ steps, int32_t n_steps, double tsamp,
    float group_widths, int32_t harmonic_primes, float harmonic_tol, double* __restrict__ period,
    double* __restrict__ lim, int32_t* __restrict__ order, int32_t* __restrict__ alive,
    ffa_candidate* __restrict__ out, int32_t max_out, int32_t* __restrict__ n_out) {
#pragma clang fp contract(off)
  const int32_t np = info[0];
  if (np < 0) {
    if (threadIdx.x == 0) *n_out = -1;
    return;
  }
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const int64_t t = ptrial[i];
    int lo = 0, hi = n_steps - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (steps[mid].first_trial <= t) lo = mid;
      else hi = mid - 1;
    }
    const StepDev s = steps[lo];
    const int64_t k = t - s.first_trial;
    const double fts = (double)s.f * tsamp;
    const double P = fts * ((double)s.P0 + (double)k / (double)(s.M - 1));
    const double span = fts * (double)s.m * (double)s.P0;
    const double wsec = fts * (double)width[t];
    period[i] = P;
    lim[i] = (double)group_widths * wsec * P / span;
    alive[i] = 1;
    // rank: stronger first, lower trial first on ties
    int32_t r = 0;
    const float si = psnr[i];
    for (int j = 0; j < np; ++j) {
      const float sj = psnr[j];
      r += (sj > si || (sj == si && ptrial[j] < ptrial[i])) ? 1 : 0;
    }
    order[r] = i;
  }
  __syncthreads();
  if (group_widths > 0.0f) {
    for (int r = 0; r < np; ++r) {
      const int i = order[r];
      if (alive[i]) {
        for (int r2 = r + 1 + threadIdx.x; r2 < np; r2 += blockDim.x) {
          const int j = order[r2];
          if (alive[j] && fabs(period[j] - period[i]) <= lim[i]) alive[j] = 0;
        }
      }
      __syncthreads();
    }
  }
  if (harmonic_primes >= 2) {
    // the primes up to the limit (168 below 1000)
    __shared__ int32_t primes[168];
    __shared__ int32_t n_primes;
    if (threadIdx.x == 0) {
      int32_t k = 0;
      for (int32_t x = 2; x <= harmonic_primes && k < 168; ++x)
        if (is_prime(x)) primes[k++] = x;
      n_primes = k;
    }
    __syncthreads();
    const double tol = (double)harmonic_tol;
    // n in [lo, hi] of 1..x-1 around a real bound pair, with one bin of margin
    // for the rounding of the bounds
    auto span = [](double a, double b, int32_t x, int32_t& lo, int32_t& hi) {
      lo = a > (double)x ? x : (int32_t)floor(fmax(a, 0.0)) - 1;
      hi = b > (double)x ? x - 1 : (int32_t)ceil(fmax(b, 0.0)) + 1;
      lo = lo < 1 ? 1 : lo;
      hi = hi > x - 1 ? x - 1 : hi;
    };
    for (int r = 0; r < np; ++r) {
      const int i = order[r];
      if (alive[i]) {
        const double Pi = period[i];
        for (int r2 = r + 1 + threadIdx.x; r2 < np; r2 += blockDim.x) {
          const int j = order[r2];
          if (!alive[j]) continue;
          const double Pj = period[j];
          const double rho = Pj / Pi;
          bool related = false;
          // P*n/x within tol of Pj needs n in [x*rho/(1+tol), x*rho/(1-tol)];
          // P*x/n needs n in [x*(1-tol)/rho, x*(1+tol)/rho].  Each n there is
          // tested with the same expression as the full scan over 0 < n < x,
          // so the decision is the same.
          for (int q = 0; q < n_primes && !related; ++q) {
            const int32_t x = primes[q];
            int32_t lo, hi;
            span((double)x * rho / (1.0 + tol), tol < 1.0 ? (double)x * rho / (1.0 - tol) : 1e300, x, lo, hi);
            for (int32_t nn = lo; nn <= hi && !related; ++nn) {
              const double r1 = Pi * (double)nn / (double)x;
              if (fabs(Pj - r1) <= tol * r1) related = true;
            }
            span((double)x * (1.0 - tol) / rho, (double)x * (1.0 + tol) / rho, x, lo, hi);
            for (int32_t nn = lo; nn <= hi && !related; ++nn) {
              const double r2v = Pi * (double)x / (double)nn;
              if (fabs(Pj - r2v) <= tol * r2v) related = true;
            }
          }
          if (related) alive[j] = 0;
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    int32_t k = 0;
    for (int r = 0; r < np; ++r) {
      const int i = order[r];
      if (!alive[i]) continue;
      if (k < max_out) {
        ffa_candidate c;
        c.trial = ptrial[i];
        c.period_s = period[i];
        c.snr = psnr[i];
        c.width = width[ptrial[i]];
        out[k] = c;
      }
      ++k;
    }
    *n_out = k;
  }
}

// ------------------------------------------------------------ S/N histogram
//
// Each workgroup counts its share of the scores in an LDS histogram (32-bit
// counters; the launcher keeps every workgroup under 2^31 scores), then adds
// its non-zero bins to the 64-bit device histogram.

__global__ __launch_bounds__(1024) void snr_hist_kernel(const float* __restrict__ snr, int64_t n, float lo,
                                                        float bpu, int32_t nb,
                                                        unsigned long long* __restrict__ hist) {
#pragma clang fp contract(off)
  extern __shared__ uint32_t h_lds[];
  for (int i = threadIdx.x; i < nb; i += 1024) h_lds[i] = 0;
  __syncthreads();
  const float top = (float)(nb - 1);
  const int64_t stride = (int64_t)gridDim.x * 1024;
  for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += stride) {
    const float s = snr[i];
    if (__builtin_isnan(s)) continue;
    const float x = (s - lo) * bpu;
    const int b = !(x >= 0.0f) ? 0 : (x >= top ? nb - 1 : (int)x);
    atomicAdd(&h_lds[b], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += 1024) {
    const uint32_t c = h_lds[i];
    if (c) atomicAdd(&hist[i], (unsigned long long)c);
  }
}

}  // namespace

// --------------------------------------------------------------- launchers

// Series header: 1024 doubles of partial sums, then the centring constant.
hipError_t launch_mean(const float* x, int64_t n, void* ws, hipStream_t st) {
  double* part = reinterpret_cast<double*>(ws);
  float* c = reinterpret_cast<float*>(part + kMeanBlocks);
  mean_partial_kernel<<<kMeanBlocks, kMeanThreads, 0, st>>>(x, n, part);
  mean_final_kernel<<<1, kMeanBlocks, 0, st>>>(part, n, c);
  return hipGetLastError();
}

hipError_t launch_prep(const void* series, int is_int, int64_t n, void* ws, int64_t out_off,
                       int center, hipStream_t st) {
  const int tpb = 256;
  const int64_t blocks = (n + tpb - 1) / tpb;
  if (is_int) {
    int32_t* out = reinterpret_cast<int32_t*>(ws) + out_off;
    prep_u8_kernel<<<blocks, tpb, 0, st>>>(reinterpret_cast<const uint8_t*>(series), n, out);
  } else {
    const float* c = reinterpret_cast<const float*>(reinterpret_cast<const double*>(ws) + kMeanBlocks);
    float* out = reinterpret_cast<float*>(ws) + out_off;
    prep_f32_kernel<<<blocks, tpb, 0, st>>>(reinterpret_cast<const float*>(series), n, c, center,
                                            out);
  }
  return hipGetLastError();
}

hipError_t launch_prep_f64(const float* series, int64_t n, void* ws, int64_t out_off, hipStream_t st) {
  const int tpb = 256;
  prep_f64_kernel<<<(unsigned)((n + tpb - 1) / tpb), tpb, 0, st>>>(
      series, n, reinterpret_cast<double*>(reinterpret_cast<float*>(ws) + out_off));
  return hipGetLastError();
}

hipError_t launch_deredden(void* ws, int src_type, int64_t src_off, int64_t n, int32_t window, int32_t stride,
                           int64_t knots_off, int64_t out_off, hipStream_t st) {
  if (n < 1) return hipSuccess;
  if (window < 1 || stride < 1) return hipErrorInvalidValue;
  float* w = reinterpret_cast<float*>(ws);
  double* med = reinterpret_cast<double*>(w + knots_off);
  float* out = w + out_off;
  const int64_t nk = (n - 1) / stride + 1;
  if (nk > 0x7fffffff) return hipErrorInvalidValue;
  const int tpb = 256;
  const unsigned gs = (unsigned)((n + tpb - 1) / tpb);
  // exact running median (stride 1): blocks of kRmBlock outputs, the union
  // of their windows staged in LDS when it fits
  const int64_t nb = (n + kRmBlock - 1) / kRmBlock;
  const int64_t stage_n = std::min<int64_t>((int64_t)window + kRmBlock - 1, n);
  const int use_stage = stage_n <= kRmStageMax ? 1 : 0;
  const size_t rm_lds = ((sizeof(RmShared) + 15) & ~(size_t)15) + (use_stage ? (size_t)stage_n * sizeof(double) : 0);
  if (stride == 1 && nb > 0x7fffffff) return hipErrorInvalidValue;
#define FFA_DERED(TT)                                                                              \
  do {                                                                                             \
    const TT* x = reinterpret_cast<const TT*>(w + src_off);                                        \
    if (stride == 1) {                                                                             \
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&running_median_kernel<TT>),         \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);       \
      running_median_kernel<TT><<<(unsigned)nb, kRmThreads, rm_lds, st>>>(x, n, window, use_stage, med); \
      median_subtract_kernel<TT><<<gs, tpb, 0, st>>>(x, n, med, out);                              \
    } else {                                                                                       \
      knot_median_kernel<TT><<<(unsigned)nk, kKnotThreads, 0, st>>>(x, n, window, stride, med);    \
      dered_subtract_kernel<TT><<<gs, tpb, 0, st>>>(x, n, stride, nk, med, out);                   \
    }                                                                                              \
  } while (0)
  if (src_type == 0) FFA_DERED(int32_t);
  else if (src_type == 1) FFA_DERED(float);
  else FFA_DERED(double);
#undef FFA_DERED
  return hipGetLastError();
}

size_t dered_block_lds(int64_t n, int32_t window, int32_t* use_stage) {
  const int64_t stage_n = std::min<int64_t>((int64_t)window + kRmBlock - 1, n);
  *use_stage = stage_n <= kRmStageMax ? 1 : 0;
  return ((sizeof(RmShared) + 15) & ~(size_t)15) + (*use_stage ? (size_t)stage_n * sizeof(double) : 0);
}

int64_t dered_block_count(int64_t n) { return (n + kRmBlock - 1) / kRmBlock; }

hipError_t prepare_dered_batch() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&dered_batch_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
}

hipError_t launch_dered_batch(const DeredSeg* segs, const int32_t* block_seg, const DeredLaunch& L, void* ws,
                              hipStream_t st) {
  if (L.blocks < 1) return hipSuccess;
  if (L.blocks > 0x7fffffff || L.lds > (int32_t)kLdsBytes) return hipErrorInvalidValue;
  dered_batch_kernel<<<(unsigned)L.blocks, kRmThreads, (size_t)L.lds, st>>>(segs, block_seg, L.block0,
                                                                          reinterpret_cast<float*>(ws));
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

hipError_t launch_halve_f64(void* ws, int64_t in_off, int64_t n_out, int64_t out_off, hipStream_t st) {
  const int tpb = 256;
  const int64_t blocks = (n_out + tpb - 1) / tpb;
  if (n_out <= 0) return hipSuccess;
  float* w = reinterpret_cast<float*>(ws);
  halve_kernel<double><<<blocks, tpb, 0, st>>>(reinterpret_cast<const double*>(w + in_off), n_out,
                                               reinterpret_cast<double*>(w + out_off));
  return hipGetLastError();
}

template <bool INT, int EMAX, int ALG>
const void* tile_fn() {
  return reinterpret_cast<const void*>(&ffa_tile_kernel<INT, EMAX, ALG>);
}

template <int ALG>
const void* pick_tile_fn_alg(int is_int, int max_P0) {
  if (is_int) {
    if (max_P0 <= 512) return tile_fn<true, 8, ALG>();
    if (max_P0 <= 1024) return tile_fn<true, 16, ALG>();
    return tile_fn<true, 32, ALG>();
  }
  if (max_P0 <= 512) return tile_fn<false, 8, ALG>();
  if (max_P0 <= 1024) return tile_fn<false, 16, ALG>();
  return tile_fn<false, 32, ALG>();
}

const void* pick_tile_fn(int is_int, int max_P0, int alg) {
  return alg == 2 ? pick_tile_fn_alg<2>(is_int, max_P0) : pick_tile_fn_alg<1>(is_int, max_P0);
}

bool tiles_fit(int is_int, int max_P0, int lds_bytes, int alg) {
  // Static LDS of the variant plus the request must fit one workgroup; the
  // answer depends on the device and the variant only, so it is cached.
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> static_lds;
  const void* fn = pick_tile_fn(is_int, max_P0, alg);
  int dev = -1, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  int fixed = -1;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = static_lds.find({dev, fn});
    if (it != static_lds.end()) {
      fixed = it->second;
    } else {
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
      (void)hipGetLastError();
      hipFuncAttributes fa{};
      if (hipFuncGetAttributes(&fa, fn) != hipSuccess) return false;
      fixed = (int)fa.sharedSizeBytes;
      static_lds[{dev, fn}] = fixed;
    }
  }
  return lds_bytes >= 0 && (size_t)lds_bytes <= kLdsBytes && fixed + lds_bytes <= max_lds;
}

hipError_t launch_tiles(const TileArgs& a, int64_t ntiles, int lds_bytes, int max_P0, int is_int,
                        void* ws, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7fffffff || max_P0 > 2 * kMaxBinsMin || (a.alg != 1 && a.alg != 2) ||
      !tiles_fit(is_int, max_P0, lds_bytes, a.alg))
    return hipErrorInvalidValue;
  TileArgs b = a;
  b.select_cand = a.select_cand < 1 ? 1 : (a.select_cand > kWave ? kWave : a.select_cand);
  const unsigned g = (unsigned)ntiles;
#define FFA_LAUNCH(I, EM, AL) ffa_tile_kernel<I, EM, AL><<<g, kThreads, (unsigned)lds_bytes, st>>>(b, ws)
#define FFA_LAUNCH_ALG(AL)                             \
  do {                                                 \
    if (is_int) {                                      \
      if (max_P0 <= 512) FFA_LAUNCH(true, 8, AL);      \
      else if (max_P0 <= 1024) FFA_LAUNCH(true, 16, AL); \
      else FFA_LAUNCH(true, 32, AL);                   \
    } else {                                           \
      if (max_P0 <= 512) FFA_LAUNCH(false, 8, AL);     \
      else if (max_P0 <= 1024) FFA_LAUNCH(false, 16, AL); \
      else FFA_LAUNCH(false, 32, AL);                  \
    }                                                  \
  } while (0)
  if (a.alg == 2) FFA_LAUNCH_ALG(2);
  else FFA_LAUNCH_ALG(1);
#undef FFA_LAUNCH_ALG
#undef FFA_LAUNCH
  return hipGetLastError();
}

hipError_t launch_sift(const float* snr, const int32_t* width, int64_t n, const ffa_sift_params& prm,
                       const StepDev* steps, int32_t n_steps, double tsamp, void* ws, int64_t scratch,
                       ffa_candidate* out, int32_t max_out, int32_t* n_out, hipStream_t st) {
  if (n < 1 || n > 0x7fffffff) return hipErrorInvalidValue;
  auto up = [](int64_t v) { return (v + 63) / 64 * 64; };
  const int64_t nb = (n + kSiftBlock - 1) / kSiftBlock;
  float* w = reinterpret_cast<float*>(ws) + scratch;
  int32_t* ctrial = reinterpret_cast<int32_t*>(w);
  float* csnr = w + n;
  int32_t* counts = reinterpret_cast<int32_t*>(w + up(2 * n));
  int32_t* offs = counts + up(nb + 1);
  int32_t* info = offs + up(nb + 1);
  int32_t* ptrial = info + 64;
  float* psnr = reinterpret_cast<float*>(ptrial + kSiftMaxPeaks);
  double* period = reinterpret_cast<double*>(psnr + kSiftMaxPeaks);  // 8-byte aligned: offsets above are even
  double* lim = period + kSiftMaxPeaks;
  int32_t* order = reinterpret_cast<int32_t*>(lim + kSiftMaxPeaks);
  int32_t* alive = order + kSiftMaxPeaks;
  sift_count_kernel<<<(unsigned)nb, kSiftBlock, 0, st>>>(snr, n, prm.min_snr, counts);
  sift_scan_kernel<<<1, 1024, 0, st>>>(counts, nb, offs);
  sift_write_kernel<<<(unsigned)nb, kSiftBlock, 0, st>>>(snr, n, prm.min_snr, offs, ctrial, csnr);
  sift_peaks_kernel<<<1, 1024, 0, st>>>(ctrial, csnr, offs + nb, prm.frac_fall, prm.abs_fall, ptrial, psnr, info);
  sift_final_kernel<<<1, 1024, 0, st>>>(ptrial, psnr, info, width, steps, n_steps, tsamp, prm.group_widths,
                                        prm.harmonic_primes, prm.harmonic_tol, period, lim, order, alive, out,
                                        max_out, n_out);
  return hipGetLastError();
}

hipError_t launch_snr_histogram(const float* snr, int64_t n, float lo, float bins_per_unit, int32_t n_bins,
                                uint64_t* hist, hipStream_t st) {
  if (n < 0 || n_bins < 1 || n_bins > kHistMaxBins) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  // about 64K scores per workgroup, at most 1024 workgroups unless a
  // workgroup would then count more than 2^31 scores
  int64_t blocks = std::min<int64_t>((n + 65535) / 65536, 1024);
  blocks = std::max<int64_t>(blocks, (n + (1ll << 31) - 1) >> 31);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  snr_hist_kernel<<<(unsigned)blocks, 1024, (size_t)n_bins * 4, st>>>(
      snr, n, lo, bins_per_unit, n_bins, reinterpret_cast<unsigned long long*>(hist));
  return hipGetLastError();
}

hipError_t launch_set_outs(SeriesOut* dst, const SeriesOut* src, int32_t n, hipStream_t st) {
  for (int32_t i0 = 0; i0 < n; i0 += kOutsPerLaunch) {
    const int32_t k = std::min<int32_t>(kOutsPerLaunch, n - i0);
    OutsChunk c{};
    for (int32_t j = 0; j < k; ++j) c.e[j] = src[i0 + j];
    set_outs_kernel<<<1, kOutsPerLaunch, 0, st>>>(c, k, dst + i0);
  }
  return hipGetLastError();
}

hipError_t launch_best(const float* snr, int64_t n, int64_t* best, hipStream_t st) {
  if (n < 1 || n > 0xffffffffll) return hipErrorInvalidValue;
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(best);
  const int tpb = 256;
  const int64_t blocks = std::min<int64_t>((n + tpb * 8 - 1) / (tpb * 8), 2048);
  best_init_kernel<<<1, 1, 0, st>>>(acc);
  best_max_kernel<<<(unsigned)blocks, tpb, 0, st>>>(snr, n, acc);
  best_final_kernel<<<1, 1, 0, st>>>(best);
  return hipGetLastError();
}

}  // namespace ffa
