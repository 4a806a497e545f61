// common.hpp -- device helpers shared by the GRNND kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grnnd {

constexpr int kWave = 64;
constexpr int kMaxR = 64;
constexpr uint64_t kTagUpdate = 0x1000;   // h(seed, 0x1000 + round, v, id): arrival order
constexpr uint64_t kTagReverse = 0x2000;  // h(seed, 0x2000 + t1, v, id): reverse sampling
constexpr uint64_t kTagInit = 0x3000;     // h(seed, 0x3000, v, j): initial draws
constexpr int kStatSlots = 256;           // spread counter atomics over this many lines
constexpr int kStatStride = 16;           // uint64 per slot (128 B)

typedef float v4f __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ hashing
// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014): the state is
// advanced by the golden gamma, then mixed by two xor-shift-multiply steps.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Counter-based hash used for every random choice of the method.
__device__ __forceinline__ uint64_t hash4(uint64_t seed, uint64_t a, uint64_t b, uint64_t c) {
  return mix64(mix64(mix64(mix64(seed) ^ a) ^ b) ^ c);
}

// Sort key of "hash order": high 32 bits of the hash, then the id.
__device__ __forceinline__ uint64_t hash_order_key(uint64_t h, int32_t id) {
  return (h & 0xFFFFFFFF00000000ull) | (uint64_t)(uint32_t)id;
}

// ----------------------------------------------------------- ordered keys
// Monotone map float -> uint32 (for non-NaN keys; -0 is folded onto +0), so
// that (key, id) order is the unsigned order of (ord(key) << 32 | id).
__device__ __forceinline__ uint32_t key_to_ord(float f) {
  uint32_t u = __float_as_uint(f + 0.0f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_to_key(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int readlane_i(int x, int l) { return __shfl(x, l); }
__device__ __forceinline__ float readlane_f(float x, int l) { return __shfl(x, l); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of one uint64 per lane across the wave.
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t x, int lane) {
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      uint64_t y = shfl_xor_u64(x, j);
      bool up = (lane & k) == 0;
      bool lower = (lane & j) == 0;
      x = (lower == up) ? (x < y ? x : y) : (x < y ? y : x);
    }
  }
  return x;
}

// --------------------------------------------------- canonical distance
// The one distance routine whose result is ever stored as a key. Lane l
// accumulates the float4 groups l, l+64, l+128, ... in order with fused
// multiply-adds, then the 64 partial sums are combined by an xor butterfly;
// every lane ends with the same bits, and the result is symmetric in (a, b)
// and independent of the memory (global or LDS) the rows live in.
template <int METRIC>
__device__ __forceinline__ float dist_canon(const float* __restrict__ a,
                                            const float* __restrict__ b, int d4, int lane) {
  float acc = 0.0f;
  for (int q = lane; q < d4; q += kWave) {
    const float4 x = *reinterpret_cast<const float4*>(a + 4 * q);
    const float4 y = *reinterpret_cast<const float4*>(b + 4 * q);
    if (METRIC == 0) {
      float t;
      t = x.x - y.x; acc = __builtin_fmaf(t, t, acc);
      t = x.y - y.y; acc = __builtin_fmaf(t, t, acc);
      t = x.z - y.z; acc = __builtin_fmaf(t, t, acc);
      t = x.w - y.w; acc = __builtin_fmaf(t, t, acc);
    } else {
      acc = __builtin_fmaf(x.x, y.x, acc);
      acc = __builtin_fmaf(x.y, y.y, acc);
      acc = __builtin_fmaf(x.z, y.z, acc);
      acc = __builtin_fmaf(x.w, y.w, acc);
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc = acc + __shfl_xor(acc, m);
  return METRIC == 0 ? acc : -acc;
}

// ---------------------------------------------------------- LDS layout
// Per-wave LDS of the candidate round: Kp = 16 * nb padded candidate rows plus
// one row for x_v, row stride rs floats (d rounded up to 16, plus 4 so that
// the 16 rows an MFMA operand read touches fall in distinct bank groups); the
// distance tile (Kp x (Kp+1) floats, odd stride); diagonal norms; metadata.
struct RoundLds {
  int rs;         // row stride (floats)
  int ts;         // tile stride (floats)
  int rows_off;   // float offsets
  int tile_off;
  int g_off;
  int meta_off;   // 3 x 64 words: ids, keys, key-rank
  int sk_off;     // 64 x uint64 sort keys (8-byte aligned)
  int total;      // floats
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

__host__ __device__ inline RoundLds round_lds(int kp, int d) {
  RoundLds L;
  L.rs = round_up(d, 16) + 4;
  L.ts = kp + 1;
  L.rows_off = 0;
  L.tile_off = L.rows_off + (kp + 1) * L.rs;
  L.g_off = L.tile_off + kp * L.ts;
  L.meta_off = L.g_off + kp;
  L.sk_off = round_up(L.meta_off + 3 * kWave, 2);
  L.total = L.sk_off + 2 * kWave;
  return L;
}

}  // namespace grnnd
