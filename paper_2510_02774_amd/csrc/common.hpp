// common.hpp -- device helpers shared by the GRNND kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace grnnd {

constexpr int kWave = 64;
constexpr int kMaxR = 64;  // largest pool width (one candidate per lane)
constexpr int kOrderPivots = 256;  // cells of the vertex locality order
constexpr uint64_t kTagUpdate = 0x1000;   // h(seed, 0x1000 + round, v, id): arrival order
constexpr uint64_t kTagReverse = 0x2000;  // h(seed, 0x2000 + t1, v, id): reverse sampling
constexpr uint64_t kTagInit = 0x3000;     // h(seed, 0x3000, v, j): initial draws
constexpr int kCursorWords = 16;          // device counters of a build (see MergeArgs)
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

// Item-row header of a vertex (nitem): the items it keeps for itself sit in
// slots [0, own) of its item row, the items it sends to other vertices in
// slots [own, total).
__device__ __forceinline__ int32_t items_hdr(int own, int total) { return own | (total << 16); }
__device__ __forceinline__ int items_own(int32_t h) { return h & 0xFFFF; }
__device__ __forceinline__ int items_total(int32_t h) { return (int)((uint32_t)h >> 16); }

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
// The one distance routine whose result is ever stored or compared as a key.
// A wave computes four pairs at once, one per 16-lane group: lane s of a
// group accumulates the float4 groups s, s+16, s+32, ... of its pair in order
// with fused multiply-adds (components x, y, z, w in order), then the 16
// partial sums are combined by an xor butterfly over 8, 4, 2, 1. Every lane of
// the group ends with the same bits, the result is symmetric in (a, b), and
// it does not depend on where the rows live (global memory or LDS) or on
// which group computes it.
template <int METRIC>
__device__ __forceinline__ float pair_acc(const float4 x, const float4 y, float acc) {
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
  return acc;
}

// Row in global memory (contiguous float4 groups).
struct GlobalRow {
  const float* p;
  __device__ __forceinline__ float4 operator()(int q) const {
    return *reinterpret_cast<const float4*>(p + 4 * q);
  }
};

// DPP lane exchange within rows of 16 lanes (the control must be a constant).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over a 16-lane row with the pairing of an xor butterfly 1, 2, 4, 8.
// Steps 1 and 2 exchange lanes xor 1 and xor 2 (quad permutations); after
// them each quad is uniform, so the half-row mirror (lane i <-> 7 - i)
// pairs quads exactly as xor 4 would, and the row mirror (i <-> 15 - i)
// pairs half rows as xor 8 would. Every lane ends with the same bits.
__device__ __forceinline__ float row16_sum(float acc) {
  acc = acc + dpp_f<0xB1>(acc);   // quad_perm [1,0,3,2]
  acc = acc + dpp_f<0x4E>(acc);   // quad_perm [2,3,0,1]
  acc = acc + dpp_f<0x141>(acc);  // row_half_mirror
  acc = acc + dpp_f<0x140>(acc);  // row_mirror
  return acc;
}

// Canonical distances of NOP x 4 pairs of rows in global memory: op k, group g
// (= lane / 16) takes the pair of rows (pa[k], pb[k]) its lanes hold. All
// loads of a 32-group slice of every op are issued before the arithmetic, so
// the batch costs one memory round trip per slice; the per-lane summation
// order is that of dist16.
template <int METRIC, int NOP>
__device__ __forceinline__ void dist16_rows(const float* const (&pa)[NOP],
                                            const float* const (&pb)[NOP], int d4, int sub,
                                            float (&out)[NOP]) {
  float acc[NOP];
#pragma unroll
  for (int k = 0; k < NOP; ++k) acc[k] = 0.0f;
  for (int q0 = 0; q0 < d4; q0 += 32) {
    float4 xa[NOP][2], xb[NOP][2];
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = q0 + sub + 16 * h;
        xa[k][h] = make_float4(0.f, 0.f, 0.f, 0.f);
        xb[k][h] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (q < d4) {
          xa[k][h] = *reinterpret_cast<const float4*>(pa[k] + 4 * q);
          xb[k][h] = *reinterpret_cast<const float4*>(pb[k] + 4 * q);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (q0 + sub + 16 * h < d4) acc[k] = pair_acc<METRIC>(xa[k][h], xb[k][h], acc[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < NOP; ++k) {
    const float s = row16_sum(acc[k]);
    out[k] = METRIC == 0 ? s : -s;
  }
}

// As dist16_rows, for pairs of point ids (ia[k], ib[k]) of X.
template <int METRIC, int NOP>
__device__ __forceinline__ void dist16_batch(const float* __restrict__ X, int64_t ld, int d4,
                                             const int (&ia)[NOP], const int (&ib)[NOP],
                                             int sub, float (&out)[NOP]) {
  const float* pa[NOP];
  const float* pb[NOP];
#pragma unroll
  for (int k = 0; k < NOP; ++k) {
    pa[k] = X + (int64_t)ia[k] * ld;
    pb[k] = X + (int64_t)ib[k] * ld;
  }
  dist16_rows<METRIC, NOP>(pa, pb, d4, sub, out);
}

template <int METRIC, class RA, class RB>
__device__ __forceinline__ float dist16(const RA& a, const RB& b, int d4, int sub) {
  float acc = 0.0f;
  for (int q = sub; q < d4; q += 16) acc = pair_acc<METRIC>(a(q), b(q), acc);
  acc = row16_sum(acc);
  return METRIC == 0 ? acc : -acc;
}

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }


// ----------------------------------------------------- wave utilities
__device__ __forceinline__ float rl_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ int rl_i(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

// Per lane: a where the lane's bit of the wave mask m is set, else b (one
// select with the mask as its condition).
__device__ __forceinline__ int lane_select(uint64_t m, int a, int b) {
  // m is wave-uniform; the read-first-lanes fold away when it already sits in
  // scalar registers and otherwise tell the compiler so
  const uint64_t mu =
      ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(m >> 32)) << 32) |
      (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)m);
  int r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mu));
  return r;
}
__device__ __forceinline__ uint64_t rl_u64(uint64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Lane T of each 16-lane row, broadcast to the whole row (DPP row_newbcast).
template <int T>
__device__ __forceinline__ int bcast16_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x150 + T, 0xF, 0xF, false);
}
template <int T>
__device__ __forceinline__ float bcast16_f(float x) {
  return __int_as_float(bcast16_i<T>(__float_as_int(x)));
}
template <int T>
__device__ __forceinline__ uint64_t bcast16_u64(uint64_t x) {
  const uint32_t lo = (uint32_t)bcast16_i<T>((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)bcast16_i<T>((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Calls f(std::integral_constant<int, I>) for I = B .. E-1, unrolled.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Rank of this lane's key among the keys of lanes [0, K), all distinct.
template <int KP>
__device__ __forceinline__ int rank_u64(uint64_t key, int K) {
  int r = 0;
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    if (j < K) r += (rl_u64(key, j) < key) ? 1 : 0;
  }
  return r;
}

}  // namespace grnnd
