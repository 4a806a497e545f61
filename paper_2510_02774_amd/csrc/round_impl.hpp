// round_impl.hpp -- update round and output pass, the hot path (gfx950, wave64).
//
// A classification pass (or the class the previous merge recorded) splits the
// vertices by pool shape. Compact pools (valid entries first) go to the
// grouped kernel of their size: at most 16 candidates (most pools after the
// first round) four vertices per wave, one per 16-lane row; at most 32, two
// per wave; at most 64, one per wave. Pools with holes (only ever handed in
// by a caller of grnnd_step) go to the one-pool kernel. Each wave takes its
// vertices from its class's list. For a vertex the grouped kernels
//   1. read the pool row (K candidates, sorted by (key, id)) and compute the
//      candidates' arrival order (Section 3.3);
//   2. load the candidate rows, in arrival order, straight into registers in
//      the operand layout of the matrix instructions (lane l holds row
//      16 I + l % 16, elements 4 (l / 16) .. + 3 of each 16-element step):
//      when every row of a pass is a BF16 value, one exact BF16 product per
//      element (16x16x16 BF16); other FP32 rows on the FP32 16x16x4
//      instruction, or, for rows of 512 elements or more, split into
//      hi = bf16(x) and lo = bf16(x - hi) with the Gram entry the sum of
//      hi hi', hi lo' and lo hi' on the BF16 instruction; narrow tiles use
//      the copy's 16x16x32 instruction;
//   3. turn the Gram tile into a symmetric distance tile in LDS, a packed
//      triangle in arrival order (D = G_ii + G_jj - 2 G_ij for L2, -G_ij for
//      IP); a decision within the tile's rigorous error bound of its
//      threshold is re-decided with the canonical distance (none when every
//      row is an integer row with a squared norm below 2^22: the tile is then
//      exact);
//   4. run the prune scan of Eq. 2 in arrival order on wave masks, reading
//      the comparison with arrival T at a fixed offset from each lane's row;
//   5. take each redirect key from the tile when it is exact; else, for
//      rows below 512 elements, compute it with the canonical distance on the
//      rows in global memory (one pair per 16-lane group per memory round
//      trip), and for longer rows leave it to the partner's merge
//      (kDeferredKey); emit one item per candidate (Alg. 4), or, for the
//      output pass, write the kept row.
// The one-pool kernel forms its tile on the FP32 matrix cores in pool order.
#pragma once
#include <math.h>

#include <type_traits>

#include "common.hpp"
#include "items.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {

// Task of this workgroup when ntask tasks are spread over the launch:
// workgroups are dealt to the 8 XCDs in turn, so XCD x takes the contiguous
// task range [x c, x c + c), c = ceil(ntask / 8), and the waves resident on
// one XCD work on neighbouring vertices of the list (whose candidate rows
// overlap in that XCD's L2). Returns ntask (no task) for workgroups beyond.
// The launch must have at least round_up(ntask, 8) workgroups.
__device__ __forceinline__ uint32_t xcd_task(uint32_t ntask) {
  const uint32_t c = (ntask + 7u) >> 3;
  const uint32_t x = blockIdx.x & 7u, k = blockIdx.x >> 3;
  if (k >= c) return ntask;
  const uint32_t t = x * c + k;
  return t < ntask ? t : ntask;
}

// Flags of row id (bit 0 integer, bit 1 BF16) for a lane holding a valid
// candidate: the build-wide value when every row has the same flags (two
// wave-uniform loads), else the row's own byte.
__device__ __forceinline__ uint32_t row_flags(const RoundArgs& A, bool valid, int id) {
  if (!A.rexact) return 0u;
  const uint32_t fa = A.rsum[0], fo = A.rsum[1];
  if (fa == fo) return valid ? fa : 0u;
  return valid ? (uint32_t)A.rexact[id] : 0u;
}

// Wave-uniform counters a round kernel accumulates over its vertices.
struct RoundStats {
  unsigned long long pairs = 0, rechecks = 0, redirects = 0, survivors = 0, cands = 0;
};

__device__ __forceinline__ void stat_add_r(unsigned long long* statp, int slot, int idx,
                                           unsigned long long v) {
  if (v) atomicAdd(statp + (size_t)slot * kStatStride + idx, v);
}

__device__ __forceinline__ void flush_stats(const RoundStats& st, unsigned long long* statp,
                                            bool final_pass, int lane) {
  if (lane != 0) return;
  const int slot = (int)(blockIdx.x % kStatSlots);
  if (final_pass) {
    stat_add_r(statp, slot, 7, st.pairs);
    stat_add_r(statp, slot, 1, st.rechecks);
  } else {
    stat_add_r(statp, slot, 0, st.pairs);
    stat_add_r(statp, slot, 1, st.rechecks);
    stat_add_r(statp, slot, 2, st.redirects);
    stat_add_r(statp, slot, 3, st.survivors);
    stat_add_r(statp, slot, 5, st.cands);
  }
}

// Per-wave LDS of the general kernel (floats): pool-order ids, keys and
// arrival->pool permutation (64 each), redirect pairs and keys, the distance
// tile (kp x ts, ts = kp + 4, row j holds D(i, j) at column i, both
// triangles), Gram diagonal.
struct Round3Lds {
  int ts, pid_off, pkey_off, perm_off, pair_off, rkey_off, sc_off, tile_off, g_off, total;
};

__host__ __device__ inline Round3Lds round3_lds(int kp) {
  Round3Lds L;
  L.ts = kp + 4;
  L.pid_off = 0;
  L.pkey_off = kWave;
  L.perm_off = 2 * kWave;
  L.pair_off = 3 * kWave;           // redirect pairs (2 x 64 ints)
  L.rkey_off = L.pair_off + 2 * kWave;  // redirect keys (64)
  L.sc_off = L.rkey_off + kWave;        // per-row scales of an FP8 tile (64)
  L.tile_off = L.sc_off + kWave;
  L.g_off = L.tile_off + kp * L.ts;
  L.total = L.g_off + kp;
  return L;
}

// Per-wave LDS of the grouped kernel with G = 64 / W pools of at most KW
// candidates each (floats): Gram diagonals (64), FP8 row scales (64, FP8
// tiles only), arrival-order records (key, pool index, margin, id, and for
// a narrow tile the row's rounding error and norm; 4 or 8 x 64), and G
// distance tiles, each the packed upper triangle of KW x KW with the
// diagonal (tri_index). The footprint sets how many waves a CU holds
// (160 KB of LDS), so arrays with disjoint lifetimes share space:
//   - the pool-order keys and the arrival permutation (64 each) are dead
//     before the records are written: they live in the record region;
//   - the ids (64) are read by each Gram pass before it writes its pools'
//     tiles: they live in the last pool's tile (after the sort keys when
//     there is one pool);
//   - the arrival sort keys (64 x 8 bytes) are dead before the tiles are
//     written, and the redirect pairs (2 x 64 ints) and keys (64) are
//     written only after the comparison masks and exact keys have been taken
//     from the tiles: both live at the start of the tile region.
template <int W, int PREC, int KW = W>
struct GroupLds {
  static constexpr int G = kWave / W;
  static constexpr int TILE = KW * (KW + 1) / 2;
  static constexpr int RS = PREC == GRNND_PREC_FP32 ? 4 : 8;  // record stride
  static constexpr int gdiag = 0;
  static constexpr int scale = kWave;  // per-row scales of an FP8 tile (64)
  static constexpr int rec = scale + (PREC == GRNND_PREC_FP8_E4M3 ? kWave : 0);
  static constexpr int pkey = rec, perm = rec + kWave;
  static constexpr int tiles = rec + RS * kWave;
  static constexpr int skey = tiles;
  static constexpr int pair = tiles;
  static constexpr int rkey = tiles + 2 * kWave;
  static constexpr int pid = tiles + (G - 1) * TILE + (G == 1 ? 2 * kWave : 0);
  static constexpr int total = tiles + G * TILE;
  static_assert(KW <= W && KW % 16 == 0, "pools of at most W candidates");
  static_assert(RS * kWave >= 2 * kWave, "the record region holds keys and permutation");
  static_assert(G * TILE >= 3 * kWave, "tile region holds the sort keys and redirect lists");
  static_assert(pid + kWave <= total, "the ids fit in the last tile");
};

// Position of D(lo, hi), lo <= hi < W, in a packed upper triangle of rows
// lo = 0, 1, ... (row lo holds hi = lo .. W - 1).
template <int W>
__device__ __forceinline__ int tri_index(int lo, int hi) {
  // both factors are below 2W <= 128: a full-rate 24-bit multiply
  return (int)(__umul24((unsigned)lo, (unsigned)(2 * W - 1 - lo)) >> 1) + hi;
}

// Canonical distances of up to four pairs given by point ids (global rows).
template <int METRIC>
__device__ __forceinline__ float glb_pair(const float* X, int64_t ld, int d4, int ia, int ib,
                                          int lane) {
  const GlobalRow a{X + (int64_t)ia * ld};
  const GlobalRow b{X + (int64_t)ib * ld};
  return dist16<METRIC>(a, b, d4, lane & 15);
}

// Re-decides the comparisons of lanes in nm with the canonical distance
// between the lane's candidate (cid) and the arriving candidate it meets
// (idt, as held by that lane); four pairs per wave operation.
template <int METRIC>
__device__ __forceinline__ void recheck_pairs(const float* X, int64_t ld, int d4, uint64_t nm,
                                              int cid, int idt, float thr, int lane, bool& cond,
                                              unsigned& nrecheck) {
  const int lk = lane >> 4;
  while (nm) {
    int w[4], ia[4], ib[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      w[g] = nm ? __ffsll((long long)nm) - 1 : -1;
      if (nm) nm &= nm - 1;
      const int wg = w[g] >= 0 ? w[g] : 0;
      ia[g] = rl_i(idt, wg);
      ib[g] = rl_i(cid, wg);
    }
    int ma = ia[0], mb = ib[0];
#pragma unroll
    for (int g = 1; g < 4; ++g)
      if (lk == g && w[g] >= 0) {
        ma = ia[g];
        mb = ib[g];
      }
    const float dd = glb_pair<METRIC>(X, ld, d4, ma, mb, lane);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (w[g] >= 0) {
        const float dg = rl_f(dd, 16 * g);
        if (lane == w[g]) cond = dg < thr;
        ++nrecheck;
      }
    }
  }
}

// Canonical redirect keys d(cid, pid) of the lanes in dm: the pairs are
// listed in LDS in lane order (s_pair, 2 ints each), computed 4 NOP per
// memory round trip (op k, lane group g: pair b + 4 k + g), and each such
// lane reads its key back from s_key. s_pair and s_key hold 128 ints and 64
// floats.
template <int METRIC, int NOP = 4>
__device__ __forceinline__ void redirect_keys(const float* X, int64_t ld, int d4, uint64_t dm,
                                              int cid, int pid, int lane, int* s_pair,
                                              float* s_key, float& ikey) {
  const int nred = __popcll(dm);
  if (nred == 0) return;
  const int li = lane & 15, lk = lane >> 4;
  const bool mine = (dm >> lane) & 1ull;
  const int rank = __popcll(dm & lanemask_lt(lane));
  if (mine) {
    s_pair[2 * rank] = cid;
    s_pair[2 * rank + 1] = pid;
  }
  __syncthreads();
  for (int b = 0; b < nred; b += 4 * NOP) {
    int ia[NOP], ib[NOP];
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
      const int r = min(b + 4 * k + lk, nred - 1);
      ia[k] = s_pair[2 * r];
      ib[k] = s_pair[2 * r + 1];
    }
    float dd[NOP];
    dist16_batch<METRIC, NOP>(X, ld, d4, ia, ib, li, dd);
    if (li == 0) {
#pragma unroll
      for (int k = 0; k < NOP; ++k) {
        const int r = b + 4 * k + lk;
        if (r < nred) s_key[r] = dd[k];
      }
    }
  }
  __syncthreads();
  if (mine) ikey = s_key[rank];
}

// Operand of one 32-element step of a narrow (BF16, FP16 or FP8) row: lane
// (li, lk) holds elements [32 s + 8 lk, 32 s + 8 lk + 8) of its row, the
// layout of the 16x16x32 matrix instructions (k = 8 (lane / 16) + element).
template <int PREC>
struct NarrowOp {
  using T = typename std::conditional<PREC == GRNND_PREC_FP8_E4M3, uint2, float4>::type;
  static constexpr int esz = PREC == GRNND_PREC_FP8_E4M3 ? 1 : 2;
};

template <int PREC>
__device__ __forceinline__ typename NarrowOp<PREC>::T narrow_load(const void* Xr, int64_t ldr,
                                                                  int row, int s, int lk) {
  const char* p = static_cast<const char*>(Xr) +
                  ((int64_t)row * ldr + 32 * s + 8 * lk) * NarrowOp<PREC>::esz;
  return *reinterpret_cast<const typename NarrowOp<PREC>::T*>(p);
}

typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef _Float16 v8f16 __attribute__((ext_vector_type(8)));

template <int PREC>
__device__ __forceinline__ v4f narrow_mfma(typename NarrowOp<PREC>::T a,
                                           typename NarrowOp<PREC>::T b, v4f c) {
  if constexpr (PREC == GRNND_PREC_BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, a),
                                                   __builtin_bit_cast(v8bf16, b), c, 0, 0, 0);
  } else if constexpr (PREC == GRNND_PREC_FP16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8f16, a),
                                                  __builtin_bit_cast(v8f16, b), c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                      __builtin_bit_cast(long, b), c, 0, 0, 0);
  }
}

// FP32 tile on the BF16 matrix cores: a float4 of a row (elements
// 4 (lane / 16) + 0..3 of a 16-element step, the operand layout of the
// 16x16x16 BF16 instruction) split into hi = bf16(x) and lo = bf16(x - hi)
// (round to nearest even; x - hi is exact in FP32).
typedef __bf16 v4bf16 __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf16 __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void split_bf16x4(const float4 x, v4bf16& hi, v4bf16& lo) {
  const v2bf16 h01 = __builtin_convertvector((v2f){x.x, x.y}, v2bf16);
  const v2bf16 h23 = __builtin_convertvector((v2f){x.z, x.w}, v2bf16);
  const uint32_t u01 = __builtin_bit_cast(uint32_t, h01), u23 = __builtin_bit_cast(uint32_t, h23);
  const v2bf16 l01 = __builtin_convertvector(
      (v2f){x.x - __uint_as_float(u01 << 16), x.y - __uint_as_float(u01 & 0xFFFF0000u)}, v2bf16);
  const v2bf16 l23 = __builtin_convertvector(
      (v2f){x.z - __uint_as_float(u23 << 16), x.w - __uint_as_float(u23 & 0xFFFF0000u)}, v2bf16);
  hi = __builtin_shufflevector(h01, h23, 0, 1, 2, 3);
  lo = __builtin_shufflevector(l01, l23, 0, 1, 2, 3);
}

// hi = bf16(x) alone, for rows whose elements are all BF16 values (exact).
__device__ __forceinline__ v4bf16 to_bf16x4(const float4 x) {
  const v2bf16 h01 = __builtin_convertvector((v2f){x.x, x.y}, v2bf16);
  const v2bf16 h23 = __builtin_convertvector((v2f){x.z, x.w}, v2bf16);
  return __builtin_shufflevector(h01, h23, 0, 1, 2, 3);
}

// One 16-element step of an FP32 Gram chain: c += hi_i hi_j + hi_i lo_j +
// lo_i hi_j, or hi_i hi_j alone when every row of the tile is a BF16 value
// (X1: the low parts are zero).
template <bool X1>
__device__ __forceinline__ v4f x3_mfma(const v4bf16 hi, const v4bf16 lo, const v4bf16 hj,
                                       const v4bf16 lj, v4f c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hi, hj, c, 0, 0, 0);
  if constexpr (!X1) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hi, lj, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lo, hj, c, 0, 0, 0);
  }
  return c;
}

// Bound on |D - D_exact| of a narrow tile entry D for the pair (a, b), from
// each row's rounding error e = |s q - (x - c)| and norm nn = |x - c|, with
// acc the bound on the entry's FP32 accumulation error (the per-row terms
// mcoef (nn + e)^2 of both rows). L2: with E = e_a + e_b and y~, y the
// narrow and exact rows, | |y~_a - y~_b| - |y_a - y_b| | <= E, so
// |D - D_exact| <= E (2 |y~_a - y~_b| + E) + acc, and |y~_a - y~_b|^2 <=
// max(D, 0) + acc; the bound scales with the distance, not the norms.
// IP: e_a nn_b + e_b nn_a + e_a e_b + acc. Raised slightly for its own FP32
// rounding.
template <int METRIC>
__device__ __forceinline__ float narrow_pair_margin(float D, float acc, float ea, float na,
                                                    float eb, float nb) {
  float m;
  if (METRIC == 0) {
    const float E = ea + eb;
    m = E * (2.0f * sqrtf(fmaxf(D, 0.0f) + acc) + E);
  } else {
    m = ea * nb + eb * na + ea * eb;
  }
  return m * 1.0001f;
}

// Source of the Gram tile: the FP32 points, or a narrow copy (ldr elements
// per row, zero padded to a multiple of 32) with per-row FP8 scales sc
// (indexed like the pool; null for BF16 and FP16).
struct GramSrc {
  const float* X;
  int64_t ld;
  int d4;
  const void* Xr;
  int64_t ldr;
  const float* sc;
};

// Gram tile of the first NBK 16-row blocks of the pool (rows past K repeat
// row 0) on the 16x16x4 FP32 matrix cores, then the symmetric distance tile
// in LDS: D(i, j) = G_ii + G_jj - 2 G_ij (L2) or -G_ij (IP); row j of the tile
// holds D(i, j) at column i, and gdiag receives G_ii. Every block runs the
// same number of chained steps (out-of-range float4 groups load as zeros), so
// the chains carry no branches. Lane l supplies row 16 I + l % 16, float4
// group 4 s + l / 16 of a step; the accumulator of block (I, J) holds
// G(16 I + 4 (l / 16) + r, 16 J + l % 16) in register r.
template <int METRIC, int NBK, int PREC, class F>
__device__ __forceinline__ void gram_tile(const GramSrc& S, const int* m_pid, int K, float* tile,
                                          float* gdiag, int ts, int li, int lk, F&& first) {
  constexpr int CH = NBK <= 2 ? 8 : 4;  // steps per load batch
  constexpr int NBL = NBK * (NBK + 1) / 2;
  const float* X = S.X;
  const int64_t ld = S.ld;
  const int d4 = S.d4;
  int rid[NBK];
#pragma unroll
  for (int I = 0; I < NBK; ++I) {
    const int r = 16 * I + li;
    rid[I] = (r < K) ? m_pid[r] : m_pid[0];
  }
  v4f acc[NBL];
#pragma unroll
  for (int b = 0; b < NBL; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC != GRNND_PREC_FP32) {
    using T = typename NarrowOp<PREC>::T;
    const int nsteps = (int)(S.ldr / 32);
    for (int s0 = 0; s0 < nsteps; s0 += CH) {
      T ra[NBK][CH];
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int I = 0; I < NBK; ++I) {
          ra[I][c] = T{};
          if (s0 + c < nsteps) ra[I][c] = narrow_load<PREC>(S.Xr, S.ldr, rid[I], s0 + c, lk);
        }
      if (s0 == 0) first();
#pragma unroll
      for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int I = 0; I < NBK; ++I)
#pragma unroll
          for (int J = 0; J <= I; ++J)
            acc[I * (I + 1) / 2 + J] = narrow_mfma<PREC>(ra[I][c], ra[J][c], acc[I * (I + 1) / 2 + J]);
    }
  } else {
  const int nsteps = (d4 + 3) >> 2;
  for (int s0 = 0; s0 < nsteps; s0 += CH) {
    float4 ra[NBK][CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int g = 4 * (s0 + c) + lk;
#pragma unroll
      for (int I = 0; I < NBK; ++I) {
        ra[I][c] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g < d4) ra[I][c] = *reinterpret_cast<const float4*>(X + (int64_t)rid[I] * ld + 4 * g);
      }
    }
    if (s0 == 0) first();
#pragma unroll
    for (int c = 0; c < CH; ++c) {
#pragma unroll
      for (int I = 0; I < NBK; ++I) {
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          v4f cc = acc[I * (I + 1) / 2 + J];
          const float4 ai = ra[I][c], aj = ra[J][c];
          cc = __builtin_amdgcn_mfma_f32_16x16x4f32(ai.x, aj.x, cc, 0, 0, 0);
          cc = __builtin_amdgcn_mfma_f32_16x16x4f32(ai.y, aj.y, cc, 0, 0, 0);
          cc = __builtin_amdgcn_mfma_f32_16x16x4f32(ai.z, aj.z, cc, 0, 0, 0);
          cc = __builtin_amdgcn_mfma_f32_16x16x4f32(ai.w, aj.w, cc, 0, 0, 0);
          acc[I * (I + 1) / 2 + J] = cc;
        }
      }
    }
  }
  }
  if constexpr (PREC == GRNND_PREC_FP8_E4M3) {  // undo the per-row scales
#pragma unroll
    for (int I = 0; I < NBK; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const float scj = S.sc[16 * J + li];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[I * (I + 1) / 2 + J][r] *= S.sc[16 * I + 4 * lk + r] * scj;
      }
  }
#pragma unroll
  for (int I = 0; I < NBK; ++I) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * lk + r == li) gdiag[16 * I + li] = acc[I * (I + 1) / 2 + I][r];
  }
  __syncthreads();
#pragma unroll
  for (int I = 0; I < NBK; ++I) {
    float gi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) gi[r] = gdiag[16 * I + 4 * lk + r];
#pragma unroll
    for (int J = 0; J <= I; ++J) {
      const int j = 16 * J + li;
      const float gj = gdiag[j];
      const v4f G = acc[I * (I + 1) / 2 + J];
      float Dv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) Dv[r] = (METRIC == 0) ? (gi[r] + gj) - 2.0f * G[r] : -G[r];
      const int i0 = 16 * I + 4 * lk;
      *reinterpret_cast<float4*>(tile + j * ts + i0) = make_float4(Dv[0], Dv[1], Dv[2], Dv[3]);
      if (I != J) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tile[(i0 + r) * ts + j] = Dv[r];
      }
    }
  }
}

// Gram and distance tiles of pools QB .. QB + PP - 1 of width W of a grouped
// wave (pool q's ids at s_pid[q W, q W + W), absent entries standing as row
// 0). All chains (NBK (NBK + 1) / 2 row-block pairs per pool, NBK = W / 16) advance
// together one 16-float step at a time, with the loads of the next step in
// flight while the current one runs on the matrix cores (deeper prefetch
// costs registers, and with them waves per SIMD); out-of-range
// float4 groups load as zeros, so the chains carry no branches. Tile q is
// written like gram_tile's, with row stride W + 4.
// FP32 tiles (PREC == GRNND_PREC_FP32) take one of three forms: X1, every
// row a BF16 value: one BF16 product per element (exact); else X3: the
// three-product BF16 split (for long rows, where the FP32 matrix cores'
// time matters); else four 16x16x4 FP32 products per 16 elements.
template <int METRIC, int W, int PREC, int QB, int PP, bool X1, int NBKP = W / 16,
          bool X3 = false>
__device__ __forceinline__ void gram_pass(const GramSrc& S, const int* s_pid, float* tiles,
                                          float* gdiag, int li, int lk) {
  using L = GroupLds<W, PREC, 16 * NBKP>;
  constexpr int G = PP, NBK = NBKP, NBL = NBK * (NBK + 1) / 2, CS = 1;
  using T = typename std::conditional<PREC == GRNND_PREC_FP32, float4,
                                      typename NarrowOp<PREC>::T>::type;
  const float* X = S.X;
  const int64_t ld = S.ld;
  const int d4 = S.d4;
  // FP32: 16-float steps (four 16x16x4 instructions); narrow: 32-element
  // steps (one 16x16x32 instruction)
  const int nsteps = PREC == GRNND_PREC_FP32 ? (d4 + 3) >> 2 : (int)(S.ldr / 32);
  int rid[G][NBK];
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int I = 0; I < NBK; ++I) rid[q][I] = s_pid[(QB + q) * W + 16 * I + li];
  v4f acc[G][NBL];
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int b = 0; b < NBL; ++b) acc[q][b] = v4f{0.f, 0.f, 0.f, 0.f};
  T a[G][NBK][CS], b[G][NBK][CS];
  auto load = [&](T(&buf)[G][NBK][CS], int s0) {
#pragma unroll
    for (int c = 0; c < CS; ++c) {
#pragma unroll
      for (int q = 0; q < G; ++q)
#pragma unroll
        for (int I = 0; I < NBK; ++I) {
          buf[q][I][c] = T{};
          if constexpr (PREC == GRNND_PREC_FP32) {
            const int g = 4 * (s0 + c) + lk;
            if (g < d4)
              buf[q][I][c] = *reinterpret_cast<const float4*>(X + (int64_t)rid[q][I] * ld + 4 * g);
          } else {
            if (s0 + c < nsteps) buf[q][I][c] = narrow_load<PREC>(S.Xr, S.ldr, rid[q][I], s0 + c, lk);
          }
        }
    }
  };
  auto chains = [&](const T(&buf)[G][NBK][CS]) {
#pragma unroll
    for (int c = 0; c < CS; ++c)
#pragma unroll
      for (int q = 0; q < G; ++q) {
        if constexpr (PREC == GRNND_PREC_FP32 && X1) {
          v4bf16 hi[NBK];
#pragma unroll
          for (int I = 0; I < NBK; ++I) hi[I] = to_bf16x4(buf[q][I][c]);
#pragma unroll
          for (int I = 0; I < NBK; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J)
              acc[q][I * (I + 1) / 2 + J] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                  hi[I], hi[J], acc[q][I * (I + 1) / 2 + J], 0, 0, 0);
        } else if constexpr (PREC == GRNND_PREC_FP32 && X3) {
          v4bf16 hi[NBK], lo[NBK];
#pragma unroll
          for (int I = 0; I < NBK; ++I) split_bf16x4(buf[q][I][c], hi[I], lo[I]);
#pragma unroll
          for (int I = 0; I < NBK; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J)
              acc[q][I * (I + 1) / 2 + J] =
                  x3_mfma<false>(hi[I], lo[I], hi[J], lo[J], acc[q][I * (I + 1) / 2 + J]);
        } else if constexpr (PREC == GRNND_PREC_FP32) {
#pragma unroll
          for (int I = 0; I < NBK; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J) {
              v4f cc = acc[q][I * (I + 1) / 2 + J];
              const float4 xi = buf[q][I][c], xj = buf[q][J][c];
              cc = __builtin_amdgcn_mfma_f32_16x16x4f32(xi.x, xj.x, cc, 0, 0, 0);
              cc = __builtin_amdgcn_mfma_f32_16x16x4f32(xi.y, xj.y, cc, 0, 0, 0);
              cc = __builtin_amdgcn_mfma_f32_16x16x4f32(xi.z, xj.z, cc, 0, 0, 0);
              cc = __builtin_amdgcn_mfma_f32_16x16x4f32(xi.w, xj.w, cc, 0, 0, 0);
              acc[q][I * (I + 1) / 2 + J] = cc;
            }
        } else {
#pragma unroll
          for (int I = 0; I < NBK; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J)
              acc[q][I * (I + 1) / 2 + J] =
                  narrow_mfma<PREC>(buf[q][I][c], buf[q][J][c], acc[q][I * (I + 1) / 2 + J]);
        }
      }
  };
  if constexpr (PREC == GRNND_PREC_FP32) {
    load(a, 0);
    for (int s0 = 0; s0 < nsteps; s0 += 2 * CS) {
      load(b, s0 + CS);
      chains(a);
      load(a, s0 + 2 * CS);
      chains(b);
    }
  } else {
    // one buffer: with a ping-pong pair the compiler rotates the narrow
    // chains through different accumulator tuples
    for (int s0 = 0; s0 < nsteps; s0 += CS) {
      load(a, s0);
      chains(a);
    }
  }
  if constexpr (PREC == GRNND_PREC_FP8_E4M3) {  // undo the per-row scales
#pragma unroll
    for (int q = 0; q < G; ++q)
#pragma unroll
      for (int I = 0; I < NBK; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          const float scj = S.sc[(QB + q) * W + 16 * J + li];
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[q][I * (I + 1) / 2 + J][r] *= S.sc[(QB + q) * W + 16 * I + 4 * lk + r] * scj;
        }
  }
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int I = 0; I < NBK; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * lk + r == li) gdiag[(QB + q) * W + 16 * I + li] = acc[q][I * (I + 1) / 2 + I][r];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < G; ++q) {
    float* tile = tiles + (QB + q) * L::TILE;
#pragma unroll
    for (int I = 0; I < NBK; ++I) {
      float gi[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) gi[r] = gdiag[(QB + q) * W + 16 * I + 4 * lk + r];
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int j = 16 * J + li;
        const float gj = gdiag[(QB + q) * W + j];
        const v4f Gm = acc[q][I * (I + 1) / 2 + J];
        float Dv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Dv[r] = (METRIC == 0) ? (gi[r] + gj) - 2.0f * Gm[r] : -Gm[r];
        const int i0 = 16 * I + 4 * lk;
        // each pair once, at (min, max) of the packed triangle
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r;
          if (I != J || i <= j)
            tile[tri_index<16 * NBKP>(I != J ? j : i, I != J ? i : j)] = Dv[r];
        }
      }
    }
  }
}

// All G pools of the wave. The FP32 kernels form their pools' tiles in
// passes -- the 32-wide one pool at a time, the 16-wide two at a time -- so
// that only part of the accumulators and load buffers is live at once, which
// keeps both at six waves per SIMD.
// bf16m: wave mask of the lanes whose pool entry is absent or a row of BF16
// values; a pass over pools that hold only such rows skips the low parts.
template <int METRIC, int W, int PREC, int NBKP = W / 16, bool X3 = false>
__device__ __forceinline__ void gram_group(const GramSrc& S, const int* s_pid, float* tiles,
                                           float* gdiag, int li, int lk, uint64_t bf16m) {
  constexpr int G = GroupLds<W, PREC>::G;
  constexpr uint64_t kSeg = W == 64 ? ~0ull : ((1ull << W) - 1ull);
  if constexpr (W == 32 && PREC == GRNND_PREC_FP32) {
    if ((bf16m & kSeg) == kSeg)
      gram_pass<METRIC, W, PREC, 0, 1, true, W / 16, X3>(S, s_pid, tiles, gdiag, li, lk);
    else
      gram_pass<METRIC, W, PREC, 0, 1, false, W / 16, X3>(S, s_pid, tiles, gdiag, li, lk);
    if ((bf16m >> 32) == kSeg)
      gram_pass<METRIC, W, PREC, 1, 1, true, W / 16, X3>(S, s_pid, tiles, gdiag, li, lk);
    else
      gram_pass<METRIC, W, PREC, 1, 1, false, W / 16, X3>(S, s_pid, tiles, gdiag, li, lk);
  } else if constexpr (W == 16 && PREC == GRNND_PREC_FP32) {
    // two passes of two pools: half the live accumulators and loads
    if ((bf16m & 0xFFFFFFFFull) == 0xFFFFFFFFull)
      gram_pass<METRIC, W, PREC, 0, 2, true, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk);
    else
      gram_pass<METRIC, W, PREC, 0, 2, false, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk);
    if ((bf16m >> 32) == 0xFFFFFFFFull)
      gram_pass<METRIC, W, PREC, 2, 2, true, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk);
    else
      gram_pass<METRIC, W, PREC, 2, 2, false, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk);
  } else if constexpr (PREC == GRNND_PREC_FP32) {
    if (bf16m == ~0ull)
      gram_pass<METRIC, W, PREC, 0, G, true, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk);
    else
      gram_pass<METRIC, W, PREC, 0, G, false, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk);
  } else {
    gram_pass<METRIC, W, PREC, 0, G, false, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk);
  }
}

}  // namespace

// ------------------------------------------------------- general kernel
// One vertex per wave, any pool (holes allowed, up to 64 candidates).
template <int METRIC, int NB, int PREC, bool FINAL>
__device__ __forceinline__ void round_vertex(const RoundArgs& A, int64_t v, float* lds,
                                             RoundStats& st) {
  constexpr int KP = 16 * NB;
  const Round3Lds L = round3_lds(KP);
  int* m_pid = reinterpret_cast<int*>(lds + L.pid_off);
  float* m_pkey = lds + L.pkey_off;
  int* m_perm = reinterpret_cast<int*>(lds + L.perm_off);
  float* tile = lds + L.tile_off;
  float* gdiag = lds + L.g_off;
  const int ts = L.ts, d4 = A.d4, R = A.R;
  const int64_t ld = A.ld;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;

  int id0 = -1;
  float key0 = INFINITY;
  if (lane < R) {
    id0 = A.in_ids[v * R + lane];
    key0 = A.in_keys[v * R + lane];
  }
  // ---- 1. pool row, compacted to valid ids in [0, n)
  const bool valid0 = id0 >= 0 && (int64_t)id0 < A.n;
  const uint64_t vm = ballot(valid0);
  const int K = __popcll(vm);
  if (vm != (K == 64 ? ~0ull : ((1ull << K) - 1ull))) {
    if (valid0) {
      const int pos = __popcll(vm & lanemask_lt(lane));
      m_pid[pos] = id0;
      m_pkey[pos] = key0;
    }
    __syncthreads();
    id0 = lane < K ? m_pid[lane] : -1;
    key0 = lane < K ? m_pkey[lane] : INFINITY;
    __syncthreads();
  }
  const bool valid = lane < K;
  const int id = valid ? id0 : -1;
  const float key = valid ? key0 : INFINITY;

  if (K <= 1) {
    if (FINAL) {
      if (lane < R) {
        A.out_adj[v * R + lane] = id;
        if (A.out_keys) A.out_keys[v * R + lane] = key;
      }
    } else {
      if (lane == 0) {
        A.items.nown[v] = K;
        if (K == 1) A.items.own[v * R] = item_pack(id, key);
      }
      st.survivors += (unsigned)K;
      st.cands += (unsigned)K;
    }
    return;
  }

  m_pid[lane] = id;
  m_pkey[lane] = key;
  if (PREC == GRNND_PREC_FP8_E4M3) lds[L.sc_off + lane] = valid ? A.rscale[id] : 1.0f;
  // row flags of the pool entry this lane holds (bit 0 integer, bit 1 BF16)
  const uint32_t rf = row_flags(A, valid, id);
  __syncthreads();
  const GramSrc S{A.X, ld, d4, A.Xr, A.ldr, lds + L.sc_off};

  // ---- 2-3. arrival order, Gram tile and distance tile of the active
  //           16-row blocks (a straight-line chain per block count)
  auto arrival = [&]() {  // Section 3.3, computed while the rows arrive
    int arr = lane;
    if (!FINAL) {
      if (A.order == 2) {
        arr = K - 1 - lane;
      } else if (A.order == 0) {
        const VSeg sg = vseg_of(A.seg, v, A.seed, A.n);
        const uint64_t sk =
            valid ? hash_order_key(hash4(sg.seed, kTagUpdate + A.round, (uint64_t)(v - sg.base),
                                         (uint64_t)(uint32_t)(id - sg.base)), id)
                  : ~0ull;
        arr = rank_u64<KP>(sk, K);
      }
    }
    if (valid) m_perm[arr] = lane;
  };
  const int nbk = (K + 15) >> 4;
  auto tile_nb = [&](auto nbc) {
    gram_tile<METRIC, decltype(nbc)::value, PREC>(S, m_pid, K, tile, gdiag, ts, li, lk, arrival);
  };
  if (nbk <= 1) {
    tile_nb(std::integral_constant<int, 1>{});
  } else if (nbk == 2) {
    if constexpr (NB >= 2) tile_nb(std::integral_constant<int, 2>{});
  } else if (nbk == 3) {
    if constexpr (NB >= 3) tile_nb(std::integral_constant<int, 3>{});
  } else {
    if constexpr (NB >= 4) tile_nb(std::integral_constant<int, 4>{});
  }
  __syncthreads();
  // a tile over integer rows with squared norms below 2^22 is exact (every
  // partial sum an integer below 2^24) and equal to the canonical
  // distances: then no comparison needs re-deciding
  const bool exact_pool =
      PREC == GRNND_PREC_FP32 &&
      ballot(valid && !((rf & 1u) && gdiag[lane] < 4194304.0f)) == 0ull;

  // ---- 4. candidates in arrival order: lane t holds candidate t
  const int pidx = valid ? m_perm[lane] : 0;  // its pool index = (key, id) rank
  const int cid = valid ? m_pid[pidx] : -1;
  const float ckey = valid ? m_pkey[pidx] : INFINITY;
  // per-candidate margin term; a narrow tile adds a pair term from the rows'
  // rounding errors and norms
  float ce = 0.0f, cn = 0.0f, cg;
  if constexpr (PREC == GRNND_PREC_FP32) {
    cg = (valid && !exact_pool) ? A.mcoef_f32 * fabsf(gdiag[pidx]) : 0.0f;
  } else {
    if (valid) {
      const float2 ri = A.rinfo[cid];
      ce = ri.x;
      cn = ri.y;
    }
    cg = valid ? A.mcoef * (cn + ce) * (cn + ce) : 0.0f;
  }
  const float* trow = tile + pidx * ts;  // D(., this candidate) in pool order

  uint64_t alive = 1ull;
  int partner = -1;
  unsigned nrecheck = 0;
#pragma unroll 1
  for (int t = 1; t < K; ++t) {
    const float kt = rl_f(ckey, t);
    const int pt = rl_i(pidx, t);
    float band = rl_f(cg, t) + cg;
    const bool inA = (alive >> lane) & 1ull;
    const float Dtw = trow[pt];
    if constexpr (PREC != GRNND_PREC_FP32)
      band += narrow_pair_margin<METRIC>(Dtw, band, ce, cn, rl_f(ce, t), rl_f(cn, t));
    const float thr = fmaxf(kt, ckey);
    bool cond = inA && (Dtw < thr);
    const uint64_t nm = ballot(inA && (fabsf(Dtw - thr) <= band));
    if (nm) recheck_pairs<METRIC>(A.X, ld, d4, nm, cid, rl_i(cid, t), thr, lane, cond, nrecheck);
    const uint64_t hit = ballot(cond);
    const uint64_t ufar = ballot(cond && pidx < pt);  // a closer alive w: t is the far one
    if (ufar) {
      const int p = __ffsll((long long)ufar) - 1;
      const uint64_t rem = hit & ((1ull << p) - 1ull);
      alive &= ~rem;
      if ((rem >> lane) & 1ull) partner = t;
      if (lane == t) partner = p;
    } else {
      alive &= ~hit;
      if ((hit >> lane) & 1ull) partner = t;
      alive |= 1ull << t;
    }
  }
  st.pairs += (unsigned long long)K * (K - 1) / 2;
  st.rechecks += nrecheck;

  if (FINAL) {
    const bool isal = (alive >> lane) & 1ull;
    const int na = __popcll(alive);
    const int pos = __popcll(alive & lanemask_lt(lane));
    const int64_t o = v * R;
    if (isal) {
      A.out_adj[o + pos] = cid;
      if (A.out_keys) A.out_keys[o + pos] = ckey;
    }
    if (lane >= na && lane < R) {  // padding; slots >= na are never written above
      A.out_adj[o + lane] = -1;
      if (A.out_keys) A.out_keys[o + lane] = INFINITY;
    }
    return;
  }

  // ---- 5. one item per candidate: a survivor stays with v (head of v's own
  //         row, in pool order); a redirected candidate goes to its partner
  const bool isdead = valid && !((alive >> lane) & 1ull);
  const int pid_all = __shfl(cid, partner >= 0 ? partner : 0);  // partner's id
  const uint64_t dm = ballot(isdead);
  const int nred = __popcll(dm);
  uint32_t slot = 0;
  if (isdead) slot = atomicAdd(&A.items.cnt[pid_all], 1u);
  float ikey = ckey;
  if (A.defer) {  // left to the partner's merge
    if (isdead) ikey = __uint_as_float(kDeferredKey);
  } else {
    redirect_keys<METRIC>(A.X, ld, d4, dm, cid, pid_all, lane,
                          reinterpret_cast<int*>(lds + L.pair_off), lds + L.rkey_off, ikey);
  }
  if (valid && !isdead)
    A.items.own[v * R + (lane - __popcll(dm & lanemask_lt(lane)))] = item_pack(cid, ikey);
  send_items(A.items, isdead, pid_all, slot, cid, ikey, lane);
  if (lane == 0) A.items.nown[v] = K - nred;
  st.redirects += (unsigned)nred;
  st.survivors += (unsigned)(K - nred);
  st.cands += (unsigned)K;
}

template <int METRIC, int NB, int PREC, bool FINAL>
__global__ __launch_bounds__(64) void k_round(const RoundArgs A) {
  extern __shared__ __align__(16) float lds[];
  const uint32_t nv = min(A.vcount[3], (uint32_t)A.n);
  const uint32_t task = xcd_task(nv);
  if (task >= nv) return;
  RoundStats st;
  round_vertex<METRIC, NB, PREC, FINAL>(A, (int64_t)A.vlist_b[task], lds, st);
  flush_stats(st, A.statp, FINAL, threadIdx.x);
}

// ------------------------------------------------------- grouped kernel
// G = 64 / W vertices per wave, one per W-lane group g; lane (g, t) first
// holds pool entry t of its vertex, then, once the arrival order is known,
// the candidate that arrives t-th. Pools are compact with K <= W entries.
// The arriving candidate's key, pool index and margin reach its group by a
// DPP row broadcast (W = 16) or one LDS record read (W = 32).
template <int METRIC, int W, int PREC, bool FINAL, int NBKP = W / 16, bool X3 = false>
__global__ __launch_bounds__(64) void k_round_g(const RoundArgs A) {
  constexpr int KW = 16 * NBKP;  // the most candidates a pool of this kernel has
  using L = GroupLds<W, PREC, KW>;
  constexpr int G = L::G;
  constexpr uint64_t kSeg = W == 64 ? ~0ull : ((1ull << W) - 1ull);
  extern __shared__ __align__(16) float lds[];
  int* s_pid = reinterpret_cast<int*>(lds + L::pid);
  float* s_pkey = lds + L::pkey;
  int* s_perm = reinterpret_cast<int*>(lds + L::perm);
  float* s_rec = lds + L::rec;
  uint64_t* s_sk = reinterpret_cast<uint64_t*>(lds + L::skey);
  float* tiles = lds + L::tiles;
  float* gdiag = lds + L::gdiag;
  const int lane = threadIdx.x;
  const int g = lane / W, t = lane % W;
  const int li = lane & 15, lk = lane >> 4;
  const int d4 = A.d4, R = A.R;
  const int64_t ld = A.ld;
  const int cls = W == 16 ? 0 : (W == 32 ? 1 : 2);
  const uint32_t nv = min(A.vcount[cls], (uint32_t)A.n);
  const uint32_t ntask = (nv + (uint32_t)G - 1u) / (uint32_t)G;
  const uint32_t task = xcd_task(ntask);
  if (task >= ntask) return;
  const int32_t* vlist = W == 16 ? A.vlist_s : (W == 32 ? A.vlist_m : A.vlist_l);
  RoundStats st;

  const uint32_t vi = (uint32_t)G * task + (uint32_t)g;
  const bool gv = vi < nv;
  const int64_t v = gv ? (int64_t)vlist[vi] : 0;
  int id = -1;
  float key = INFINITY;
  if (gv && t < R) {
    id = A.in_ids[v * R + t];
    key = A.in_keys[v * R + t];
  }
  const bool valid = gv && id >= 0 && (int64_t)id < A.n;  // a prefix of each group
  if (!valid) {
    id = -1;
    key = INFINITY;
  }
  const uint64_t vm = ballot(valid);
  const int Kg = __popcll((vm >> (W * g)) & kSeg);
  int Kmax = 0;
#pragma unroll
  for (int q = 0; q < G; ++q) Kmax = max(Kmax, __popcll((vm >> (W * q)) & kSeg));

  s_pid[lane] = valid ? id : 0;  // row 0 stands in for absent entries
  s_pkey[lane] = key;
  if (PREC == GRNND_PREC_FP8_E4M3) lds[L::scale + lane] = A.rscale[valid ? id : 0];

  // ---- arrival order within each group (Section 3.3)
  int arr = t;
  if (!FINAL) {
    if (A.order == 2) {
      arr = Kg - 1 - t;
    } else if (A.order == 0) {
      const VSeg sg = vseg_of(A.seg, v, A.seed, A.n);
      const uint64_t sk =
          valid ? hash_order_key(hash4(sg.seed, kTagUpdate + A.round, (uint64_t)(v - sg.base),
                                       (uint64_t)(uint32_t)(id - sg.base)), id)
                : ~0ull;
      int r = 0;
      if constexpr (W == 16) {
        static_for<0, 16>([&](auto jc) {
          constexpr int J = decltype(jc)::value;
          r += (bcast16_u64<J>(sk) < sk) ? 1 : 0;
        });
      } else {
        s_sk[lane] = sk;
        __syncthreads();
#pragma unroll 8
        for (int j = 0; j < W; ++j) r += (s_sk[g * W + j] < sk) ? 1 : 0;
      }
      arr = r;
    }
  }
  __syncthreads();
  if (valid) s_perm[g * W + arr] = t;
  __syncthreads();

  // ---- lane (g, t) takes the candidate arriving t-th: its pool index (the
  //      rank of its (key, id)), id and key
  const int pidx = valid ? s_perm[g * W + t] : 0;
  const int cid = valid ? s_pid[g * W + pidx] : -1;
  const float ckey = valid ? s_pkey[g * W + pidx] : INFINITY;
  __syncthreads();
  // the tiles are formed in arrival order: row t of group g is the candidate
  // arriving t-th, so the scan finds D(t, T) at a fixed offset from a
  // per-lane base
  s_pid[lane] = valid ? cid : 0;  // row 0 stands in for absent entries
  if (PREC == GRNND_PREC_FP8_E4M3) lds[L::scale + lane] = A.rscale[valid ? cid : 0];
  __syncthreads();

  // ---- Gram and distance tiles of the G vertices; row flags of the
  //      candidate this lane holds (bit 0 integer, bit 1 BF16)
  const uint32_t rf = row_flags(A, valid, cid);
  const GramSrc S{A.X, ld, d4, A.Xr, A.ldr, lds + L::scale};
  gram_group<METRIC, W, PREC, NBKP, X3>(S, s_pid, tiles, gdiag, li, lk,
                                        ballot(!valid || (rf & 2u)));
  __syncthreads();
  // groups whose rows are all integers with squared norms below 2^22 have an
  // exact tile equal to the canonical distances: nothing to re-decide
  uint32_t exact_grp = 0;
  if constexpr (PREC == GRNND_PREC_FP32) {
    const uint64_t bad = ballot(valid && !((rf & 1u) && gdiag[lane] < 4194304.0f));
    exact_grp = ((bad >> (W * g)) & kSeg) == 0ull ? 1u : 0u;
  }
  // integer-valued candidate row (its redirect key may come from the tile)
  constexpr bool kExactKeys =
      !FINAL && METRIC == 0 && (PREC == GRNND_PREC_FP32 || PREC == GRNND_PREC_BF16 ||
                                PREC == GRNND_PREC_FP16);
  const bool rowx = kExactKeys && (rf & 1u) != 0;
  float ce = 0.0f, cn = 0.0f, cg;
  if constexpr (PREC == GRNND_PREC_FP32) {
    cg = (valid && !exact_grp) ? A.mcoef * fabsf(gdiag[lane]) : 0.0f;
  } else {
    if (valid) {
      const float2 ri = A.rinfo[cid];
      ce = ri.x;
      cn = ri.y;
    }
    cg = valid ? A.mcoef * (cn + ce) * (cn + ce) : 0.0f;
  }
  const float* gtile = tiles + g * L::TILE;
  // trow[T] = D(t, T) for t <= T (lanes t >= KW hold no candidate and read
  // the last row)
  const float* trow = gtile + tri_index<KW>(min(t, KW - 1), 0);
  if constexpr (W != 16) {
    *reinterpret_cast<float4*>(s_rec + L::RS * lane) =
        make_float4(ckey, __int_as_float(pidx), cg, __int_as_float(cid));
    if constexpr (PREC != GRNND_PREC_FP32)
      *reinterpret_cast<float2*>(s_rec + L::RS * lane + 4) = make_float2(ce, cn);
    __syncthreads();
  }

  // ---- what each lane needs of arrival T of its group: its key, pool
  //      index, margin term (and a narrow tile's row error and norm), and
  //      the tile entry D(this candidate, arrival T)
  struct Arrival {
    float D, kt, cgt, et, nt;
    int pt;
  };
  auto record = [&](auto tc) {  // all of arrival T but its tile entry
    constexpr int T = decltype(tc)::value;
    Arrival r;
    r.D = 0.0f;
    r.et = 0.0f;
    r.nt = 0.0f;
    if constexpr (W == 16) {
      r.kt = bcast16_f<T>(ckey);
      r.pt = bcast16_i<T>(pidx);
      r.cgt = bcast16_f<T>(cg);
      if constexpr (PREC != GRNND_PREC_FP32) {
        r.et = bcast16_f<T>(ce);
        r.nt = bcast16_f<T>(cn);
      }
    } else {
      const float4 rc = *reinterpret_cast<const float4*>(s_rec + L::RS * (g * W + T));
      r.kt = rc.x;
      r.pt = __float_as_int(rc.y);
      r.cgt = rc.z;
      if constexpr (PREC != GRNND_PREC_FP32) {
        const float2 re = *reinterpret_cast<const float2*>(s_rec + L::RS * (g * W + T) + 4);
        r.et = re.x;
        r.nt = re.y;
      }
    }
    return r;
  };
  auto fetch = [&](auto tc) {  // arrival T with the tile entry D(t, T)
    constexpr int T = decltype(tc)::value;
    Arrival r = record(tc);
    r.D = trow[T];  // read by the lanes t < T only (the others are not compared)
    return r;
  };
  int kq[G];
#pragma unroll
  for (int q = 0; q < G; ++q) kq[q] = __popcll((vm >> (W * q)) & kSeg);

  // ---- the prune scan (Eq. 2) over arrivals, on wave masks. The comparison
  //      of each lane's candidate with arrival T comes straight from the tile
  //      (at the fixed offset T from the lane's row base) as the scan reaches
  //      T; step T + 1's reads are issued before step T's branches, so they
  //      overlap with it.
  uint64_t group0 = 0;
#pragma unroll
  for (int q = 0; q < G; ++q) group0 |= 1ull << (W * q);
  uint64_t alive = vm & group0;  // the first arrival of each group
  int partner = -1;
  unsigned nrecheck = 0;
  Arrival cur = fetch(std::integral_constant<int, 1>{});
  static_for<1, KW>([&](auto tc) {
    constexpr int T = decltype(tc)::value;
    if (T < Kmax) {
      Arrival nxt = cur;
      if constexpr (T + 1 < KW) nxt = fetch(std::integral_constant<int, T + 1>{});
      float band = cur.cgt + cg;
      if constexpr (PREC != GRNND_PREC_FP32)
        band += narrow_pair_margin<METRIC>(cur.D, band, ce, cn, cur.et, cur.nt);
      const float thr = fmaxf(cur.kt, ckey);
      uint64_t gm = 0;  // groups whose vertex has a T-th arrival
#pragma unroll
      for (int q = 0; q < G; ++q)
        if (kq[q] > T) gm |= kSeg << (W * q);
      const uint64_t act = alive & gm;
      uint64_t hit = ballot(cur.D < thr) & act;
      const uint64_t nb = ballot(fabsf(cur.D - thr) <= band) & act;
      if (nb) {  // near the threshold: decide with the canonical distance
        int idt;
        if constexpr (W == 16) {
          idt = bcast16_i<T>(cid);
        } else {
          idt = __float_as_int(s_rec[L::RS * (g * W + T) + 3]);
        }
        bool cond = (hit >> lane) & 1ull;
        recheck_pairs<METRIC>(A.X, ld, d4, nb, cid, idt, thr, lane, cond, nrecheck);
        hit = (hit & ~nb) | (ballot(cond) & nb);
      }
      // a hit closer than T (smaller pool index) makes T the far one: the
      // first such hit in arrival order kills T and spares the later hits;
      // without one every hit dies. Each lane finds the first closer hit of
      // its own group (p; none: all ones, above every t) and decides for
      // itself.
      const uint64_t ufar = ballot(pidx < cur.pt) & hit;
      const uint64_t ufg = (ufar >> (W * g)) & kSeg;
      const uint32_t p = ufg ? (uint32_t)__builtin_ctzll(ufg) : ~0u;
      const uint64_t rem = ballot((uint32_t)t < p) & hit;     // killed by T
      const uint64_t tdm = ballot(ufg != 0ull) & (group0 << T);  // T-th arrivals killed
      alive = (alive & ~rem) | ((group0 << T) & ~tdm & vm);
      partner = lane_select(rem, T, partner);
      partner = lane_select(tdm, (int)p, partner);
      cur = nxt;
    }
  });
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const unsigned long long kq = (unsigned long long)__popcll((vm >> (W * q)) & kSeg);
    st.pairs += kq * (kq - (kq > 0 ? 1 : 0)) / 2;
  }
  st.rechecks += nrecheck;

  if (FINAL) {
    const uint64_t aseg = (alive >> (W * g)) & kSeg;
    const int na = __popcll(aseg);
    const int pos = __popcll(aseg & lanemask_lt(t));
    if (gv) {
      const int64_t o = v * R;
      if ((aseg >> t) & 1ull) {
        A.out_adj[o + pos] = cid;
        if (A.out_keys) A.out_keys[o + pos] = ckey;
      }
      for (int sl = t; sl < R; sl += W) {
        if (sl >= na) {
          A.out_adj[o + sl] = -1;
          if (A.out_keys) A.out_keys[o + sl] = INFINITY;
        }
      }
    }
  } else {
    const bool isdead = valid && !((alive >> lane) & 1ull);
    const int psrc = g * W + (partner >= 0 ? partner : 0);
    const int pid_all = __shfl(cid, psrc);
    const uint64_t dm = ballot(isdead);
    // bucket slots, one counter update per partner: each redirected lane
    // ranks itself among the lanes sent to the same partner (LDS counters in
    // the record region, which the scan no longer needs) and the partner's
    // lane reserves that many slots of its own id's bucket at once
    uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_rec);
    s_cnt[lane] = 0u;
    __syncthreads();
    uint32_t rank = 0;
    if (isdead) rank = atomicAdd(&s_cnt[psrc], 1u);
    __syncthreads();
    const uint32_t nto = s_cnt[lane];
    uint32_t base = 0;
    if (nto) base = atomicAdd(&A.items.cnt[cid], nto);  // this lane is the partner
    __syncthreads();
    s_cnt[lane] = base;
    __syncthreads();
    uint32_t slot = 0;
    if (isdead) slot = s_cnt[psrc] + rank;
    float ikey = ckey;
    // exact redirect keys: when both rows are integer-valued, held exactly
    // and with squared norms below 2^22, every partial sum and product of the
    // tile entry ((g_a + g_b) - 2 G_ab, with |G_ab| <= sqrt(g_a g_b) and the
    // distance at most 2 (g_a + g_b) < 2^24) and of the canonical distance is
    // an integer below 2^24, hence exact: the tile entry is the key
    uint64_t dx = 0;
    if constexpr (kExactKeys) {
      // a narrow copy must hold the row exactly (zero rounding error)
      const bool xs = rowx && (PREC == GRNND_PREC_FP32 || ce == 0.0f) &&
                      gdiag[lane] < 4194304.0f;
      const bool ex = isdead && xs && __shfl((int)xs, psrc) != 0;
      dx = ballot(ex);
      // the tile is in arrival order: the pair (t, partner)
      if (ex) ikey = gtile[tri_index<KW>(min(t, partner), max(t, partner))];
    }
    if (A.defer) {
      // left to the partner's merge, which reads the partner's row once for
      // all the items it receives and skips candidates it already holds
      if (((dm & ~dx) >> lane) & 1ull) ikey = __uint_as_float(kDeferredKey);
    } else {
      // one pair per 16-lane group per memory round trip: the batch's row
      // buffers would otherwise set the kernel's register count
      redirect_keys<METRIC, 1>(A.X, ld, d4, dm & ~dx, cid, pid_all, lane,
                               reinterpret_cast<int*>(lds + L::pair), lds + L::rkey, ikey);
    }
    const uint64_t dseg = (dm >> (W * g)) & kSeg;
    if (valid && !isdead)  // survivors at the head of v's own row, in arrival order
      A.items.own[v * R + (t - __popcll(dseg & lanemask_lt(t)))] = item_pack(cid, ikey);
    send_items(A.items, isdead, pid_all, slot, cid, ikey, lane);
    if (gv && t == 0) A.items.nown[v] = Kg - __popcll(dseg);
    const unsigned nred = (unsigned)__popcll(dm), ncand = (unsigned)__popcll(vm);
    st.redirects += nred;
    st.survivors += ncand - nred;
    st.cands += ncand;
  }
  flush_stats(st, A.statp, FINAL, lane);
}

// ------------------------------------------------------- tile probe
// One candidate set per wave: its tile formed as in a round (gram_tile), then
// for every ordered pair of its K entries the tile distance, the recheck band
// the rounds use and the canonical distance.
template <int METRIC, int NB, int PREC>
__global__ __launch_bounds__(64) void k_tile_probe(const RoundArgs A, const int32_t* __restrict__ ids,
                                                   float* __restrict__ out_tile,
                                                   float* __restrict__ out_band,
                                                   float* __restrict__ out_canon) {
  constexpr int KP = 16 * NB;
  const Round3Lds L = round3_lds(KP);
  extern __shared__ __align__(16) float lds[];
  int* m_pid = reinterpret_cast<int*>(lds + L.pid_off);
  float* tile = lds + L.tile_off;
  float* gdiag = lds + L.g_off;
  float* s_cg = lds + L.pkey_off;
  float* s_ce = lds + L.perm_off;
  float* s_cn = lds + L.pair_off;
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int R = A.R, ts = L.ts;
  const int64_t q = blockIdx.x;
  const int id0 = lane < R ? ids[q * R + lane] : -1;
  const bool valid0 = id0 >= 0 && (int64_t)id0 < A.n;
  const uint64_t vm = ballot(valid0);
  const int K = __popcll(vm);
  if (valid0) m_pid[__popcll(vm & lanemask_lt(lane))] = id0;
  __syncthreads();
  const bool valid = lane < K;
  const int id = valid ? m_pid[lane] : 0;
  __syncthreads();
  m_pid[lane] = id;  // row 0 stands in for absent entries
  if (PREC == GRNND_PREC_FP8_E4M3) lds[L.sc_off + lane] = valid ? A.rscale[id] : 1.0f;
  __syncthreads();
  if (K < 2) return;
  const GramSrc S{A.X, A.ld, A.d4, A.Xr, A.ldr, lds + L.sc_off};
  auto none = [] {};
  const uint32_t rf = row_flags(A, valid, id);
  const int nbk = (K + 15) >> 4;
  auto tile_nb = [&](auto nbc) {
    gram_tile<METRIC, decltype(nbc)::value, PREC>(S, m_pid, K, tile, gdiag, ts, li, lk, none);
  };
  if (nbk <= 1) {
    tile_nb(std::integral_constant<int, 1>{});
  } else if (nbk == 2) {
    if constexpr (NB >= 2) tile_nb(std::integral_constant<int, 2>{});
  } else if (nbk == 3) {
    if constexpr (NB >= 3) tile_nb(std::integral_constant<int, 3>{});
  } else {
    if constexpr (NB >= 4) tile_nb(std::integral_constant<int, 4>{});
  }
  __syncthreads();
  const bool exact_pool =
      PREC == GRNND_PREC_FP32 &&
      ballot(valid && !((rf & 1u) && gdiag[lane] < 4194304.0f)) == 0ull;
  float ce = 0.0f, cn = 0.0f, cg;
  if constexpr (PREC == GRNND_PREC_FP32) {
    cg = (valid && !exact_pool) ? A.mcoef_f32 * fabsf(gdiag[lane]) : 0.0f;
  } else {
    if (valid) {
      const float2 ri = A.rinfo[id];
      ce = ri.x;
      cn = ri.y;
    }
    cg = valid ? A.mcoef * (cn + ce) * (cn + ce) : 0.0f;
  }
  s_cg[lane] = cg;
  s_ce[lane] = ce;
  s_cn[lane] = cn;
  __syncthreads();
  if (valid) {
    const int64_t o = (q * R + lane) * R;
    for (int j = 0; j < K; ++j) {
      if (j == lane) continue;
      const float D = tile[lane * ts + j];
      float band = s_cg[j] + cg;
      if constexpr (PREC != GRNND_PREC_FP32)
        band += narrow_pair_margin<METRIC>(D, band, ce, cn, s_ce[j], s_cn[j]);
      out_tile[o + j] = D;
      out_band[o + j] = band;
    }
  }
  // canonical distances, four pairs per step (one per 16-lane group); the
  // distance is symmetric, so pair (i, j), i < j, also gives (j, i)
  for (int p0 = 0; p0 < K * K; p0 += 4) {
    const int pp = p0 + lk;
    const int i = pp / K, j = pp % K;
    const bool use = pp < K * K && i < j;
    const float dc = glb_pair<METRIC>(A.X, A.ld, A.d4, m_pid[use ? i : 0], m_pid[use ? j : 0], lane);
    if (use && li == 0) {
      out_canon[(q * R + i) * R + j] = dc;
      out_canon[(q * R + j) * R + i] = dc;
    }
  }
}

template <int METRIC, int NB, int PREC>
static hipError_t launch_tile_probe_t(const RoundArgs& a, const int32_t* ids, int64_t nv,
                                      float* out_tile, float* out_band, float* out_canon,
                                      hipStream_t s) {
  const size_t lds = (size_t)round3_lds(16 * NB).total * sizeof(float);
  hipLaunchKernelGGL((k_tile_probe<METRIC, NB, PREC>), dim3((unsigned)nv), dim3(64), lds, s, a, ids,
                     out_tile, out_band, out_canon);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_tile_probe_prec(const RoundArgs& a, int metric, const int32_t* ids,
                                         int64_t nv, float* t, float* b, float* c, hipStream_t s) {
  const int nb = (a.R + 15) / 16;
  if (metric == 0) {
    switch (nb) {
      case 1: return launch_tile_probe_t<0, 1, PREC>(a, ids, nv, t, b, c, s);
      case 2: return launch_tile_probe_t<0, 2, PREC>(a, ids, nv, t, b, c, s);
      case 3: return launch_tile_probe_t<0, 3, PREC>(a, ids, nv, t, b, c, s);
      default: return launch_tile_probe_t<0, 4, PREC>(a, ids, nv, t, b, c, s);
    }
  }
  switch (nb) {
    case 1: return launch_tile_probe_t<1, 1, PREC>(a, ids, nv, t, b, c, s);
    case 2: return launch_tile_probe_t<1, 2, PREC>(a, ids, nv, t, b, c, s);
    case 3: return launch_tile_probe_t<1, 3, PREC>(a, ids, nv, t, b, c, s);
    default: return launch_tile_probe_t<1, 4, PREC>(a, ids, nv, t, b, c, s);
  }
}

// ------------------------------------------------------- launch templates
template <int METRIC, int NB, int PREC, bool FINAL>
static hipError_t launch_round_t(const RoundArgs& a, hipStream_t s) {
  const size_t lds = (size_t)round3_lds(16 * NB).total * sizeof(float);
  const unsigned grid = (unsigned)((a.n + 7) / 8 * 8);
  hipLaunchKernelGGL((k_round<METRIC, NB, PREC, FINAL>), dim3(grid), dim3(64), lds, s, a);
  return hipGetLastError();
}

template <int METRIC, int W, int PREC, bool FINAL, int NBKP = W / 16>
static hipError_t launch_round_g(const RoundArgs& a, hipStream_t s) {
  constexpr int G = kWave / W;
  constexpr size_t lds = (size_t)GroupLds<W, PREC, 16 * NBKP>::total * sizeof(float);
  const unsigned grid = (unsigned)(((a.n + G - 1) / G + 7) / 8 * 8);
  if (PREC == GRNND_PREC_FP32 && a.x3)
    hipLaunchKernelGGL((k_round_g<METRIC, W, PREC, FINAL, NBKP, PREC == GRNND_PREC_FP32>),
                       dim3(grid), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL((k_round_g<METRIC, W, PREC, FINAL, NBKP, false>), dim3(grid), dim3(64),
                       lds, s, a);
  return hipGetLastError();
}

// Compact pools go to the grouped kernels by size (at most 16, 32, 64
// candidates; the last one sized for R), other pools to the one-pool kernel.
// compact_pools: every input row is known to be compact (it was written by
// init or a merge), so the one-pool kernel has nothing to do; classes above
// what R allows are empty and not launched either.
template <int METRIC, int PREC, bool FINAL>
static hipError_t launch_round_m(const RoundArgs& a, bool compact_pools, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (!compact_pools) {
    switch ((a.R + 15) / 16) {
      case 1: e = launch_round_t<METRIC, 1, PREC, FINAL>(a, s); break;
      case 2: e = launch_round_t<METRIC, 2, PREC, FINAL>(a, s); break;
      case 3: e = launch_round_t<METRIC, 3, PREC, FINAL>(a, s); break;
      default: e = launch_round_t<METRIC, 4, PREC, FINAL>(a, s); break;
    }
    if (e != hipSuccess) return e;
  }
  if (a.R > 32) {
    e = a.R <= 48 ? launch_round_g<METRIC, 64, PREC, FINAL, 3>(a, s)
                  : launch_round_g<METRIC, 64, PREC, FINAL, 4>(a, s);
    if (e != hipSuccess) return e;
  }
  if (a.R > 16)
    if ((e = launch_round_g<METRIC, 32, PREC, FINAL>(a, s)) != hipSuccess) return e;
  return launch_round_g<METRIC, 16, PREC, FINAL>(a, s);
}

// All round launches of one tile precision and metric.
template <int PREC, int METRIC>
static hipError_t launch_round_pm(const RoundArgs& a, bool final_pass, bool compact_pools,
                                  hipStream_t s) {
  return final_pass ? launch_round_m<METRIC, PREC, true>(a, compact_pools, s)
                    : launch_round_m<METRIC, PREC, false>(a, compact_pools, s);
}

// All round launches of one tile precision.
template <int PREC>
static hipError_t launch_round_prec(const RoundArgs& a, int metric, bool final_pass,
                                    bool compact_pools, hipStream_t s) {
  return metric == 0 ? launch_round_pm<PREC, 0>(a, final_pass, compact_pools, s)
                     : launch_round_pm<PREC, 1>(a, final_pass, compact_pools, s);
}

}  // namespace grnnd
