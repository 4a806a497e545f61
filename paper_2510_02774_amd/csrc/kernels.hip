// kernels.hip -- GRNND construction kernels for gfx950 (wave64, MFMA).
//
// Initial pools, reverse-edge sampling, and the merge that fills the write
// pool from the items a round emits (Section 3.5). The round kernel itself is
// in round.hip.
#include <math.h>

#include "common.hpp"
#include "items.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {

__device__ __forceinline__ void stat_add(unsigned long long* statp, int slot, int idx,
                                         unsigned long long v) {
  if (v) atomicAdd(statp + (size_t)slot * kStatStride + idx, v);
}

}  // namespace

// ------------------------------------------------------------------- clear
__global__ void k_clear(uint32_t* __restrict__ cnt, int64_t n, uint32_t* cursor,
                        unsigned long long* statp, float* zero16) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = 0;
  if (i < (int64_t)kStatSlots * kStatStride && statp) statp[i] = 0ull;
  if (i < 64 && zero16) zero16[i] = 0.0f;
  if (i < kCursorWords && cursor) cursor[i] = 0u;  // merge cursors, list lengths
}

// Copies points into rows of ldp floats (d rounded up to 4), zero padded.
__global__ void k_pad_copy(const float* __restrict__ X, int64_t n, int32_t d,
                           float* __restrict__ Xp, int32_t ldp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * (int64_t)ldp) return;
  const int64_t r = i / ldp;
  const int32_t c = (int32_t)(i % ldp);
  Xp[i] = (c < d) ? X[r * d + c] : 0.0f;
}

// -------------------------------------------------------------------- init
// Initial pools (Alg. 3): the first min(S, n-1) distinct ids
// != v of the hash stream h(seed, 0x3000, v, j) mod n, j = 0, 1, ..., with
// their keys, written as a pool row sorted by (key, id) and padded.
template <int METRIC, int NB>
__global__ __launch_bounds__(64) void k_init(const InitArgs A) {
  __shared__ int coll[kWave];
  __shared__ float ckey[kWave];
  constexpr int KP = 16 * NB;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t v = blockIdx.x;
  // the vertex's collection (the whole point set unless the build is batched)
  const VSeg sg = vseg_of(A.seg, v, A.seed, A.n);
  const int want = (int)((int64_t)A.S < sg.n - 1 ? (int64_t)A.S : sg.n - 1);

  int got = 0;
  for (uint64_t j0 = 0; got < want; j0 += kWave) {
    const uint64_t h = hash4(sg.seed, kTagInit, (uint64_t)(v - sg.base), j0 + (uint64_t)lane);
    const int c = (int)(sg.base + (int64_t)(h % (uint64_t)sg.n));
    bool ok = (int64_t)c != v;
    for (int q = 0; q < got; ++q) ok = ok && (coll[q] != c);
    const uint64_t okm = ballot(ok);
    bool dup = false;
    for (int l2 = 0; l2 < kWave; ++l2) {
      const int c2 = rl_i(c, l2);
      dup = dup || (((okm >> l2) & 1ull) && l2 < lane && c2 == c);
    }
    const bool nw = ok && !dup;
    const uint64_t nm = ballot(nw);
    const int pos = got + __popcll(nm & lanemask_lt(lane));
    if (nw && pos < want) coll[pos] = c;
    __syncthreads();
    got = min(want, got + __popcll(nm));
  }

  // canonical keys d(v, coll[q]) straight from the rows in memory, 16 pairs
  // per round trip (op k, lane group lk: pair b + 4 k + lk)
  for (int b = 0; b < want; b += 16) {
    constexpr int NOP = 4;
    int ia[NOP], ib[NOP];
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
      ia[k] = (int)v;
      ib[k] = coll[min(b + 4 * k + lk, want - 1)];
    }
    float dd[NOP];
    dist16_batch<METRIC, NOP>(A.X, A.ld, A.d4, ia, ib, li, dd);
    if (li == 0) {
#pragma unroll
      for (int k = 0; k < NOP; ++k)
        if (b + 4 * k + lk < want) ckey[b + 4 * k + lk] = dd[k];
    }
  }
  __syncthreads();
  const float mykey = lane < want ? ckey[lane] : INFINITY;
  const int myid = lane < want ? coll[lane] : -1;
  const uint64_t sk =
      lane < want ? (((uint64_t)key_to_ord(mykey) << 32) | (uint32_t)myid) : ~0ull;
  const int rnk = rank_u64<KP>(sk, want);
  const int64_t o = v * A.R;
  if (lane < want) {
    A.out_ids[o + rnk] = myid;
    A.out_keys[o + rnk] = mykey;
  } else if (lane < A.R) {
    A.out_ids[o + lane] = -1;
    A.out_keys[o + lane] = INFINITY;
  }
  if (lane == 0) {
    if (A.cnt) A.cnt[v] = 0u;
    stat_add(A.statp, (int)(blockIdx.x % kStatSlots), 6, (unsigned long long)want);
  }
}

// ----------------------------------------------------------------- reverse
// REVERSE_EDGE_SAMPLING (Section 3.6): v sends itself to the floor(rho * k)
// entries of its row that come first in hash order (or, with A.nearest, the
// nearest ones: first by (key, id)), and re-sends its whole row to itself;
// the merge then fills the write pool as in a round.
// G = 64 / W vertices per wave (W >= R), one per W-lane group; a lane's rank
// in that order counts the smaller sort keys of its group, read from LDS
// (rows padded by two words so that the groups' broadcast reads hit other
// banks).
template <int W>
__global__ __launch_bounds__(64) void k_reverse(const ReverseArgs A) {
  constexpr int G = kWave / W, SP = W + 2;
  __shared__ int m_id[kWave];
  __shared__ float m_key[kWave];
  __shared__ uint64_t m_sk[G * SP];
  const int lane = threadIdx.x, g = lane / W, t = lane % W;
  const int64_t v = (int64_t)blockIdx.x * G + g;
  const bool live = v < A.n;
  int id0 = -1;
  float key0 = INFINITY;
  if (live && t < A.R) {
    id0 = A.in_ids[v * A.R + t];
    key0 = A.in_keys[v * A.R + t];
  }
  const bool valid0 = id0 >= 0 && (int64_t)id0 < A.n;
  const uint64_t vm = ballot(valid0);
  const uint64_t gmask = W == kWave ? ~0ull : ((1ull << W) - 1ull);
  const uint64_t seg = (vm >> (g * W)) & gmask;
  const int K = __popcll(seg);
  if (valid0) {
    const int pos = __popcll(seg & ((1ull << t) - 1ull));
    m_id[g * W + pos] = id0;
    m_key[g * W + pos] = key0;
  }
  // floor(rho * K) of each group from wave-uniform table lookups
  int m = 0;
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int mq = A.mtab[__popcll((vm >> (q * W)) & gmask)];
    if (g == q) m = mq;
  }
  __syncthreads();
  const bool valid = t < K;
  const int id = valid ? m_id[lane] : -1;
  const float key = valid ? m_key[lane] : INFINITY;
  const VSeg sg = vseg_of(A.seg, live ? v : 0, A.seed, A.n);
  const uint64_t sk =
      !valid ? ~0ull
      : A.nearest ? (((uint64_t)key_to_ord(key) << 32) | (uint32_t)id)
                  : hash_order_key(hash4(sg.seed, kTagReverse + A.t1, (uint64_t)(v - sg.base),
                                         (uint64_t)(uint32_t)(id - sg.base)), id);
  m_sk[g * SP + t] = sk;
  __syncthreads();
  int rnk = 0;
#pragma unroll 8
  for (int j = 0; j < W; ++j) rnk += (j < K && m_sk[g * SP + j] < sk) ? 1 : 0;
  if (valid) A.items.own[v * A.R + t] = item_pack(id, key);  // the row, in pool order
  const bool send = valid && rnk < m;
  uint32_t slot = 0;
  if (send) slot = atomicAdd(&A.items.cnt[id], 1u);
  send_items(A.items, send, id, slot, (int)v, key, lane);
  if (live && t == 0) A.items.nown[v] = K;
}

// --------------------------------------------------------- exact rows
// 1 when every element of the row is an integer. Sixteen lanes per row, each
// reading 16-byte groups (rows start 16-byte aligned, ld is a multiple of 4),
// so a wave reads four rows with full-width loads; elements past d are not
// looked at.
// Row flags: bit 0 when every element is an integer, bit 1 when every element
// is exactly a BF16 value (the low 16 bits of its FP32 encoding are zero).
__device__ __forceinline__ bool is_bf16(float x) { return (__float_as_uint(x) & 0xFFFFu) == 0u; }

__global__ void k_rowflags_init(uint32_t* rsum) {
  rsum[0] = 3u;
  rsum[1] = 0u;
}

__global__ __launch_bounds__(256) void k_rowflags(const float* __restrict__ X, int64_t n,
                                                  int32_t d, int32_t ld, uint8_t* __restrict__ rexact,
                                                  uint32_t* __restrict__ rsum) {
  const int64_t v = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int l16 = threadIdx.x & 15;
  bool ok = true, hb = true;
  if (v < n) {
    const float* row = X + v * ld;
    for (int q = l16; 4 * q < d; q += 16) {
      const float4 x = *reinterpret_cast<const float4*>(row + 4 * q);
      const int e = 4 * q;
      ok = ok && x.x == rintf(x.x) && (e + 1 >= d || x.y == rintf(x.y)) &&
           (e + 2 >= d || x.z == rintf(x.z)) && (e + 3 >= d || x.w == rintf(x.w));
      hb = hb && is_bf16(x.x) && (e + 1 >= d || is_bf16(x.y)) && (e + 2 >= d || is_bf16(x.z)) &&
           (e + 3 >= d || is_bf16(x.w));
    }
  }
  const unsigned long long bad = ballot(!ok), badh = ballot(!hb);
  const int g = (threadIdx.x & 63) >> 4;
  const uint32_t f = ((((bad >> (16 * g)) & 0xffffull) == 0ull) ? 1u : 0u) |
                     ((((badh >> (16 * g)) & 0xffffull) == 0ull) ? 2u : 0u);
  if (v < n && l16 == 0) rexact[v] = (uint8_t)f;
  // the wave's AND and OR over its rows, merged into rsum only where they
  // change it (on uniform data almost no wave writes)
  uint32_t fa = 3u, fo = 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t vq = (int64_t)blockIdx.x * 16 + 4 * (threadIdx.x >> 6) + q;
    const uint32_t fq = (uint32_t)__shfl((int)f, 16 * q);
    if (vq < n) {
      fa &= fq;
      fo |= fq;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    const uint32_t ca = __atomic_load_n(&rsum[0], __ATOMIC_RELAXED);
    const uint32_t co = __atomic_load_n(&rsum[1], __ATOMIC_RELAXED);
    if ((ca & fa) != ca) atomicAnd(&rsum[0], fa);
    if ((co | fo) != co) atomicOr(&rsum[1], fo);
  }
}

// ------------------------------------------------------------------- merge
// Merge input of destination x: the nown[x] items it kept (head of its own
// row), min(cnt[x], bcap) items in its bucket and cnt[x] - bcap overflow
// items, which k_alloc gives a contiguous range of seg and k_scatter moves
// there. k_alloc also sorts the destinations into four merge lists by input
// size (at most 16, 32, 64, more). Placement and list order are irrelevant:
// the merge result depends only on the multiset of items per destination.

// Merge width class of an input of m items.
__device__ __forceinline__ int merge_class(uint32_t m) {
  return m <= 16u ? 0 : (m <= 32u ? 1 : (m <= 64u ? 2 : 3));
}

// 1024 destinations per block, 4 per thread; one cursor update per block for
// the overflow ranges and one per list.
__global__ __launch_bounds__(256) void k_alloc(const MergeArgs A) {
  __shared__ uint32_t wsum[5][4];
  __shared__ uint32_t base_s[5];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t x0 = (int64_t)blockIdx.x * 1024 + 4 * threadIdx.x;
  const uint32_t bcap = (uint32_t)A.items.bcap;
  uint32_t o[4], nwn[4], rcv[4];
  uint32_t cm[4];  // class bit masks of the thread's destinations
  uint32_t cnum[5] = {0u, 0u, 0u, 0u, 0u};  // overflow items, then list counts
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[k] = nwn[k] = rcv[k] = 0u;
    cm[k] = 0u;
    if (x0 + k < A.n) {
      const uint32_t f = A.items.cnt[x0 + k];
      A.items.cnt[x0 + k] = 0u;  // cleared for the next pass, in id order
      nwn[k] = (uint32_t)A.items.nown[x0 + k];
      rcv[k] = f;
      const uint32_t m = nwn[k] + f;
      o[k] = f > bcap ? f - bcap : 0u;
      const int c = merge_class(m);
      cm[k] = 1u << c;
      cnum[1 + c] += 1u;
    }
    cnum[0] += o[k];
  }
  uint32_t incl[5];
#pragma unroll
  for (int l = 0; l < 5; ++l) incl[l] = cnum[l];
#pragma unroll
  for (int sh = 1; sh < kWave; sh <<= 1) {
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      const uint32_t y = __shfl_up(incl[l], sh);
      if (lane >= sh) incl[l] += y;
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int l = 0; l < 5; ++l) wsum[l][wv] = incl[l];
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int l = threadIdx.x;
    const uint32_t tot = wsum[l][0] + wsum[l][1] + wsum[l][2] + wsum[l][3];
    uint32_t* cur = l == 0 ? &A.cursor[0] : &A.cursor[4 + l];
    base_s[l] = tot ? atomicAdd(cur, tot) : 0u;
    // counters: items beyond their destination's bucket, and destinations
    // with more than 64 input items (the chunked merge)
    if (l == 0 || l == 4) stat_add(A.statp, (int)(blockIdx.x % kStatSlots), l == 0 ? 8 : 9, tot);
  }
  __syncthreads();
  uint32_t pos[5];
#pragma unroll
  for (int l = 0; l < 5; ++l) {
    pos[l] = base_s[l] + incl[l] - cnum[l];
    for (int k = 0; k < wv; ++k) pos[l] += wsum[l][k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (x0 + k < A.n) {
      // list entry: destination, kept items, received items, overflow start
      const uint4 e = make_uint4((uint32_t)(x0 + k), nwn[k], rcv[k], pos[0]);
      if (o[k]) A.off[x0 + k] = pos[0];  // read by the overflow scatter only
      pos[0] += o[k];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (cm[k] & (1u << c)) A.mlist[(int64_t)c * A.n + pos[1 + c]++] = e;
    }
  }
}

// Moves the overflow items into their destinations' ranges of seg.
__global__ __launch_bounds__(256) void k_scatter(const MergeArgs A) {
  const uint32_t total = *A.items.ovf_n;
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < total; i += gridDim.x * 256u) {
    const uint4 e = A.items.ovf[i];
    A.seg[A.off[e.x] + e.y] = make_uint2(e.z, e.w);
  }
}

namespace {
// Lane exchange x[lane ^ j] of a 32-bit value. For j <= 8 it stays in the
// vector ALU with data-parallel lane moves (quad permutes, the row rotate by
// 8, and for j = 4 the half-row mirror followed by the quad reversal), so the
// short steps that make up most of a sorting network do not go through the
// LDS crossbar; j = 16 and 32 use the LDS permute.
template <int C>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, C, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int j) {
  switch (j) {
    case 1: return dpp_mov<0xB1>(v);                  // quad_perm [1, 0, 3, 2]
    case 2: return dpp_mov<0x4E>(v);                  // quad_perm [2, 3, 0, 1]
    case 4: return dpp_mov<0x1B>(dpp_mov<0x141>(v));  // quad_perm [3, 2, 1, 0] after row_half_mirror
    case 8: return dpp_mov<0x128>(v);                 // row_ror:8
    default: return (uint32_t)__shfl_xor(v, j);
  }
}
__device__ __forceinline__ uint64_t lane_xor_u64(uint64_t x, int j) {
  const uint32_t lo = lane_xor((uint32_t)x, j), hi = lane_xor((uint32_t)(x >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}
// x[lane - 1] (0 in lane 0) with the whole-wave shift by one lane.
__device__ __forceinline__ uint64_t lane_up1_u64(uint64_t x) {
  const uint32_t lo = dpp_mov<0x138>((uint32_t)x), hi = dpp_mov<0x138>((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// One compare-exchange of a bitonic network: keeps min(x, y) where keep_min,
// else max(x, y). Written as one compare and one select so that the lane
// pattern keep_min stays a wave mask (one compare, a mask op and two selects
// per 64-bit exchange).
__device__ __forceinline__ uint64_t cmp_xchg(uint64_t x, uint64_t y, bool keep_min) {
  return ((x < y) == keep_min) ? x : y;
}

// Bitonic sort of 128 uint64 held two per lane (index h*64 + lane).
__device__ __forceinline__ void wave_sort128(uint64_t& e0, uint64_t& e1, int lane) {
#pragma unroll
  for (int k = 2; k <= 2 * kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == kWave) {
        const uint64_t lo = e0 < e1 ? e0 : e1, hi = e0 < e1 ? e1 : e0;
        e0 = lo;
        e1 = hi;
      } else {
        const uint64_t y0 = lane_xor_u64(e0, j), y1 = lane_xor_u64(e1, j);
        const bool lower = (lane & j) == 0;
        const bool up0 = (lane & k) == 0, up1 = ((kWave + lane) & k) == 0;
        e0 = cmp_xchg(e0, y0, lower == up0);
        e1 = cmp_xchg(e1, y1, lower == up1);
      }
    }
  }
}

// Bitonic sort within independent segments of W lanes (W a power of two).
template <int W>
__device__ __forceinline__ uint64_t seg_sort_u64(uint64_t x, int lane) {
#pragma unroll
  for (int k = 2; k <= W; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t y = lane_xor_u64(x, j);
      const bool up = k == W || (lane & k) == 0;  // every segment ends ascending
      const bool lower = (lane & j) == 0;
      x = cmp_xchg(x, y, lower == up);
    }
  }
  return x;
}

// (cand, key order); a deferred key (kDeferredKey) takes the largest order,
// so that after a sort by (cand, order) a key the destination already holds
// for the same candidate comes first.
constexpr uint32_t kOrdDeferred = 0xFFFFFFFFu;
__device__ __forceinline__ uint64_t cand_ord(uint2 it) {
  const uint32_t o = it.y == kDeferredKey ? kOrdDeferred : key_to_ord(__uint_as_float(it.y));
  return ((uint64_t)it.x << 32) | o;
}
// (cand, ord) -> (ord, cand) or sentinel
__device__ __forceinline__ uint64_t swap_halves(uint64_t e) {
  return (e == ~0ull) ? e : ((e << 32) | (e >> 32));
}

// Sorts by (cand, key) and drops duplicate cands (keeping the smallest key,
// a held key before a deferred one) and the self id, within segments of W
// lanes; returns the kept (cand, key order) elements, SENT elsewhere.
template <int W>
__device__ __forceinline__ uint64_t seg_dedupe(uint64_t e, uint32_t self, int lane) {
  const uint64_t SENT = ~0ull;
  e = seg_sort_u64<W>(e, lane);
  const uint64_t pv = lane_up1_u64(e);
  const uint32_t cd = (uint32_t)(e >> 32);
  const bool first = (lane & (W - 1)) == 0;
  const bool keep = e != SENT && cd != self && (first || (uint32_t)(pv >> 32) != cd);
  return keep ? e : SENT;
}

// seg_dedupe and a sort by (key, cand), for inputs in which equal cands carry
// equal keys (and no key is deferred): one sort
// by (key, cand) puts the repeats of a cand next to each other, so dropping
// every element equal to its left neighbour deduplicates; the kept elements
// then move to the front of the segment, in order, by one forward permute
// (kept element -> its rank among the kept, dropped ones -> the lanes after
// them: a bijection of the segment's lanes).
template <int W>
__device__ __forceinline__ uint64_t seg_sort_canon(uint64_t e, uint32_t self, int lane) {
  constexpr uint64_t SENT = ~0ull;
  constexpr uint64_t kSeg = W == 64 ? ~0ull : ((1ull << W) - 1ull);
  e = seg_sort_u64<W>(swap_halves(e), lane);  // (key, cand)
  const uint64_t pv = lane_up1_u64(e);
  const uint32_t cd = (uint32_t)e;
  const int i = lane & (W - 1), base = lane & ~(W - 1);
  const bool keep = e != SENT && cd != self && (i == 0 || pv != e);
  const uint64_t seg = (ballot(keep) >> base) & kSeg;
  const int pos = __popcll(seg & ((1ull << i) - 1ull)), cnt = __popcll(seg);
  const int dst = base + (keep ? pos : cnt + (i - pos));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(4 * dst, (int)(uint32_t)e);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(4 * dst, (int)(uint32_t)(e >> 32));
  return i < cnt ? (((uint64_t)hi << 32) | lo) : SENT;
}
}  // namespace

namespace {
// Orders one wave's LDS accesses (the merge's blocks hold several waves that
// take different numbers of tasks, so a block barrier cannot be used).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS of a merge task's deferred keys: up to kWave x kMaxDefer
// (destination, candidate) pairs and their keys.
constexpr int kMaxDefer = 4;
// Pairs per 16-lane group per memory round trip of the deferred keys.
constexpr int kDeferOps = 1;
struct DeferLds {
  int pair[2 * kWave * kMaxDefer];
  float key[kWave * kMaxDefer];
};

// Gives every deferred element of e (a kept merge element (cand, order)
// whose order is kOrdDeferred) its key: the canonical distance between its
// destination dst[m] and its candidate. The wave's deferred elements are
// listed in LDS and computed 16 pairs per memory round trip (op k, lane
// group lk: pair b + 4 k + lk); the destination's row is the same for all of
// its items, so after the first pair it is read from the caches.
template <int METRIC, int M>
__device__ __forceinline__ void resolve_deferred(const MergeArgs& A, uint64_t (&e)[M],
                                                 const int64_t (&dst)[M], int lane, DeferLds& S,
                                                 unsigned long long& ndef) {
  static_assert(M <= kMaxDefer, "LDS holds kMaxDefer elements per lane");
  constexpr uint64_t SENT = ~0ull;
  bool df[M];
  int rank[M];
  int tot = 0;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    df[m] = e[m] != SENT && (uint32_t)e[m] == kOrdDeferred;
    const uint64_t dm = ballot(df[m]);
    rank[m] = tot + __popcll(dm & lanemask_lt(lane));
    tot += __popcll(dm);
  }
  if (tot == 0) return;
  ndef += (unsigned long long)tot;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (df[m]) {
      S.pair[2 * rank[m]] = (int)dst[m];
      S.pair[2 * rank[m] + 1] = (int)(uint32_t)(e[m] >> 32);
    }
  }
  wave_lds_sync();
  const int li = lane & 15, lk = lane >> 4;
  for (int b = 0; b < tot; b += 4 * kDeferOps) {
    constexpr int NOP = kDeferOps;
    int ia[NOP], ib[NOP];
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
      const int r = min(b + 4 * k + lk, tot - 1);
      ia[k] = S.pair[2 * r];
      ib[k] = S.pair[2 * r + 1];
    }
    float dd[NOP];
    dist16_batch<METRIC, NOP>(A.X, A.ld, A.d4, ia, ib, li, dd);
    if (li == 0) {
#pragma unroll
      for (int k = 0; k < NOP; ++k)
        if (b + 4 * k + lk < tot) S.key[b + 4 * k + lk] = dd[k];
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (df[m]) e[m] = (e[m] & 0xFFFFFFFF00000000ull) | key_to_ord(S.key[rank[m]]);
  }
  // the list is rewritten by the wave's next task
  wave_lds_sync();
}

// Element j of destination x's merge input: its a kept items, then the f
// items other vertices sent it (bucket first, then its overflow range at b).
__device__ __forceinline__ uint64_t merge_elem(const MergeArgs& A, int64_t x, uint32_t a,
                                               uint32_t f, uint32_t b, uint32_t j) {
  if (j < a) return cand_ord(A.items.own[x * A.R + j]);
  j -= a;
  if (j >= f) return ~0ull;
  const uint32_t bcap = (uint32_t)A.items.bcap;
  if (j < bcap) return cand_ord(A.items.bkt[x * bcap + j]);
  return cand_ord(A.seg[b + (j - bcap)]);
}

__device__ __forceinline__ uint32_t pool_class(int k) { return k <= 16 ? 0u : (k <= 32 ? 1u : 2u); }

// Writes destination x's new pool row from its W-lane segment (entry i of the
// sorted, deduplicated input in lane i of the segment) and its pool class
// (k_alloc has cleared its item counter).
template <int W>
__device__ __forceinline__ void merge_store(const MergeArgs& A, int64_t x, uint64_t best, int lane) {
  constexpr uint64_t kSeg = W == 64 ? ~0ull : ((1ull << W) - 1ull);
  const int i = lane & (W - 1);
  const bool ok = best != ~0ull;
  const uint64_t okm = ballot(ok && i < A.R);
  const int64_t o = x * A.R;
  for (int sl = i; sl < A.R; sl += W) {
    const bool v = sl == i && ok;
    A.out_ids[o + sl] = v ? (int32_t)(uint32_t)best : -1;
    A.out_keys[o + sl] = v ? ord_to_key((uint32_t)(best >> 32)) : INFINITY;
  }
  if (i == 0) {
    A.pool_cls[x] = (uint8_t)pool_class(__popcll((okm >> (lane & ~(W - 1))) & kSeg));
  }
}

// Destinations first .. first + NT (64/W) - 1 of merge list c (inputs of
// at most W items), one per W-lane segment, in NT independent parts whose
// loads and sorting networks interleave (each hides the others' latency).
template <int W, int NT, bool CANON, int METRIC, bool DEFER>
__device__ __forceinline__ void merge_group(const MergeArgs& A, int c, uint32_t count,
                                            uint32_t first, int lane, unsigned long long& items,
                                            DeferLds& S, unsigned long long& ndef) {
  constexpr uint32_t NS = kWave / W;
  const uint32_t i = (uint32_t)(lane & (W - 1));
  uint4 h[NT];
  bool has[NT];
  uint64_t v[NT];
#pragma unroll
  for (int p = 0; p < NT; ++p) {
    const uint32_t idx = first + (uint32_t)(lane / W) + NS * (uint32_t)p;
    has[p] = idx < count;
    h[p] = has[p] ? A.mlist[(int64_t)c * A.n + idx] : make_uint4(0u, 0u, 0u, 0u);
  }
  int64_t dst[NT];
#pragma unroll
  for (int p = 0; p < NT; ++p) {
    v[p] = has[p] ? merge_elem(A, (int64_t)h[p].x, h[p].y, h[p].z, h[p].w, i) : ~0ull;
    dst[p] = (int64_t)h[p].x;
    items += (unsigned long long)__popcll(ballot(v[p] != ~0ull));
  }
  bool anydef = false;
  if constexpr (DEFER) {
#pragma unroll
    for (int p = 0; p < NT; ++p)
      anydef = anydef || (v[p] != ~0ull && (uint32_t)v[p] == kOrdDeferred);
  }
  if (CANON && (!DEFER || ballot(anydef) == 0ull)) {
#pragma unroll
    for (int p = 0; p < NT; ++p) v[p] = seg_sort_canon<W>(v[p], h[p].x, lane);
  } else {
    // deduplicate by candidate first, so that only candidates the
    // destination does not already hold have their deferred keys computed
#pragma unroll
    for (int p = 0; p < NT; ++p) v[p] = seg_dedupe<W>(v[p], h[p].x, lane);
    if constexpr (DEFER) resolve_deferred<METRIC, NT>(A, v, dst, lane, S, ndef);
#pragma unroll
    for (int p = 0; p < NT; ++p) v[p] = seg_sort_u64<W>(swap_halves(v[p]), lane);
  }
#pragma unroll
  for (int p = 0; p < NT; ++p)
    if (has[p]) merge_store<W>(A, (int64_t)h[p].x, v[p], lane);
}

// One destination with more than 64 input items: 128-element chunks, each
// sorted together with the running top R.
template <int METRIC, bool DEFER>
__device__ __forceinline__ void merge_long(const MergeArgs& A, uint4 h, int lane,
                                           unsigned long long& items, DeferLds& S,
                                           unsigned long long& ndef) {
  const uint64_t SENT = ~0ull;
  const int64_t x = (int64_t)h.x;
  const uint32_t a = h.y, f = h.z, b = h.w;
  const uint32_t m = a + f;
  uint64_t best = SENT;
  const int chunk = 2 * kWave - A.R;
  for (uint32_t p0 = 0; p0 < m; p0 += (uint32_t)chunk) {
    uint64_t e0 = SENT, e1 = SENT, n0 = SENT;
    if (lane < A.R) {
      e0 = swap_halves(best);
    } else {
      const uint32_t i0 = p0 + (uint32_t)(lane - A.R);
      if (i0 < m) n0 = e0 = merge_elem(A, x, a, f, b, i0);
    }
    const uint32_t i1 = p0 + (uint32_t)(kWave - A.R + lane);
    if (i1 < m) e1 = merge_elem(A, x, a, f, b, i1);
    items += (unsigned long long)(__popcll(ballot(n0 != SENT)) + __popcll(ballot(e1 != SENT)));
    wave_sort128(e0, e1, lane);
    const uint64_t p0v = lane_up1_u64(e0);
    const uint64_t p1v = lane_up1_u64(e1);
    const uint64_t last0 = __shfl((unsigned long long)e0, 63);
    const uint64_t pr1 = (lane == 0) ? last0 : p1v;
    const uint32_t c0 = (uint32_t)(e0 >> 32), c1 = (uint32_t)(e1 >> 32);
    const uint32_t xs = (uint32_t)x;
    const bool k0 = e0 != SENT && c0 != xs && (lane == 0 || (uint32_t)(p0v >> 32) != c0);
    const bool k1 = e1 != SENT && c1 != xs && (uint32_t)(pr1 >> 32) != c1;
    uint64_t ee[2] = {k0 ? e0 : SENT, k1 ? e1 : SENT};
    const int64_t dd[2] = {x, x};
    if constexpr (DEFER) resolve_deferred<METRIC, 2>(A, ee, dd, lane, S, ndef);
    uint64_t f0 = swap_halves(ee[0]), f1 = swap_halves(ee[1]);
    wave_sort128(f0, f1, lane);
    best = (lane < A.R) ? f0 : SENT;
  }
  merge_store<kWave>(A, x, best, lane);
}
}  // namespace

// Write pool (Alg. 6 taken to completion): the first R by (key, id) of the
// items sent to a vertex, one per id (smallest key), self dropped. Each wave
// takes tasks from the four merge lists in turn: 4 kMergeParts destinations
// of at most 16 input items (16-lane segments), 2 kMergeParts of at most 32,
// kMergeParts of at most 64, or one larger destination (128-element chunks
// with a running top R). The
// class of every new pool is recorded for the next round's classification.
// CANON (equal cands carry equal keys, as in every merge of a build, whose
// keys are all the symmetric canonical distance of their pair) lets the
// segments deduplicate after a single sort by (key, id).
// Independent parts of one merge task (interleaved to hide each other's
// latency).
constexpr uint32_t kMergeParts = 4;
// fewer with deferred keys, whose distance loads need the registers
constexpr uint32_t kMergePartsDefer = 2;

template <bool CANON, int METRIC, bool DEFER>
__global__ __launch_bounds__(256) void k_merge(const MergeArgs A) {
  // LDS for the deferred keys only where the round left any
  __shared__ DeferLds defer_lds[DEFER ? 4 : 1];
  DeferLds& S = defer_lds[DEFER ? (threadIdx.x >> 6) : 0];
  const int lane = threadIdx.x & 63;
  const uint32_t c0 = A.cursor[5], c1 = A.cursor[6], c2 = A.cursor[7], c3 = A.cursor[8];
  constexpr uint32_t NT = DEFER ? kMergePartsDefer : kMergeParts;
  const uint32_t e0 = (c0 + 4u * NT - 1u) / (4u * NT), e1 = e0 + (c1 + 2u * NT - 1u) / (2u * NT),
                 e2 = e1 + (c2 + NT - 1u) / NT, e3 = e2 + c3;
  const uint32_t nw = gridDim.x * 4u;
  unsigned long long items = 0, ndef = 0;
  for (uint32_t task = blockIdx.x * 4u + (threadIdx.x >> 6); task < e3; task += nw) {
    if (task < e0)
      merge_group<16, NT, CANON, METRIC, DEFER>(A, 0, c0, 4u * NT * task, lane, items, S, ndef);
    else if (task < e1)
      merge_group<32, NT, CANON, METRIC, DEFER>(A, 1, c1, 2u * NT * (task - e0), lane, items, S, ndef);
    else if (task < e2)
      merge_group<kWave, NT, CANON, METRIC, DEFER>(A, 2, c2, NT * (task - e1), lane, items, S, ndef);
    else
      merge_long<METRIC, DEFER>(A, A.mlist[3 * A.n + (task - e2)], lane, items, S, ndef);
  }
  if (lane == 0) {
    stat_add(A.statp, (int)(blockIdx.x % kStatSlots), 4, items);
    if (DEFER) stat_add(A.statp, (int)(blockIdx.x % kStatSlots), 10, ndef);
  }
}

// Resets the allocation cursor and the vertex-list lengths after all merges of
// a round (stream ordered).
__global__ void k_reset_cursor(uint32_t* cursor) {
  if (threadIdx.x < kCursorWords) cursor[threadIdx.x] = 0u;
}

static_assert(GRNND_NSTATS <= kStatStride, "a stat slot holds every counter");

__global__ void k_stats_reduce(const unsigned long long* __restrict__ statp,
                               uint64_t* __restrict__ out) {
  const int i = threadIdx.x;
  if (i >= GRNND_NSTATS) return;
  unsigned long long s = 0;
  for (int k = 0; k < kStatSlots; ++k) s += statp[(size_t)k * kStatStride + i];
  out[i] += s;
}

// ------------------------------------------------------------ pool check
// Debugging aid: verifies that a pool is canonical (the form every call of
// the library writes). One wave per row v, lane j on entry j. Codes: 1 id
// outside [-1, n); 2 id == v; 3 a valid entry after padding, or padding
// whose key is not +inf; 4 an id twice; 5 valid entries not strictly
// ascending by (key, id); 6 a key that is not the canonical distance
// d(v, id). The smallest (v << 3 | code) over the pool is min-combined into
// *first_bad, which the caller has set to ~0.
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v) { *p = v; }

template <int METRIC>
__global__ __launch_bounds__(64) void k_check_pool(const float* __restrict__ X, int64_t ld,
                                                   int d4, int64_t n, int32_t R,
                                                   const int32_t* __restrict__ ids,
                                                   const float* __restrict__ keys,
                                                   unsigned long long* first_bad) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t v = blockIdx.x;
  const int64_t o = v * R;
  const bool in = lane < R;
  const int id = in ? ids[o + lane] : -1;
  const float key = in ? keys[o + lane] : INFINITY;
  const bool valid = in && id != -1;
  const bool ranged = valid && id >= 0 && (int64_t)id < n;  // safe to gather
  const uint64_t vm = ballot(valid);
  const uint64_t rm = ballot(ranged);
  uint32_t code = 0;
  if (in && (id < -1 || (int64_t)id >= n)) code = 1;
  else if (valid && (int64_t)id == v) code = 2;
  else if (in && !valid && ((vm >> lane) != 0 || !(__builtin_isinf(key) && key > 0.0f))) code = 3;
  bool dup = false;
  for (int l2 = 0; l2 < kWave; ++l2) {
    const int id2 = rl_i(id, l2);
    dup = dup || (l2 < lane && ((vm >> l2) & 1ull) && id2 == id);
  }
  if (code == 0 && valid && dup) code = 4;
  const uint64_t sk = ((uint64_t)key_to_ord(key) << 32) | (uint32_t)id;
  const uint64_t nx = ((uint64_t)__shfl((int)(uint32_t)(sk >> 32), (lane + 1) & 63) << 32) |
                      (uint32_t)__shfl(id, (lane + 1) & 63);
  if (code == 0 && valid && lane + 1 < R && ((vm >> (lane + 1)) & 1ull) && !(sk < nx)) code = 5;
  // canonical distances, 16 entries per pass (op k, lane group lk: entry b + 4 k + lk)
  for (int b = 0; b < R; b += 16) {
    constexpr int NOP = 4;
    int ia[NOP], ib[NOP];
    int e[NOP];
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
      e[k] = b + 4 * k + lk;
      const int ide = __shfl(id, e[k] & 63);
      ia[k] = (int)v;
      ib[k] = (e[k] < R && ((rm >> e[k]) & 1ull)) ? ide : (int)v;
    }
    float dd[NOP];
    dist16_batch<METRIC, NOP>(X, ld, d4, ia, ib, li, dd);
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
      const float ke = __shfl(key, e[k] & 63);
      if (li == 0 && code == 0 && e[k] < R && ((rm >> e[k]) & 1ull) &&
          __float_as_uint(ke) != __float_as_uint(dd[k]))
        code = 6;
    }
  }
  // lanes with li == 0 report entries of other lanes; fold every code to one
  uint64_t mine = code ? (((uint64_t)v << 3) | code) : ~0ull;
  for (int m = 1; m < kWave; m <<= 1) {
    const uint64_t y = shfl_xor_u64(mine, m);
    mine = y < mine ? y : mine;
  }
  if (lane == 0 && mine != ~0ull) atomicMin(first_bad, (unsigned long long)mine);
}

// ------------------------------------------------------- batched builds
__global__ __launch_bounds__(256) void k_seg_fill(const SegTable T, int64_t n, SegInfo* segs,
                                                 uint16_t* vseg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < T.count) segs[i] = T.seg[i];
  if (i >= n) return;
  int lo = 0, hi = T.count - 1;  // the last segment whose base is <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (T.seg[mid].base <= i) lo = mid; else hi = mid - 1;
  }
  vseg[i] = (uint16_t)lo;
}

// Row v of the batch to row v - base of its collection, ids made local.
__global__ __launch_bounds__(256) void k_seg_split(const int32_t* __restrict__ adj,
                                                  const float* __restrict__ keys, int64_t n,
                                                  int32_t R, const SegMap M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * R) return;
  const int64_t v = i / R;
  const SegInfo& sg = M.segs[M.vseg[v]];
  const int64_t o = (v - sg.base) * R + (i - v * R);
  const int32_t id = adj[i];
  sg.out_adj[o] = id >= 0 ? (int32_t)(id - sg.base) : -1;
  if (sg.out_keys) sg.out_keys[o] = keys[i];
}

// ----------------------------------------------------------------- launchers
hipError_t launch_seg_fill(const SegTable& t, int64_t n, SegInfo* segs, uint16_t* vseg,
                           hipStream_t s) {
  const int64_t m = n > t.count ? n : t.count;
  hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, t, n, segs,
                     vseg);
  return hipGetLastError();
}

hipError_t launch_seg_split(const int32_t* adj, const float* keys, int64_t n, int32_t R,
                            const SegMap& m, hipStream_t s) {
  const int64_t tot = n * R;
  hipLaunchKernelGGL(k_seg_split, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, adj, keys,
                     n, R, m);
  return hipGetLastError();
}

hipError_t launch_clear(uint32_t* cnt, int64_t n, uint32_t* cursor,
                        unsigned long long* statp, float* zero16, hipStream_t s) {
  const int64_t m = n > (int64_t)kStatSlots * kStatStride ? n : (int64_t)kStatSlots * kStatStride;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, cnt, n,
                     cursor, statp, zero16);
  return hipGetLastError();
}

hipError_t launch_pad_copy(const float* X, int64_t n, int32_t d, float* Xp, int32_t ldp,
                           hipStream_t s) {
  const int64_t tot = n * (int64_t)ldp;
  hipLaunchKernelGGL(k_pad_copy, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, n,
                     d, Xp, ldp);
  return hipGetLastError();
}

template <int METRIC, int NB>
static hipError_t launch_init_t(const InitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_init<METRIC, NB>), dim3((unsigned)a.n), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, int metric, hipStream_t s) {
  const int nb = (a.R + 15) / 16;
  if (metric == 0) {
    switch (nb) {
      case 1: return launch_init_t<0, 1>(a, s);
      case 2: return launch_init_t<0, 2>(a, s);
      case 3: return launch_init_t<0, 3>(a, s);
      default: return launch_init_t<0, 4>(a, s);
    }
  }
  switch (nb) {
    case 1: return launch_init_t<1, 1>(a, s);
    case 2: return launch_init_t<1, 2>(a, s);
    case 3: return launch_init_t<1, 3>(a, s);
    default: return launch_init_t<1, 4>(a, s);
  }
}

hipError_t launch_reverse(const ReverseArgs& a, hipStream_t s) {
  if (a.R <= 16)
    hipLaunchKernelGGL(k_reverse<16>, dim3((unsigned)((a.n + 3) / 4)), dim3(64), 0, s, a);
  else if (a.R <= 32)
    hipLaunchKernelGGL(k_reverse<32>, dim3((unsigned)((a.n + 1) / 2)), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_reverse<64>, dim3((unsigned)a.n), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_alloc, dim3((unsigned)((a.n + 1023) / 1024)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter, dim3(1024), dim3(256), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // about one task per wave (most destinations share a wave with others);
  // without deferred keys at most 8,192 blocks (32 waves per SIMD over the
  // launch, four times what a SIMD holds at once), each wave then taking
  // several tasks in turn: fewer wave launches, 2-4% faster merges at 10^6
  // destinations. The deferred-key merge, bound by its distance loads, keeps
  // one task per wave (the cap made it 2% slower).
  const int64_t nb = (a.n + 8 * kMergeParts - 1) / (8 * kMergeParts);
  const int64_t cap = a.deferred ? (int64_t)1 << 20 : 8192;
  const dim3 grid((unsigned)(nb < cap ? nb : cap));
  // the metric matters only to the deferred keys
  if (!a.deferred) {
    if (a.canon)
      hipLaunchKernelGGL((k_merge<true, 0, false>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_merge<false, 0, false>), grid, dim3(256), 0, s, a);
  } else if (a.metric == 0) {
    if (a.canon)
      hipLaunchKernelGGL((k_merge<true, 0, true>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_merge<false, 0, true>), grid, dim3(256), 0, s, a);
  } else {
    if (a.canon)
      hipLaunchKernelGGL((k_merge<true, 1, true>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_merge<false, 1, true>), grid, dim3(256), 0, s, a);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reset_cursor, dim3(1), dim3(64), 0, s, a.cursor);
  return hipGetLastError();
}

hipError_t launch_rowflags(const float* X, int64_t n, int32_t d, int32_t ld, uint8_t* rexact,
                           uint32_t* rsum, hipStream_t s) {
  hipLaunchKernelGGL(k_rowflags_init, dim3(1), dim3(1), 0, s, rsum);
  hipLaunchKernelGGL(k_rowflags, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, s, X, n, d, ld, rexact,
                     rsum);
  return hipGetLastError();
}

hipError_t launch_stats_reduce(const unsigned long long* statp, uint64_t* dev_stats,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(64), 0, s, statp, dev_stats);
  return hipGetLastError();
}

hipError_t launch_check_pool(const float* X, int64_t ld, int d4, int64_t n, int32_t R,
                             int32_t metric, const int32_t* ids, const float* keys,
                             unsigned long long* first_bad, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, first_bad, ~0ull);
  if (metric == 0)
    hipLaunchKernelGGL(k_check_pool<0>, dim3((unsigned)n), dim3(64), 0, s, X, ld, d4, n, R, ids,
                       keys, first_bad);
  else
    hipLaunchKernelGGL(k_check_pool<1>, dim3((unsigned)n), dim3(64), 0, s, X, ld, d4, n, R, ids,
                       keys, first_bad);
  return hipGetLastError();
}

}  // namespace grnnd
