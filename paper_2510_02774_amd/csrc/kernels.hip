// kernels.hip -- GRNND construction kernels for gfx950 (wave64, MFMA).
//
// One wave handles one vertex in the init, round, reverse and merge kernels.
// The round kernel is the hot path: it reads the vertex's pool row, orders
// the candidates (Section 3.3), gathers their rows into LDS, forms the
// candidate distance tile on the matrix cores, runs the prune scan of Eq. 2
// with wave ballots, and emits exactly one item per candidate for the merge
// that fills the write pool (Section 3.5).
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {

__device__ __forceinline__ float rl_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ int rl_i(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

__device__ __forceinline__ void stat_add(unsigned long long* statp, int slot, int idx,
                                         unsigned long long v) {
  if (v) atomicAdd(statp + (size_t)slot * kStatStride + idx, v);
}

// Gathers rows src_id[0..nrows) (ids read from LDS `ids`; row `nrows` is x_v
// when with_self) into LDS rows of stride rs, zero-filling the columns
// [d, round_up(d,16)). Loads are issued in batches of kBatch float4 per lane
// before any LDS store, so every wave keeps many row loads in flight.
template <int kBatch>
__device__ __forceinline__ void gather_rows(const float* __restrict__ X, int64_t ld, int d4,
                                            const int* ids, int nrows, bool with_self,
                                            int64_t self_id, int self_slot, float* rows,
                                            int rs, int lane) {
  const int nr = nrows + (with_self ? 1 : 0);
  const int total = nr * d4;
  int r = lane / d4, c = lane % d4;
  const int sr = kWave / d4, sc = kWave % d4;
  for (int base = 0; base < total; base += kWave * kBatch) {
    float4 buf[kBatch];
    int dst[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int q = base + u * kWave + lane;
      dst[u] = -1;
      if (q < total) {
        const int64_t src = (r < nrows) ? (int64_t)ids[r] : self_id;
        buf[u] = *reinterpret_cast<const float4*>(X + src * ld + 4 * c);
        dst[u] = ((r < nrows) ? r : self_slot) * rs + 4 * c;
      }
      c += sc;
      r += sr;
      if (c >= d4) { c -= d4; ++r; }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (dst[u] >= 0) *reinterpret_cast<float4*>(rows + dst[u]) = buf[u];
  }
  // zero pad columns
  const int d16q = round_up(4 * d4, 16) / 4;
  const int padq = d16q - d4;
  if (padq > 0) {
    for (int q = lane; q < nr * padq; q += kWave) {
      const int rr = q / padq, cc = d4 + q % padq;
      const int slot = (rr < nrows) ? rr : self_slot;
      *reinterpret_cast<float4*>(rows + slot * rs + 4 * cc) = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

}  // namespace

// ------------------------------------------------------------------- clear
__global__ void k_clear(uint32_t* __restrict__ cnt, int64_t n, uint32_t* cursor,
                        unsigned long long* statp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = 0;
  if (i < (int64_t)kStatSlots * kStatStride && statp) statp[i] = 0ull;
  if (i == 0 && cursor) *cursor = 0u;
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
// INITIAL_NEIGHBORS (Alg. 3, lines 3-5): the first min(S, n-1) distinct ids
// != v of the hash stream h(seed, 0x3000, v, j) mod n, j = 0, 1, ..., with
// their keys, written as a pool row sorted by (key, id) and padded.
template <int METRIC, int NB>
__global__ __launch_bounds__(64) void k_init(const InitArgs A) {
  extern __shared__ __align__(16) float lds[];
  constexpr int KP = 16 * NB;
  const RoundLds L = round_lds(KP, 4 * A.d4);
  float* rows = lds + L.rows_off;
  int* coll = reinterpret_cast<int*>(lds + L.meta_off);
  uint64_t* m_sk = reinterpret_cast<uint64_t*>(lds + L.sk_off);
  const int lane = threadIdx.x;
  const int64_t v = blockIdx.x;
  const int want = (int)((int64_t)A.S < A.n - 1 ? (int64_t)A.S : A.n - 1);

  int got = 0;
  for (uint64_t j0 = 0; got < want; j0 += kWave) {
    const uint64_t h = hash4(A.seed, kTagInit, (uint64_t)v, j0 + (uint64_t)lane);
    const int c = (int)(h % (uint64_t)A.n);
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

  gather_rows<8>(A.X, A.ld, A.d4, coll, want, true, v, KP, rows, L.rs, lane);
  __syncthreads();

  float mykey = INFINITY;
  for (int q = 0; q < want; ++q) {
    const float dd = dist_canon<METRIC>(rows + KP * L.rs, rows + q * L.rs, A.d4, lane);
    if (lane == q) mykey = dd;
  }
  const int myid = lane < want ? coll[lane] : -1;
  const uint64_t sk =
      lane < want ? (((uint64_t)key_to_ord(mykey) << 32) | (uint32_t)myid) : ~0ull;
  m_sk[lane] = sk;
  __syncthreads();
  int rnk = 0;
  for (int j = 0; j < want; ++j) rnk += (m_sk[j] < sk) ? 1 : 0;
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

// ------------------------------------------------------------------- round
// One update round for one vertex (Alg. 4 with Eq. 2), or the output pass
// (FINAL: ascending order, strict Eq. 1 test, no redirection).
//
// Tile: the Gram matrix of the candidate rows, centred on x_v for L2, on the
// 16x16x4 FP32 matrix cores; D(i,j) = G_ii + G_jj - 2 G_ij (L2) or -G_ij
// (IP). A prune decision whose tile value lies within the tile's error bound
// of its threshold is re-evaluated with the canonical direct distance, and
// every emitted redirect key is a canonical direct distance, so stored keys
// never carry the Gram form's cancellation error.
template <int METRIC, int NB, bool FINAL>
__global__ __launch_bounds__(64) void k_round(const RoundArgs A) {
  extern __shared__ __align__(16) float lds[];
  constexpr int KP = 16 * NB;
  const RoundLds L = round_lds(KP, 4 * A.d4);
  float* rows = lds + L.rows_off;
  float* tile = lds + L.tile_off;
  float* gdiag = lds + L.g_off;
  int* m_id = reinterpret_cast<int*>(lds + L.meta_off);
  float* m_key = lds + L.meta_off + kWave;
  int* m_rk = reinterpret_cast<int*>(lds + L.meta_off + 2 * kWave);
  uint64_t* m_sk = reinterpret_cast<uint64_t*>(lds + L.sk_off);
  const int rs = L.rs, ts = L.ts;
  const int lane = threadIdx.x;
  const int64_t v = blockIdx.x;
  const int slot = (int)(blockIdx.x % kStatSlots);

  // ---- 1. read pool row, compacted to its valid entries (ids outside
  //         [0, n) are ignored). Canonical rows are already compact and
  //         sorted by (key, id), so a lane's compacted position is its rank
  //         in (key, id) order.
  int id0 = -1;
  float key0 = INFINITY;
  if (lane < A.R) {
    id0 = A.in_ids[v * A.R + lane];
    key0 = A.in_keys[v * A.R + lane];
  }
  const bool valid0 = id0 >= 0 && (int64_t)id0 < A.n;
  const uint64_t vm = ballot(valid0);
  const int K = __popcll(vm);
  if (valid0) {
    const int pos = __popcll(vm & lanemask_lt(lane));
    m_id[pos] = id0;
    m_key[pos] = key0;
  }
  __syncthreads();
  const bool valid = lane < K;
  const int id = valid ? m_id[lane] : -1;
  const float key = valid ? m_key[lane] : INFINITY;
  __syncthreads();

  if (K <= 1) {
    if (FINAL) {
      if (lane < A.R) {
        A.out_adj[v * A.R + lane] = id;
        if (A.out_keys) A.out_keys[v * A.R + lane] = key;
      }
    } else if (lane == 0) {
      A.nitem[v] = K;
      if (K == 1) {
        const int64_t o = v * A.cap;
        A.it_dest[o] = (int32_t)v;
        A.it_cand[o] = id;
        A.it_key[o] = key;
        atomicAdd(&A.cnt[v], 1u);
        stat_add(A.statp, slot, 3, 1);
        stat_add(A.statp, slot, 5, 1);
      }
    }
    return;
  }

  // ---- 2. arrival order (Section 3.3; ascending / descending for Section 4.3)
  int arr = lane;
  if (!FINAL) {
    if (A.order == 2) {
      arr = K - 1 - lane;
    } else if (A.order == 0) {
      const uint64_t sk =
          valid ? hash_order_key(hash4(A.seed, kTagUpdate + A.round, (uint64_t)v,
                                       (uint64_t)(uint32_t)id), id)
                : ~0ull;
      m_sk[lane] = sk;
      __syncthreads();
      int r = 0;
      for (int j = 0; j < K; ++j) r += (m_sk[j] < sk) ? 1 : 0;
      arr = r;
    }
  }
  if (valid) {
    m_id[arr] = id;
    m_key[arr] = key;
    m_rk[arr] = lane;  // rank in (key, id) order
  }
  __syncthreads();
  const int cid = (lane < K) ? m_id[lane] : -1;
  const float ckey = (lane < K) ? m_key[lane] : INFINITY;
  const int crk = (lane < K) ? m_rk[lane] : kWave;

  // ---- 3. gather candidate rows (and x_v for L2 centring) into LDS
  gather_rows<8>(A.X, A.ld, A.d4, m_id, K, METRIC == 0, v, KP, rows, rs, lane);
  __syncthreads();

  // ---- 4. Gram tile on the matrix cores (lower block triangle)
  const int nbk = (K + 15) >> 4;
  const int li = lane & 15, lk = lane >> 4;
  v4f acc[NB * (NB + 1) / 2];
#pragma unroll
  for (int b = 0; b < NB * (NB + 1) / 2; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
  const int d16 = round_up(4 * A.d4, 16);
  for (int s = 0; s < d16; s += 16) {
    const int col = s + 4 * lk;
    float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (METRIC == 0) xv = *reinterpret_cast<const float4*>(rows + KP * rs + col);
    float4 a[NB];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      if (I < nbk) {
        const float4 t = *reinterpret_cast<const float4*>(rows + (16 * I + li) * rs + col);
        a[I] = (METRIC == 0) ? make_float4(t.x - xv.x, t.y - xv.y, t.z - xv.z, t.w - xv.w) : t;
      }
    }
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      if (I < nbk) {
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          v4f c = acc[I * (I + 1) / 2 + J];
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[I].x, a[J].x, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[I].y, a[J].y, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[I].z, a[J].z, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[I].w, a[J].w, c, 0, 0, 0);
          acc[I * (I + 1) / 2 + J] = c;
        }
      }
    }
  }
  // accumulator layout: lane l, register r -> block row 4*(l/16)+r, column l%16
#pragma unroll
  for (int I = 0; I < NB; ++I) {
    if (I < nbk) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (4 * lk + r == li) gdiag[16 * I + li] = acc[I * (I + 1) / 2 + I][r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int I = 0; I < NB; ++I) {
    if (I < nbk) {
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int j = 16 * J + li;
        const float gj = gdiag[j];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + 4 * lk + r;
          const float G = acc[I * (I + 1) / 2 + J][r];
          const float Dv = (METRIC == 0) ? (gdiag[i] + gj) - 2.0f * G : -G;
          tile[j * ts + i] = Dv;  // pair (i, j), i >= j, read by lane j at step i
        }
      }
    }
  }
  const float cg = (lane < K) ? A.mcoef * fabsf(gdiag[lane]) : 0.0f;
  __syncthreads();

  // ---- 5. prune scan (Eq. 2): candidate t meets every alive w < t in order
  uint64_t alive = 1ull;
  int partner = -1;
  unsigned nrecheck = 0;
  for (int t = 1; t < K; ++t) {
    const float kt = rl_f(ckey, t);
    const int rkt = rl_i(crk, t);
    const float cgt = rl_f(cg, t);
    const bool inA = (alive >> lane) & 1ull;
    const float Dtw = inA ? tile[lane * ts + t] : 0.0f;
    const float thr = fmaxf(kt, ckey);
    bool cond = inA && (Dtw < thr);
    const bool near = inA && (fabsf(Dtw - thr) <= cgt + cg);
    uint64_t nm = ballot(near);
    while (nm) {
      const int w = __ffsll((long long)nm) - 1;
      nm &= nm - 1;
      const float dd = dist_canon<METRIC>(rows + t * rs, rows + w * rs, A.d4, lane);
      if (lane == w) cond = dd < thr;
      ++nrecheck;
    }
    const uint64_t hit = ballot(cond);
    const uint64_t ufar = ballot(cond && crk < rkt);  // a closer alive w: t is the far one
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

  if (FINAL) {
    const bool isal = (alive >> lane) & 1ull;
    const int na = __popcll(alive);
    const int pos = __popcll(alive & lanemask_lt(lane));
    const int64_t o = v * A.R;
    if (isal) {
      A.out_adj[o + pos] = cid;
      if (A.out_keys) A.out_keys[o + pos] = ckey;
    }
    if (lane >= na && lane < A.R) {  // padding; slots >= na are never written above
      A.out_adj[o + lane] = -1;
      if (A.out_keys) A.out_keys[o + lane] = INFINITY;
    }
    if (lane == 0) {
      stat_add(A.statp, slot, 7, (unsigned long long)K * (K - 1) / 2);
      stat_add(A.statp, slot, 1, nrecheck);
    }
    return;
  }

  // ---- 6. emit one item per candidate (survivor -> v, redirected -> partner)
  const bool isdead = lane < K && !((alive >> lane) & 1ull);
  uint64_t dm = ballot(isdead);
  const int nred = __popcll(dm);
  float ikey = ckey;
  while (dm) {
    const int w = __ffsll((long long)dm) - 1;
    dm &= dm - 1;
    const int p = rl_i(partner, w);
    const float dd = dist_canon<METRIC>(rows + w * rs, rows + p * rs, A.d4, lane);
    if (lane == w) ikey = dd;
  }
  const int idest = isdead ? m_id[partner] : (int)v;
  if (lane < K) {
    const int64_t o = v * A.cap + lane;
    A.it_dest[o] = idest;
    A.it_cand[o] = cid;
    A.it_key[o] = ikey;
    if (isdead) atomicAdd(&A.cnt[idest], 1u);
  }
  if (lane == 0) {
    A.nitem[v] = K;
    atomicAdd(&A.cnt[v], (uint32_t)(K - nred));
    stat_add(A.statp, slot, 0, (unsigned long long)K * (K - 1) / 2);
    stat_add(A.statp, slot, 1, nrecheck);
    stat_add(A.statp, slot, 2, (unsigned long long)nred);
    stat_add(A.statp, slot, 3, (unsigned long long)(K - nred));
    stat_add(A.statp, slot, 5, (unsigned long long)K);
  }
}

// ----------------------------------------------------------------- reverse
// REVERSE_EDGE_SAMPLING (Section 3.6): v sends itself to the floor(rho * k)
// entries of its row that come first in hash order, and re-sends its whole
// row to itself; the merge then fills the write pool as in a round.
__global__ __launch_bounds__(64) void k_reverse(const ReverseArgs A) {
  __shared__ uint64_t m_sk[kWave];
  __shared__ int m_id[kWave];
  __shared__ float m_key[kWave];
  const int lane = threadIdx.x;
  const int64_t v = blockIdx.x;
  int id0 = -1;
  float key0 = INFINITY;
  if (lane < A.R) {
    id0 = A.in_ids[v * A.R + lane];
    key0 = A.in_keys[v * A.R + lane];
  }
  const bool valid0 = id0 >= 0 && (int64_t)id0 < A.n;
  const uint64_t vm = ballot(valid0);
  const int K = __popcll(vm);
  if (valid0) {
    const int pos = __popcll(vm & lanemask_lt(lane));
    m_id[pos] = id0;
    m_key[pos] = key0;
  }
  __syncthreads();
  const bool valid = lane < K;
  const int id = valid ? m_id[lane] : -1;
  const float key = valid ? m_key[lane] : INFINITY;
  const int m = A.mtab[K];
  const uint64_t sk =
      valid ? hash_order_key(hash4(A.seed, kTagReverse + A.t1, (uint64_t)v,
                                   (uint64_t)(uint32_t)id), id)
            : ~0ull;
  m_sk[lane] = sk;
  __syncthreads();
  int rnk = 0;
  for (int j = 0; j < K; ++j) rnk += (m_sk[j] < sk) ? 1 : 0;
  const int64_t o = v * A.cap;
  if (valid) {
    A.it_dest[o + lane] = (int32_t)v;
    A.it_cand[o + lane] = id;
    A.it_key[o + lane] = key;
    if (rnk < m) {
      A.it_dest[o + K + rnk] = id;
      A.it_cand[o + K + rnk] = (int32_t)v;
      A.it_key[o + K + rnk] = key;
      atomicAdd(&A.cnt[id], 1u);
    }
  }
  if (lane == 0) {
    A.nitem[v] = K + m;
    if (K) atomicAdd(&A.cnt[v], (uint32_t)K);
  }
}

// ------------------------------------------------------------------- merge
// Segment allocation: each destination gets a contiguous range of the
// staging buffer. Placement order is irrelevant: the merge result depends
// only on the multiset of items per destination.
__global__ __launch_bounds__(256) void k_alloc(const MergeArgs A) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const uint32_t c = (x < A.n) ? A.cnt[x] : 0u;
  uint32_t s = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(s, o);
    if (lane >= o) s += y;
  }
  const uint32_t tot = __shfl(s, 63);
  uint32_t base = 0;
  if (lane == 63 && tot) base = atomicAdd(A.cursor, tot);
  base = __shfl(base, 63);
  if (x < A.n) {
    A.off[x] = base + s - c;
    A.cnt[x] = 0u;
  }
}

// Moves every emitted item into its destination's segment.
__global__ __launch_bounds__(256) void k_scatter(const MergeArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < A.n; v += nw) {
    const int ni = A.nitem[v];
    for (int i = lane; i < ni; i += kWave) {
      const int64_t o = v * A.cap + i;
      const int dst = A.it_dest[o];
      const uint32_t pos = A.off[dst] + atomicAdd(&A.cnt[dst], 1u);
      A.seg[pos] = make_uint2((uint32_t)A.it_cand[o], __float_as_uint(A.it_key[o]));
    }
  }
}

namespace {
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
        const uint64_t y0 = shfl_xor_u64(e0, j), y1 = shfl_xor_u64(e1, j);
        const bool lower = (lane & j) == 0;
        const bool up0 = (lane & k) == 0, up1 = ((kWave + lane) & k) == 0;
        e0 = (lower == up0) ? (e0 < y0 ? e0 : y0) : (e0 < y0 ? y0 : e0);
        e1 = (lower == up1) ? (e1 < y1 ? e1 : y1) : (e1 < y1 ? y1 : e1);
      }
    }
  }
}

__device__ __forceinline__ uint64_t cand_ord(uint2 it) {
  return ((uint64_t)it.x << 32) | key_to_ord(__uint_as_float(it.y));
}
// (cand, ord) -> (ord, cand) or sentinel
__device__ __forceinline__ uint64_t swap_halves(uint64_t e) {
  return (e == ~0ull) ? e : ((e << 32) | (e >> 32));
}
}  // namespace

// Write pool of x (Alg. 6 taken to completion): the first R by (key, id) of
// the items sent to x, one per id (smallest key), self dropped.
__global__ __launch_bounds__(256) void k_merge(const MergeArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t x = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= A.n) return;
  const uint32_t m = A.cnt[x];
  const uint32_t b = A.off[x];
  const uint64_t SENT = ~0ull;
  const uint32_t xs = (uint32_t)x;
  uint64_t best = SENT;
  if (m <= (uint32_t)kWave) {
    uint64_t e = (lane < (int)m) ? cand_ord(A.seg[b + lane]) : SENT;
    e = wave_sort_u64(e, lane);
    const uint64_t pv = __shfl_up((unsigned long long)e, 1);
    const uint32_t cd = (uint32_t)(e >> 32);
    const bool keep = e != SENT && cd != xs && (lane == 0 || (uint32_t)(pv >> 32) != cd);
    best = wave_sort_u64(keep ? swap_halves(e) : SENT, lane);
  } else {
    const int chunk = 2 * kWave - A.R;
    for (uint32_t p0 = 0; p0 < m; p0 += (uint32_t)chunk) {
      uint64_t e0 = SENT, e1 = SENT;
      if (lane < A.R) {
        e0 = swap_halves(best);
      } else {
        const uint32_t i0 = p0 + (uint32_t)(lane - A.R);
        if (i0 < m) e0 = cand_ord(A.seg[b + i0]);
      }
      const uint32_t i1 = p0 + (uint32_t)(kWave - A.R + lane);
      if (i1 < m && i1 < p0 + (uint32_t)chunk) e1 = cand_ord(A.seg[b + i1]);
      wave_sort128(e0, e1, lane);
      const uint64_t p0v = __shfl_up((unsigned long long)e0, 1);
      const uint64_t p1v = __shfl_up((unsigned long long)e1, 1);
      const uint64_t last0 = __shfl((unsigned long long)e0, 63);
      const uint64_t pr1 = (lane == 0) ? last0 : p1v;
      const uint32_t c0 = (uint32_t)(e0 >> 32), c1 = (uint32_t)(e1 >> 32);
      const bool k0 = e0 != SENT && c0 != xs && (lane == 0 || (uint32_t)(p0v >> 32) != c0);
      const bool k1 = e1 != SENT && c1 != xs && (uint32_t)(pr1 >> 32) != c1;
      uint64_t f0 = k0 ? swap_halves(e0) : SENT, f1 = k1 ? swap_halves(e1) : SENT;
      wave_sort128(f0, f1, lane);
      best = (lane < A.R) ? f0 : SENT;
    }
  }
  if (lane < A.R) {
    const int64_t o = x * A.R + lane;
    if (best != SENT) {
      A.out_ids[o] = (int32_t)(uint32_t)best;
      A.out_keys[o] = ord_to_key((uint32_t)(best >> 32));
    } else {
      A.out_ids[o] = -1;
      A.out_keys[o] = INFINITY;
    }
  }
  if (lane == 0) {
    A.cnt[x] = 0u;
    stat_add(A.statp, (int)(blockIdx.x % kStatSlots), 4, m);
  }
}

// Resets the allocation cursor after all merges of a round (stream ordered).
__global__ void k_reset_cursor(uint32_t* cursor) { *cursor = 0u; }

__global__ void k_stats_reduce(const unsigned long long* __restrict__ statp,
                               uint64_t* __restrict__ out) {
  const int i = threadIdx.x;  // 8 counters
  if (i >= 8) return;
  unsigned long long s = 0;
  for (int k = 0; k < kStatSlots; ++k) s += statp[(size_t)k * kStatStride + i];
  out[i] += s;
}

// ----------------------------------------------------------------- launchers
size_t round_lds_bytes(int R, int d) {
  const int nb = (R + 15) / 16;
  return (size_t)round_lds(16 * nb, d).total * sizeof(float);
}

static hipError_t set_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_clear(uint32_t* cnt, int64_t n, uint32_t* cursor,
                        unsigned long long* statp, hipStream_t s) {
  const int64_t m = n > (int64_t)kStatSlots * kStatStride ? n : (int64_t)kStatSlots * kStatStride;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, cnt, n,
                     cursor, statp);
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
  const size_t lds = (size_t)round_lds(16 * NB, 4 * a.d4).total * sizeof(float);
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_init<METRIC, NB>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_init<METRIC, NB>), dim3((unsigned)a.n), dim3(64), lds, s, a);
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

template <int METRIC, int NB, bool FINAL>
static hipError_t launch_round_t(const RoundArgs& a, hipStream_t s) {
  const size_t lds = (size_t)round_lds(16 * NB, 4 * a.d4).total * sizeof(float);
  hipError_t e = set_lds(reinterpret_cast<const void*>(&k_round<METRIC, NB, FINAL>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_round<METRIC, NB, FINAL>), dim3((unsigned)a.n), dim3(64), lds, s, a);
  return hipGetLastError();
}

template <int METRIC, bool FINAL>
static hipError_t launch_round_m(const RoundArgs& a, hipStream_t s) {
  switch ((a.R + 15) / 16) {
    case 1: return launch_round_t<METRIC, 1, FINAL>(a, s);
    case 2: return launch_round_t<METRIC, 2, FINAL>(a, s);
    case 3: return launch_round_t<METRIC, 3, FINAL>(a, s);
    default: return launch_round_t<METRIC, 4, FINAL>(a, s);
  }
}

hipError_t launch_round(const RoundArgs& a, int metric, bool final_pass, hipStream_t s) {
  if (metric == 0)
    return final_pass ? launch_round_m<0, true>(a, s) : launch_round_m<0, false>(a, s);
  return final_pass ? launch_round_m<1, true>(a, s) : launch_round_m<1, false>(a, s);
}

hipError_t launch_reverse(const ReverseArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_reverse, dim3((unsigned)a.n), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_alloc, dim3(nb), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t sg = (a.n + 3) / 4;
  const unsigned gs = (unsigned)(sg < 65536 * 4 ? sg : 65536 * 4);
  hipLaunchKernelGGL(k_scatter, dim3(gs), dim3(256), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_merge, dim3((unsigned)((a.n + 3) / 4)), dim3(256), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reset_cursor, dim3(1), dim3(1), 0, s, a.cursor);
  return hipGetLastError();
}

hipError_t launch_stats_reduce(const unsigned long long* statp, uint64_t* dev_stats,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(64), 0, s, statp, dev_stats);
  return hipGetLastError();
}

}  // namespace grnnd
