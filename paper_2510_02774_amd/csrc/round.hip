// round.hip -- update round and output pass, the hot path (gfx950, wave64).
//
// A classification pass splits the vertices by pool shape. Pools that are
// compact (valid entries first) with at most 16 candidates -- most of them
// after the first round -- go to the small-pool kernel, which handles four
// vertices per wave, one per 16-lane row; every other pool goes to the
// general kernel, one vertex per wave (up to 64 candidates). Both kernels walk
// their vertex list with a grid stride. For a vertex they
//   1. read the pool row (K candidates, sorted by (key, id));
//   2. load the candidate rows straight into registers in the operand
//      layout of the 16x16x4 FP32 matrix instruction (lane l holds row
//      16 I + l % 16, float4 group 4 s + l / 16), while they compute the
//      candidates' arrival order (Section 3.3);
//   3. form the Gram tile of the candidates on the matrix cores, in pool
//      order, and turn it into a symmetric distance tile in LDS
//      (D = G_ii + G_jj - 2 G_ij for L2, -G_ij for IP); a decision within the
//      tile's rigorous error bound of its threshold is re-decided exactly;
//   4. run the prune scan of Eq. 2 in arrival order with wave ballots;
//   5. compute every redirect key with the canonical distance on the rows in
//      global memory (just read, so mostly served from cache; up to 16 pairs
//      per memory round trip), and emit one item per candidate (Alg. 4), or,
//      for the output pass, write the kept row.
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {

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
// arrival->pool permutation (64 each), the distance tile (kp x ts, ts =
// kp + 4, row j holds D(i, j) at column i, both triangles), Gram diagonal.
struct Round3Lds {
  int ts, pid_off, pkey_off, perm_off, tile_off, g_off, total;
};

__host__ __device__ inline Round3Lds round3_lds(int kp) {
  Round3Lds L;
  L.ts = kp + 4;
  L.pid_off = 0;
  L.pkey_off = kWave;
  L.perm_off = 2 * kWave;
  L.tile_off = 3 * kWave;
  L.g_off = L.tile_off + kp * L.ts;
  L.total = L.g_off + kp;
  return L;
}

// Per-wave LDS of the small-pool kernel (floats): ids, keys, permutation (64
// each, row g of the wave at [16 g, 16 g + 16)), four 16 x 20 distance tiles,
// Gram diagonals (64).
constexpr int kSmallTs = 20;
constexpr int kSmallTile = 16 * kSmallTs;
constexpr int kSmallLdsFloats = 3 * kWave + 4 * kSmallTile + kWave;

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

// Canonical redirect keys d(cid, pid) of the lanes in dm (up to 16 pairs per
// memory round trip); each such lane receives its key in ikey.
template <int METRIC>
__device__ __forceinline__ void redirect_keys(const float* X, int64_t ld, int d4, uint64_t dm,
                                              int cid, int pid, int lane, float& ikey) {
  const int li = lane & 15, lk = lane >> 4;
  while (dm) {
    constexpr int NOP = 4;
    int w[NOP][4], ia[NOP], ib[NOP];
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        w[k][g] = dm ? __ffsll((long long)dm) - 1 : -1;
        if (dm) dm &= dm - 1;
      }
      int wa = w[k][0];
#pragma unroll
      for (int g = 1; g < 4; ++g)
        if (lk == g && w[k][g] >= 0) wa = w[k][g];
      if (wa < 0) wa = 0;
      ia[k] = __shfl(cid, wa);
      ib[k] = __shfl(pid, wa);
    }
    float dd[NOP];
    dist16_batch<METRIC, NOP>(X, ld, d4, ia, ib, li, dd);
#pragma unroll
    for (int k = 0; k < NOP; ++k) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if (w[k][g] >= 0) {
          const float dg = rl_f(dd[k], 16 * g);
          if (lane == w[k][g]) ikey = dg;
        }
      }
    }
  }
}

// Gram tile of the first NBK 16-row blocks of the pool (rows past K repeat
// row 0) on the 16x16x4 FP32 matrix cores, then the symmetric distance tile
// in LDS: D(i, j) = G_ii + G_jj - 2 G_ij (L2) or -G_ij (IP); row j of the tile
// holds D(i, j) at column i, and gdiag receives G_ii. Every block runs the
// same number of chained steps (out-of-range float4 groups load as zeros), so
// the chains carry no branches. Lane l supplies row 16 I + l % 16, float4
// group 4 s + l / 16 of a step; the accumulator of block (I, J) holds
// G(16 I + 4 (l / 16) + r, 16 J + l % 16) in register r.
template <int METRIC, int NBK, class F>
__device__ __forceinline__ void gram_tile(const float* __restrict__ X, int64_t ld, int d4,
                                          const int* m_pid, int K, float* tile, float* gdiag,
                                          int ts, int li, int lk, F&& first) {
  constexpr int CH = NBK <= 2 ? 8 : 4;  // 16-float steps per load batch
  constexpr int NBL = NBK * (NBK + 1) / 2;
  const int nsteps = (d4 + 3) >> 2;
  int rid[NBK];
#pragma unroll
  for (int I = 0; I < NBK; ++I) {
    const int r = 16 * I + li;
    rid[I] = (r < K) ? m_pid[r] : m_pid[0];
  }
  v4f acc[NBL];
#pragma unroll
  for (int b = 0; b < NBL; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
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

// Gram and distance tiles of the four 16-row pools of a small-pool wave
// (pool q's ids at s_pid[16 q, 16 q + 16), absent entries standing as row 0).
// The four chains advance together two 16-float steps at a time, with the
// loads of the next two steps in flight while the current ones run on the
// matrix cores; out-of-range float4 groups load as zeros (chains stay
// branch-free). Tile q is written like gram_tile's, with stride kSmallTs.
template <int METRIC>
__device__ __forceinline__ void gram_small(const float* __restrict__ X, int64_t ld, int d4,
                                           const int* s_pid, float* tiles, float* gdiag, int li,
                                           int lk) {
  constexpr int CS = 2;
  const int nsteps = (d4 + 3) >> 2;
  int rid[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) rid[q] = s_pid[16 * q + li];
  v4f acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
  float4 a[4][CS], b[4][CS];
  auto load = [&](float4(&buf)[4][CS], int s0) {
#pragma unroll
    for (int c = 0; c < CS; ++c) {
      const int g = 4 * (s0 + c) + lk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        buf[q][c] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g < d4) buf[q][c] = *reinterpret_cast<const float4*>(X + (int64_t)rid[q] * ld + 4 * g);
      }
    }
  };
  auto chains = [&](const float4(&buf)[4][CS]) {
#pragma unroll
    for (int c = 0; c < CS; ++c) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v4f cc = acc[q];
        const float4 x = buf[q][c];
        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, x.x, cc, 0, 0, 0);
        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, x.y, cc, 0, 0, 0);
        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, x.z, cc, 0, 0, 0);
        cc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, x.w, cc, 0, 0, 0);
        acc[q] = cc;
      }
    }
  };
  load(a, 0);
  for (int s0 = 0; s0 < nsteps; s0 += 2 * CS) {
    load(b, s0 + CS);
    chains(a);
    load(a, s0 + 2 * CS);
    chains(b);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * lk + r == li) gdiag[16 * q + li] = acc[q][r];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float gi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) gi[r] = gdiag[16 * q + 4 * lk + r];
    const float gj = gdiag[16 * q + li];
    float Dv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) Dv[r] = (METRIC == 0) ? (gi[r] + gj) - 2.0f * acc[q][r] : -acc[q][r];
    *reinterpret_cast<float4*>(tiles + q * kSmallTile + li * kSmallTs + 4 * lk) =
        make_float4(Dv[0], Dv[1], Dv[2], Dv[3]);
  }
}

}  // namespace

// ------------------------------------------------------- general kernel
// One vertex per wave, any pool (holes allowed, up to 64 candidates).
template <int METRIC, int NB, bool FINAL>
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
        A.nitem[v] = K;
        if (K == 1) {
          const int64_t o = v * A.cap;
          A.it_dest[o] = (int32_t)v;
          A.it_cand[o] = id;
          A.it_key[o] = key;
          atomicAdd(&A.cnt[v], 1u);
        }
      }
      st.survivors += (unsigned)K;
      st.cands += (unsigned)K;
    }
    return;
  }

  m_pid[lane] = id;
  m_pkey[lane] = key;
  __syncthreads();

  // ---- 2-3. arrival order, Gram tile and distance tile of the active
  //           16-row blocks (a straight-line chain per block count)
  auto arrival = [&]() {  // Section 3.3, computed while the rows arrive
    int arr = lane;
    if (!FINAL) {
      if (A.order == 2) {
        arr = K - 1 - lane;
      } else if (A.order == 0) {
        const uint64_t sk =
            valid ? hash_order_key(hash4(A.seed, kTagUpdate + A.round, (uint64_t)v,
                                         (uint64_t)(uint32_t)id), id)
                  : ~0ull;
        arr = rank_u64<KP>(sk, K);
      }
    }
    if (valid) m_perm[arr] = lane;
  };
  const int nbk = (K + 15) >> 4;
  if (nbk <= 1) {
    gram_tile<METRIC, 1>(A.X, ld, d4, m_pid, K, tile, gdiag, ts, li, lk, arrival);
  } else if (nbk == 2) {
    if constexpr (NB >= 2)
      gram_tile<METRIC, 2>(A.X, ld, d4, m_pid, K, tile, gdiag, ts, li, lk, arrival);
  } else if (nbk == 3) {
    if constexpr (NB >= 3)
      gram_tile<METRIC, 3>(A.X, ld, d4, m_pid, K, tile, gdiag, ts, li, lk, arrival);
  } else {
    if constexpr (NB >= 4)
      gram_tile<METRIC, 4>(A.X, ld, d4, m_pid, K, tile, gdiag, ts, li, lk, arrival);
  }
  __syncthreads();

  // ---- 4. candidates in arrival order: lane t holds candidate t
  const int pidx = valid ? m_perm[lane] : 0;  // its pool index = (key, id) rank
  const int cid = valid ? m_pid[pidx] : -1;
  const float ckey = valid ? m_pkey[pidx] : INFINITY;
  const float cg = valid ? A.mcoef * fabsf(gdiag[pidx]) : 0.0f;
  const float* trow = tile + pidx * ts;  // D(., this candidate) in pool order

  uint64_t alive = 1ull;
  int partner = -1;
  unsigned nrecheck = 0;
#pragma unroll 1
  for (int t = 1; t < K; ++t) {
    const float kt = rl_f(ckey, t);
    const int pt = rl_i(pidx, t);
    const float cgt = rl_f(cg, t);
    const bool inA = (alive >> lane) & 1ull;
    const float Dtw = trow[pt];
    const float thr = fmaxf(kt, ckey);
    bool cond = inA && (Dtw < thr);
    const uint64_t nm = ballot(inA && (fabsf(Dtw - thr) <= cgt + cg));
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

  // ---- 5. one item per candidate: survivor -> v, redirected -> partner
  const bool isdead = valid && !((alive >> lane) & 1ull);
  const int pid_all = __shfl(cid, partner >= 0 ? partner : 0);  // partner's id
  const uint64_t dm = ballot(isdead);
  const int nred = __popcll(dm);
  float ikey = ckey;
  redirect_keys<METRIC>(A.X, ld, d4, dm, cid, pid_all, lane, ikey);
  if (valid) {
    const int64_t o = v * A.cap + lane;
    const int idest = isdead ? pid_all : (int)v;
    A.it_dest[o] = idest;
    A.it_cand[o] = cid;
    A.it_key[o] = ikey;
    if (isdead) atomicAdd(&A.cnt[idest], 1u);
  }
  if (lane == 0) {
    A.nitem[v] = K;
    atomicAdd(&A.cnt[v], (uint32_t)(K - nred));
  }
  st.redirects += (unsigned)nred;
  st.survivors += (unsigned)(K - nred);
  st.cands += (unsigned)K;
}

template <int METRIC, int NB, bool FINAL>
__global__ __launch_bounds__(64) void k_round(const RoundArgs A) {
  extern __shared__ __align__(16) float lds[];
  const uint32_t nv = min(A.vcount[1], (uint32_t)A.n);
  if (blockIdx.x >= nv) return;
  RoundStats st;
  round_vertex<METRIC, NB, FINAL>(A, (int64_t)A.vlist_b[blockIdx.x], lds, st);
  flush_stats(st, A.statp, FINAL, threadIdx.x);
}

// ---------------------------------------------------- small-pool kernel
// Four vertices per wave, one per 16-lane row g; lane (g, t) first holds pool
// entry t of its vertex, then, after the arrival order is known, the
// candidate that arrives t-th. Pools are compact with K <= 16 entries.
template <int METRIC, bool FINAL>
__global__ __launch_bounds__(64) void k_round_s(const RoundArgs A) {
  extern __shared__ __align__(16) float lds[];
  int* s_pid = reinterpret_cast<int*>(lds);
  float* s_pkey = lds + kWave;
  int* s_perm = reinterpret_cast<int*>(lds + 2 * kWave);
  float* tiles = lds + 3 * kWave;
  float* gdiag = tiles + 4 * kSmallTile;
  const int lane = threadIdx.x;
  const int g = lane >> 4, t = lane & 15;
  const int li = lane & 15, lk = lane >> 4;
  const int d4 = A.d4, R = A.R;
  const int64_t ld = A.ld;
  const uint32_t nv = min(A.vcount[0], (uint32_t)A.n);
  const uint32_t ntask = (nv + 3u) >> 2;
  if (blockIdx.x >= ntask) return;
  RoundStats st;
  {
    const uint32_t task = blockIdx.x;
    const uint32_t vi = 4u * task + (uint32_t)g;
    const bool gv = vi < nv;
    const int64_t v = gv ? (int64_t)A.vlist_s[vi] : 0;
    int id = -1;
    float key = INFINITY;
    if (gv && t < R) {
      id = A.in_ids[v * R + t];
      key = A.in_keys[v * R + t];
    }
    const bool valid = gv && id >= 0 && (int64_t)id < A.n;  // a prefix of each row
    if (!valid) {
      id = -1;
      key = INFINITY;
    }
    const uint64_t vm = ballot(valid);
    const uint32_t seg = (uint32_t)(vm >> (16 * g)) & 0xFFFFu;
    const int Kg = __popc(seg);
    int Kmax = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) Kmax = max(Kmax, __popc((uint32_t)(vm >> (16 * q)) & 0xFFFFu));

    s_pid[lane] = valid ? id : 0;  // row 0 stands in for absent entries
    s_pkey[lane] = key;
    __syncthreads();

    // ---- arrival order within each row (Section 3.3)
    int arr = t;
    if (!FINAL) {
      if (A.order == 2) {
        arr = Kg - 1 - t;
      } else if (A.order == 0) {
        const uint64_t sk =
            valid ? hash_order_key(hash4(A.seed, kTagUpdate + A.round, (uint64_t)v,
                                         (uint64_t)(uint32_t)id), id)
                  : ~0ull;
        int r = 0;
        static_for<0, 16>([&](auto jc) {
          constexpr int J = decltype(jc)::value;
          r += (bcast16_u64<J>(sk) < sk) ? 1 : 0;
        });
        arr = r;
      }
    }
    if (valid) s_perm[16 * g + arr] = t;

    // ---- Gram and distance tiles of the four vertices
    gram_small<METRIC>(A.X, ld, d4, s_pid, tiles, gdiag, li, lk);
    __syncthreads();

    // ---- lane (g, t) takes the candidate arriving t-th
    const int pidx = valid ? s_perm[16 * g + t] : 0;
    const int cid = valid ? s_pid[16 * g + pidx] : -1;
    const float ckey = valid ? s_pkey[16 * g + pidx] : INFINITY;
    const float cg = valid ? A.mcoef * fabsf(gdiag[16 * g + pidx]) : 0.0f;
    const float* trow = tiles + g * kSmallTile + pidx * kSmallTs;

    uint64_t alive = vm & 0x0001000100010001ull;  // the first arrival of each row
    int partner = -1;
    unsigned nrecheck = 0;
    static_for<1, 16>([&](auto tc) {
      constexpr int T = decltype(tc)::value;
      if (T < Kmax) {
        const bool tv = T < Kg;
        const float kt = bcast16_f<T>(ckey);
        const int pt = bcast16_i<T>(pidx);
        const float cgt = bcast16_f<T>(cg);
        const bool act = tv && ((alive >> lane) & 1ull);
        const float Dtw = trow[pt];
        const float thr = fmaxf(kt, ckey);
        bool cond = act && (Dtw < thr);
        const uint64_t nm = ballot(act && (fabsf(Dtw - thr) <= cgt + cg));
        if (nm)
          recheck_pairs<METRIC>(A.X, ld, d4, nm, cid, bcast16_i<T>(cid), thr, lane, cond,
                                nrecheck);
        const uint64_t hit = ballot(cond);
        const uint64_t ufar = ballot(cond && pidx < pt);
        uint64_t rem = 0, tdead = 0, tlive = 0;
        uint32_t pgp = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t uf = (uint32_t)(ufar >> (16 * q)) & 0xFFFFu;
          const uint32_t h = (uint32_t)(hit >> (16 * q)) & 0xFFFFu;
          if (uf) {
            const uint32_t p = (uint32_t)(__ffs(uf) - 1);
            rem |= (uint64_t)(h & ((1u << p) - 1u)) << (16 * q);
            tdead |= 1ull << (16 * q + T);
            pgp |= p << (8 * q);
          } else {
            rem |= (uint64_t)h << (16 * q);
            tlive |= 1ull << (16 * q + T);
          }
        }
        tlive &= vm;  // rows whose vertex has a T-th candidate
        alive = (alive & ~rem) | tlive;
        if ((rem >> lane) & 1ull) partner = T;
        if ((tdead >> lane) & 1ull) partner = (int)((pgp >> (8 * g)) & 0xFFu);
      }
    });
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const unsigned long long kq = (unsigned long long)__popc((uint32_t)(vm >> (16 * q)) & 0xFFFFu);
      st.pairs += kq * (kq - (kq > 0 ? 1 : 0)) / 2;
    }
    st.rechecks += nrecheck;

    if (FINAL) {
      const uint32_t aseg = (uint32_t)(alive >> (16 * g)) & 0xFFFFu;
      const int na = __popc(aseg);
      const int pos = __popc(aseg & ((1u << t) - 1u));
      if (gv) {
        const int64_t o = v * R;
        if ((aseg >> t) & 1u) {
          A.out_adj[o + pos] = cid;
          if (A.out_keys) A.out_keys[o + pos] = ckey;
        }
        for (int sl = t; sl < R; sl += 16) {
          if (sl >= na) {
            A.out_adj[o + sl] = -1;
            if (A.out_keys) A.out_keys[o + sl] = INFINITY;
          }
        }
      }
    } else {
      const bool isdead = valid && !((alive >> lane) & 1ull);
      const int pid_all = __shfl(cid, 16 * g + (partner >= 0 ? partner : 0));
      const uint64_t dm = ballot(isdead);
      float ikey = ckey;
      redirect_keys<METRIC>(A.X, ld, d4, dm, cid, pid_all, lane, ikey);
      if (valid) {
        const int64_t o = v * A.cap + t;
        const int idest = isdead ? pid_all : (int)v;
        A.it_dest[o] = idest;
        A.it_cand[o] = cid;
        A.it_key[o] = ikey;
        if (isdead) atomicAdd(&A.cnt[idest], 1u);
      }
      if (gv && t == 0) {
        const int nd = __popc((uint32_t)(dm >> (16 * g)) & 0xFFFFu);
        A.nitem[v] = Kg;
        if (Kg - nd > 0) atomicAdd(&A.cnt[v], (uint32_t)(Kg - nd));
      }
      const unsigned nred = (unsigned)__popcll(dm), ncand = (unsigned)__popcll(vm);
      st.redirects += nred;
      st.survivors += ncand - nred;
      st.cands += ncand;
    }
  }
  flush_stats(st, A.statp, FINAL, lane);
}

// ------------------------------------------------------- classification
// Splits the vertices into the small-pool list (compact rows with at most 16
// valid entries) and the general list; counts[0], counts[1] must be zero.
// Each block takes 1024 consecutive vertices (4 per thread) and reserves its
// list ranges with one atomic per list. The flags come from pool_small (set
// by the merge that wrote the pools) when given, else from the rows.
constexpr int kClassPer = 4;

__device__ __forceinline__ bool row_is_small(const int32_t* __restrict__ ids, int64_t v,
                                             int64_t n, int32_t R) {
  const int32_t* row = ids + v * R;
  int32_t e[kMaxR];
#pragma unroll
  for (int j = 0; j < kMaxR; ++j) e[j] = (j < R) ? row[j] : -1;
  uint64_t vmask = 0;
#pragma unroll
  for (int j = 0; j < kMaxR; ++j)
    if (e[j] >= 0 && (int64_t)e[j] < n) vmask |= 1ull << j;
  const int K = __popcll(vmask);
  return K <= 16 && vmask == ((1ull << K) - 1ull);  // K <= 16: no shift by 64
}

__global__ __launch_bounds__(256) void k_classify(const int32_t* __restrict__ ids,
                                                  const uint8_t* __restrict__ pool_small,
                                                  int64_t n, int32_t R, int32_t* __restrict__ vs,
                                                  int32_t* __restrict__ vb,
                                                  uint32_t* __restrict__ counts) {
  __shared__ uint32_t wsum[2][4];
  __shared__ uint32_t base[2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t v0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * kClassPer;
  uint32_t fs = 0, fb = 0;  // per-vertex flags, bit k for vertex v0 + k
#pragma unroll
  for (int k = 0; k < kClassPer; ++k) {
    const int64_t v = v0 + k;
    if (v < n) {
      const bool sm = pool_small ? pool_small[v] != 0 : row_is_small(ids, v, n, R);
      if (sm) fs |= 1u << k; else fb |= 1u << k;
    }
  }
  // exclusive scan of the per-thread counts over the block, per list
  uint32_t incl[2] = {(uint32_t)__popc(fs), (uint32_t)__popc(fb)};
  const uint32_t own[2] = {incl[0], incl[1]};
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const uint32_t y = __shfl_up(incl[l], o);
      if (lane >= o) incl[l] += y;
    }
  }
  if (lane == 63) {
    wsum[0][wv] = incl[0];
    wsum[1][wv] = incl[1];
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int l = threadIdx.x;
    const uint32_t tot = wsum[l][0] + wsum[l][1] + wsum[l][2] + wsum[l][3];
    base[l] = tot ? atomicAdd(&counts[l], tot) : 0u;
  }
  __syncthreads();
  uint32_t pos[2];
#pragma unroll
  for (int l = 0; l < 2; ++l) {
    pos[l] = base[l] + incl[l] - own[l];
    for (int k = 0; k < wv; ++k) pos[l] += wsum[l][k];
  }
#pragma unroll
  for (int k = 0; k < kClassPer; ++k) {
    const int32_t v = (int32_t)(v0 + k);
    if ((fs >> k) & 1u) {
      if (pos[0] < (uint64_t)n) vs[pos[0]] = v;
      ++pos[0];
    } else if ((fb >> k) & 1u) {
      if (pos[1] < (uint64_t)n) vb[pos[1]] = v;
      ++pos[1];
    }
  }
}

// ----------------------------------------------------------------- launchers
size_t round_lds_bytes(int R, int /*d*/) {
  const int nb = (R + 15) / 16;
  const size_t g = (size_t)round3_lds(16 * nb).total * sizeof(float);
  const size_t sm = (size_t)kSmallLdsFloats * sizeof(float);
  return g > sm ? g : sm;
}

template <int METRIC, int NB, bool FINAL>
static hipError_t launch_round_t(const RoundArgs& a, hipStream_t s) {
  const size_t lds = (size_t)round3_lds(16 * NB).total * sizeof(float);
  hipLaunchKernelGGL((k_round<METRIC, NB, FINAL>), dim3((unsigned)a.n), dim3(64), lds, s, a);
  return hipGetLastError();
}

template <int METRIC, bool FINAL>
static hipError_t launch_round_m(const RoundArgs& a, hipStream_t s) {
  hipError_t e;
  switch ((a.R + 15) / 16) {
    case 1: e = launch_round_t<METRIC, 1, FINAL>(a, s); break;
    case 2: e = launch_round_t<METRIC, 2, FINAL>(a, s); break;
    case 3: e = launch_round_t<METRIC, 3, FINAL>(a, s); break;
    default: e = launch_round_t<METRIC, 4, FINAL>(a, s); break;
  }
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)((a.n + 3) / 4);
  hipLaunchKernelGGL((k_round_s<METRIC, FINAL>), dim3(grid), dim3(64),
                     (size_t)kSmallLdsFloats * sizeof(float), s, a);
  return hipGetLastError();
}

hipError_t launch_classify(const int32_t* ids, const uint8_t* pool_small, int64_t n, int32_t R,
                           int32_t* vs, int32_t* vb, uint32_t* counts, hipStream_t s) {
  const int64_t per_block = 256 * kClassPer;
  hipLaunchKernelGGL(k_classify, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(256), 0,
                     s, ids, pool_small, n, R, vs, vb, counts);
  return hipGetLastError();
}

hipError_t launch_round(const RoundArgs& a, int metric, bool final_pass, hipStream_t s) {
  if (metric == 0)
    return final_pass ? launch_round_m<0, true>(a, s) : launch_round_m<0, false>(a, s);
  return final_pass ? launch_round_m<1, true>(a, s) : launch_round_m<1, false>(a, s);
}

}  // namespace grnnd
