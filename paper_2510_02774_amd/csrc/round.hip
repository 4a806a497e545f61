// round.hip -- update round and output pass, the hot path (gfx950, wave64).
//
// One wave (one workgroup) handles one vertex. For its vertex it
//   1. reads the pool row (K candidates, sorted by (key, id));
//   2. loads the candidate rows straight into registers in the operand
//      layout of the 16x16x4 FP32 matrix instruction (lane l holds row
//      16 I + l % 16, float4 group 4 s + l / 16), while it computes the
//      candidates' arrival order (Section 3.3);
//   3. forms the Gram tile of the candidates on the matrix cores, in pool
//      order, and turns it into a symmetric distance tile in LDS
//      (D = G_ii + G_jj - 2 G_ij for L2, -G_ij for IP); a decision within the
//      tile's rigorous error bound of its threshold is re-decided exactly;
//   4. runs the prune scan of Eq. 2 in arrival order with wave ballots;
//   5. re-decides near-threshold comparisons and computes every redirect key
//      with the canonical distance on the rows in global memory (just read,
//      so served from cache; up to 16 pairs per memory round trip), and emits
//      one item per candidate (Alg. 4), or, for the output pass, writes the
//      kept row.
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {

__device__ __forceinline__ void stat_add_r(unsigned long long* statp, int slot, int idx,
                                           unsigned long long v) {
  if (v) atomicAdd(statp + (size_t)slot * kStatStride + idx, v);
}

// Per-wave LDS of the round kernel (floats): pool-order ids, keys and
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

// Canonical distances of up to four pairs given by point ids (global rows).
template <int METRIC>
__device__ __forceinline__ float glb_pair(const float* X, int64_t ld, int d4, int ia, int ib,
                                          int lane) {
  const GlobalRow a{X + (int64_t)ia * ld};
  const GlobalRow b{X + (int64_t)ib * ld};
  return dist16<METRIC>(a, b, d4, lane & 15);
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

}  // namespace

template <int METRIC, int NB, bool FINAL>
__global__ __launch_bounds__(64) void k_round(const RoundArgs A) {
  extern __shared__ __align__(16) float lds[];
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
  const int slot = (int)(blockIdx.x % kStatSlots);

  const int64_t v = blockIdx.x;
  int id0 = -1;
  float key0 = INFINITY;
  if (lane < R) {
    id0 = A.in_ids[v * R + lane];
    key0 = A.in_keys[v * R + lane];
  }
  {
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
      } else if (lane == 0) {
        A.nitem[v] = K;
        if (K == 1) {
          const int64_t o = v * A.cap;
          A.it_dest[o] = (int32_t)v;
          A.it_cand[o] = id;
          A.it_key[o] = key;
          atomicAdd(&A.cnt[v], 1u);
          stat_add_r(A.statp, slot, 3, 1);
          stat_add_r(A.statp, slot, 5, 1);
        }
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
      if constexpr (NB >= 2) gram_tile<METRIC, 2>(A.X, ld, d4, m_pid, K, tile, gdiag, ts, li, lk, arrival);
    } else if (nbk == 3) {
      if constexpr (NB >= 3) gram_tile<METRIC, 3>(A.X, ld, d4, m_pid, K, tile, gdiag, ts, li, lk, arrival);
    } else {
      if constexpr (NB >= 4) gram_tile<METRIC, 4>(A.X, ld, d4, m_pid, K, tile, gdiag, ts, li, lk, arrival);
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
    for (int t = 1; t < KP; ++t) {
      if (t < K) {
        const float kt = rl_f(ckey, t);
        const int pt = rl_i(pidx, t);
        const float cgt = rl_f(cg, t);
        const int idt = rl_i(cid, t);
        const bool inA = (alive >> lane) & 1ull;
        const float Dtw = trow[pt];
        const float thr = fmaxf(kt, ckey);
        bool cond = inA && (Dtw < thr);
        uint64_t nm = ballot(inA && (fabsf(Dtw - thr) <= cgt + cg));
        while (nm) {  // near the threshold: decide with the canonical distance
          int w[4], iw[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            w[g] = nm ? __ffsll((long long)nm) - 1 : -1;
            if (nm) nm &= nm - 1;
            iw[g] = w[g] >= 0 ? rl_i(cid, w[g]) : idt;
          }
          int mine = iw[0];
#pragma unroll
          for (int g = 1; g < 4; ++g)
            if (lk == g) mine = iw[g];
          const float dd = glb_pair<METRIC>(A.X, ld, d4, idt, mine, lane);
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            if (w[g] >= 0) {
              const float dg = rl_f(dd, 16 * g);
              if (lane == w[g]) cond = dg < thr;
              ++nrecheck;
            }
          }
        }
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
    }

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
      if (lane == 0) {
        stat_add_r(A.statp, slot, 7, (unsigned long long)K * (K - 1) / 2);
        stat_add_r(A.statp, slot, 1, nrecheck);
      }
      return;
    }

    // ---- 5. one item per candidate: survivor -> v, redirected -> partner
    const bool isdead = valid && !((alive >> lane) & 1ull);
    const int pid_all = __shfl(cid, partner >= 0 ? partner : 0);  // partner's id
    const int pid = isdead ? pid_all : -1;
    uint64_t dm = ballot(isdead);
    const int nred = __popcll(dm);
    float ikey = ckey;
    while (dm) {  // up to 16 redirect keys per memory round trip
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
        ib[k] = __shfl(pid_all, wa);
      }
      float dd[NOP];
      dist16_batch<METRIC, NOP>(A.X, ld, d4, ia, ib, li, dd);
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
    if (valid) {
      const int64_t o = v * A.cap + lane;
      const int idest = isdead ? pid : (int)v;
      A.it_dest[o] = idest;
      A.it_cand[o] = cid;
      A.it_key[o] = ikey;
      if (isdead) atomicAdd(&A.cnt[idest], 1u);
    }
    if (lane == 0) {
      A.nitem[v] = K;
      atomicAdd(&A.cnt[v], (uint32_t)(K - nred));
    }
    if (lane == 0) {
      stat_add_r(A.statp, slot, 0, (unsigned long long)K * (K - 1) / 2);
      stat_add_r(A.statp, slot, 1, nrecheck);
      stat_add_r(A.statp, slot, 2, (unsigned long long)nred);
      stat_add_r(A.statp, slot, 3, (unsigned long long)(K - nred));
      stat_add_r(A.statp, slot, 5, (unsigned long long)K);
    }
  }
}

// ----------------------------------------------------------------- launchers
size_t round_lds_bytes(int R, int /*d*/) {
  const int nb = (R + 15) / 16;
  return (size_t)round3_lds(16 * nb).total * sizeof(float);
}

template <int METRIC, int NB, bool FINAL>
static hipError_t launch_round_t(const RoundArgs& a, hipStream_t s) {
  const size_t lds = (size_t)round3_lds(16 * NB).total * sizeof(float);
  const unsigned grid = (unsigned)a.n;
  hipLaunchKernelGGL((k_round<METRIC, NB, FINAL>), dim3(grid), dim3(64), lds, s, a);
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

}  // namespace grnnd
