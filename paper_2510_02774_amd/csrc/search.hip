// search.hip -- best-first graph search, one wave per query (gfx950).
//
// The list of at most L <= 64 (key, id) entries lives one per lane, sorted.
// Each step expands the first unexpanded entry: the rows of its not yet seen
// neighbours are gathered into LDS with all loads in flight, their keys are
// computed with the canonical distance, and they are inserted in adjacency
// order. A small direct-mapped table in LDS remembers seen ids; an id whose
// entry was overwritten is recomputed and rejected, because the L-th entry of
// the list never grows, so the final list equals that of an exact visited set.
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {
constexpr int kHashBits = 12;
constexpr int kHashSize = 1 << kHashBits;

struct SearchLds {
  int q_off, rows_off, tab_off, sid_off, rs, total;
};

__host__ __device__ inline SearchLds search_lds(int R, int d) {
  SearchLds S;
  S.rs = round_up(d, 16) + 4;
  S.q_off = 0;
  S.rows_off = round_up(d, 16) + 4;
  S.tab_off = S.rows_off + R * S.rs;
  S.sid_off = S.tab_off + kHashSize;
  S.total = S.sid_off + kWave;
  return S;
}

__device__ __forceinline__ int tab_slot(int id) {
  return (int)(((uint32_t)id * 2654435761u) >> (32 - kHashBits));
}
}  // namespace

template <int METRIC>
__global__ __launch_bounds__(64) void k_search(const SearchArgs A) {
  extern __shared__ __align__(16) float lds[];
  const SearchLds S = search_lds(A.R, 4 * A.d4);
  float* q = lds + S.q_off;
  float* rows = lds + S.rows_off;
  int* tab = reinterpret_cast<int*>(lds + S.tab_off);
  int* sid = reinterpret_cast<int*>(lds + S.sid_off);
  const int lane = threadIdx.x;
  const int64_t qi = blockIdx.x;
  const int d4 = A.d4;
  const int d16q = round_up(4 * d4, 16) / 4;

  for (int c = lane; c < d16q; c += kWave)
    reinterpret_cast<float4*>(q)[c] =
        (c < d4) ? *reinterpret_cast<const float4*>(A.Q + qi * A.ldq + 4 * c)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
  for (int i = lane; i < kHashSize; i += kWave) tab[i] = -1;
  __syncthreads();

  float lk = INFINITY;
  int lid = -1;
  bool lexp = false;
  int cnt = 1;
  {
    const float k0 = dist_canon<METRIC>(q, A.X + A.entry * A.ld, d4, lane);
    if (lane == 0) {
      lk = k0;
      lid = (int)A.entry;
      tab[tab_slot((int)A.entry)] = (int)A.entry;
    }
  }
  __syncthreads();

  for (;;) {
    const uint64_t unexp = __ballot(lane < cnt && !lexp);
    if (!unexp) break;
    const int p = __ffsll((long long)unexp) - 1;
    const int u = __builtin_amdgcn_readlane(lid, p);
    if (lane == p) lexp = true;

    int nb = (lane < A.R) ? A.adj[(int64_t)u * A.R + lane] : -1;
    const bool valid = nb >= 0 && (int64_t)nb < A.n;
    const int slot = valid ? tab_slot(nb) : 0;
    bool fresh = valid && tab[slot] != nb;
    for (int i = 0; i < cnt; ++i) {
      const int x = __builtin_amdgcn_readlane(lid, i);
      fresh = fresh && (x != nb);
    }
    __syncthreads();
    if (fresh) tab[slot] = nb;
    const uint64_t fm = __ballot(fresh);
    const int nf = __popcll(fm);
    if (fresh) sid[__popcll(fm & lanemask_lt(lane))] = nb;
    __syncthreads();
    if (nf == 0) continue;

    // gather fresh rows
    {
      const int total = nf * d4;
      int r = lane / d4, c = lane % d4;
      const int sr = kWave / d4, sc = kWave % d4;
      for (int base = 0; base < total; base += kWave * 8) {
        float4 buf[8];
        int dst[8];
#pragma unroll
        for (int uu = 0; uu < 8; ++uu) {
          const int qq = base + uu * kWave + lane;
          dst[uu] = -1;
          if (qq < total) {
            buf[uu] = *reinterpret_cast<const float4*>(A.X + (int64_t)sid[r] * A.ld + 4 * c);
            dst[uu] = r * S.rs + 4 * c;
          }
          c += sc;
          r += sr;
          if (c >= d4) { c -= d4; ++r; }
        }
#pragma unroll
        for (int uu = 0; uu < 8; ++uu)
          if (dst[uu] >= 0) *reinterpret_cast<float4*>(rows + dst[uu]) = buf[uu];
      }
    }
    __syncthreads();

    float nkey = INFINITY;
    for (int f = 0; f < nf; ++f) {
      const float dd = dist_canon<METRIC>(q, rows + f * S.rs, d4, lane);
      if (lane == f) nkey = dd;
    }
    for (int f = 0; f < nf; ++f) {
      const float ck = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(nkey), f));
      const int ci = sid[f];
      if (cnt == A.L) {
        const float lastk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lk), A.L - 1));
        const int lasti = __builtin_amdgcn_readlane(lid, A.L - 1);
        if (!(ck < lastk || (ck == lastk && ci < lasti))) continue;
      }
      const bool before = lane < cnt && (lk < ck || (lk == ck && lid < ci));
      const int pos = __popcll(__ballot(before));
      const float uk = __shfl_up(lk, 1);
      const int ui = __shfl_up(lid, 1);
      const int ue = __shfl_up((int)lexp, 1);
      if (lane > pos) {
        lk = uk;
        lid = ui;
        lexp = ue != 0;
      } else if (lane == pos) {
        lk = ck;
        lid = ci;
        lexp = false;
      }
      cnt = cnt < A.L ? cnt + 1 : A.L;
    }
    __syncthreads();
  }

  if (lane < A.k) {
    const int64_t o = qi * A.k + lane;
    A.out_ids[o] = lane < cnt ? lid : -1;
    A.out_keys[o] = lane < cnt ? lk : INFINITY;
  }
}

size_t search_lds_bytes(int R, int d) { return (size_t)search_lds(R, d).total * sizeof(float); }

hipError_t launch_search(const SearchArgs& a, hipStream_t s) {
  const size_t lds = search_lds_bytes(a.R, 4 * a.d4);
  const void* fn = a.metric == 0 ? reinterpret_cast<const void*>(&k_search<0>)
                                 : reinterpret_cast<const void*>(&k_search<1>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (a.metric == 0)
    hipLaunchKernelGGL(k_search<0>, dim3((unsigned)a.nq), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL(k_search<1>, dim3((unsigned)a.nq), dim3(64), lds, s, a);
  return hipGetLastError();
}

}  // namespace grnnd
