// search.hip -- best-first graph search, one wave per query (gfx950).
//
// The list of at most L <= 256 (key, id) entries is held in LJ = L/64
// registers per lane, sorted (position j*64 + lane). Each step expands the
// first unexpanded entry: its not yet visited neighbours are marked in an LDS
// hash set (linear probing with compare-and-swap), their keys are computed
// with the canonical distance straight from the rows in memory, 16 per
// memory round trip, and they are inserted in adjacency order, keeping the
// best L. If the set ever fills up, an unseen-or-forgotten id is
// also checked against the list; an id forgotten that way and no longer in
// the list is rejected on re-insertion, because the L-th entry of the list
// never grows, so the result equals that of an exact visited set.
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {
constexpr int kHashBits = 13;
constexpr int kHashSize = 1 << kHashBits;
constexpr int kProbes = 32;

// Per-wave LDS (words): the visited hash set, the fresh ids of a step and
// their keys.
struct SearchLds {
  int tab_off, sid_off, key_off, total;
};

__host__ __device__ inline SearchLds search_lds(int /*R*/, int /*d4*/) {
  SearchLds S;
  S.tab_off = 0;
  S.sid_off = kHashSize;
  S.key_off = S.sid_off + kWave;
  S.total = S.key_off + kWave;
  return S;
}

__device__ __forceinline__ int tab_slot(int id) {
  return (int)(((uint32_t)id * 2654435761u) >> (32 - kHashBits));
}

__device__ __forceinline__ bool kid_less(float ka, int ia, float kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}
}  // namespace

template <int METRIC, int LJ>
__global__ __launch_bounds__(64) void k_search(const SearchArgs A) {
  extern __shared__ __align__(16) float lds[];
  const SearchLds S = search_lds(A.R, A.d4);
  int* tab = reinterpret_cast<int*>(lds + S.tab_off);
  int* sid = reinterpret_cast<int*>(lds + S.sid_off);
  float* skey = lds + S.key_off;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk4 = lane >> 4;
  const int64_t qi = blockIdx.x;
  const int d4 = A.d4;
  const int L = A.L;
  const float* qrow = A.Q + qi * A.ldq;

  for (int i = lane; i < kHashSize; i += kWave) tab[i] = -1;
  __syncthreads();
  const GlobalRow Q{qrow};

  float lk[LJ];
  int lid[LJ];
  bool lexp[LJ];
#pragma unroll
  for (int j = 0; j < LJ; ++j) {
    lk[j] = INFINITY;
    lid[j] = -1;
    lexp[j] = false;
  }
  {
    // the entry: the caller's, or the medoid computed on the device before
    const int64_t entry = A.entry_dev ? *A.entry_dev : A.entry;
    const float k0 = dist16<METRIC>(Q, GlobalRow{A.X + entry * A.ld}, d4, lane & 15);
    if (lane == 0) {
      lk[0] = k0;
      lid[0] = (int)entry;
      tab[tab_slot((int)entry)] = (int)entry;
    }
  }
  int cnt = 1;
  __syncthreads();

  for (;;) {
    // first unexpanded entry
    int pj = -1, pl = 0;
#pragma unroll
    for (int j = 0; j < LJ; ++j) {
      const uint64_t m = ballot(64 * j + lane < cnt && !lexp[j]);
      if (pj < 0 && m) {
        pj = j;
        pl = __ffsll((long long)m) - 1;
      }
    }
    if (pj < 0) break;
    int u = 0;
#pragma unroll
    for (int j = 0; j < LJ; ++j)
      if (j == pj) {
        u = rl_i(lid[j], pl);
        if (lane == pl) lexp[j] = true;
      }

    const int nb = (lane < A.R) ? A.adj[(int64_t)u * A.R + lane] : -1;
    const bool valid = nb >= 0 && (int64_t)nb < A.n;
    bool fresh = false, unknown = false;
    if (valid) {
      int s = tab_slot(nb);
      int pr = 0;
      for (; pr < kProbes; ++pr) {
        const int old = atomicCAS(&tab[s], -1, nb);
        if (old == -1) { fresh = true; break; }
        if (old == nb) break;
        s = (s + 1) & (kHashSize - 1);
      }
      unknown = pr == kProbes;
    }
    if (ballot(unknown)) {  // set full along this probe path: consult the list
      bool inl = false;
#pragma unroll
      for (int j = 0; j < LJ; ++j)
        for (int i = 0; i < 64 && 64 * j + i < cnt; ++i) inl = inl || (rl_i(lid[j], i) == nb);
      if (unknown) fresh = !inl;
    }
    const uint64_t fm = ballot(fresh);
    const int nf = __popcll(fm);
    if (fresh) sid[__popcll(fm & lanemask_lt(lane))] = nb;
    __syncthreads();
    if (nf == 0) continue;

    for (int f0 = 0; f0 < nf; f0 += 16) {  // op k, lane group g: fresh id f0 + 4 k + g
      constexpr int NOP = 4;
      const float* pa[NOP];
      const float* pb[NOP];
#pragma unroll
      for (int k = 0; k < NOP; ++k) {
        pa[k] = qrow;
        pb[k] = A.X + (int64_t)sid[min(f0 + 4 * k + lk4, nf - 1)] * A.ld;
      }
      float dd[NOP];
      dist16_rows<METRIC, NOP>(pa, pb, d4, li, dd);
      if (li == 0) {
#pragma unroll
        for (int k = 0; k < NOP; ++k)
          if (f0 + 4 * k + lk4 < nf) skey[f0 + 4 * k + lk4] = dd[k];
      }
    }
    __syncthreads();
    for (int f = 0; f < nf; ++f) {
      const float ck = skey[f];
      const int ci = sid[f];
      if (cnt == L) {
        float lastk = 0.f;
        int lasti = 0;
#pragma unroll
        for (int j = 0; j < LJ; ++j)
          if (j == (L - 1) >> 6) {
            lastk = rl_f(lk[j], (L - 1) & 63);
            lasti = rl_i(lid[j], (L - 1) & 63);
          }
        if (!kid_less(ck, ci, lastk, lasti)) continue;
      }
      int pos = 0;
#pragma unroll
      for (int j = 0; j < LJ; ++j)
        pos += __popcll(ballot(64 * j + lane < cnt && kid_less(lk[j], lid[j], ck, ci)));
      float uk[LJ];
      int ui[LJ];
      bool ue[LJ];
#pragma unroll
      for (int j = 0; j < LJ; ++j) {
        uk[j] = __shfl_up(lk[j], 1);
        ui[j] = __shfl_up(lid[j], 1);
        ue[j] = __shfl_up((int)lexp[j], 1) != 0;
        if (j > 0 && lane == 0) {
          uk[j] = rl_f(lk[j - 1], 63);
          ui[j] = rl_i(lid[j - 1], 63);
          ue[j] = rl_i((int)lexp[j - 1], 63) != 0;
        }
      }
#pragma unroll
      for (int j = 0; j < LJ; ++j) {
        const int p = 64 * j + lane;
        if (p > pos) {
          lk[j] = uk[j];
          lid[j] = ui[j];
          lexp[j] = ue[j];
        } else if (p == pos) {
          lk[j] = ck;
          lid[j] = ci;
          lexp[j] = false;
        }
      }
      cnt = cnt < L ? cnt + 1 : L;
    }
    __syncthreads();
  }

#pragma unroll
  for (int j = 0; j < LJ; ++j) {
    const int p = 64 * j + lane;
    if (p < A.k) {
      const int64_t o = qi * A.k + p;
      A.out_ids[o] = p < cnt ? lid[j] : -1;
      A.out_keys[o] = p < cnt ? lk[j] : INFINITY;
    }
  }
}

// ------------------------------------------------------------------ medoid
// The approximate medoid of the points (the search's default entry point,
// Section 4.1): the point nearest, in L2, to the mean of all points, ties by
// the smaller id. FP64 throughout: the mean is a sum of FP32 rows, exact in
// any order for integer-valued data; each point's squared distance to the
// mean is summed over the coordinates in order with separately rounded
// subtractions, products and sums, so for a given mean every distance and
// the choice between equal distances are reproducible exactly.

// Block b sums rows [b chunk, b chunk + chunk) of every column.
__global__ __launch_bounds__(256) void k_colsum64(const float* __restrict__ X, int64_t n, int d,
                                                 int64_t chunk, double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
  for (int c = threadIdx.x; c < d; c += blockDim.x) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)X[r * d + c];
    part[(int64_t)blockIdx.x * d + c] = s;
  }
}

// mean[c] = (sum over blocks of part[b][c]) / n; resets the arg-min state.
__global__ __launch_bounds__(256) void k_mean64(const double* __restrict__ part, int nb, int64_t n,
                                               int d, double* __restrict__ mean,
                                               unsigned long long* __restrict__ best,
                                               int64_t* __restrict__ out) {
  for (int c = threadIdx.x; c < d; c += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * d + c];
    mean[c] = s / (double)n;
  }
  if (threadIdx.x == 0) {
    best[0] = ~0ull;
    *out = n;  // above every id; lowered by k_mpick
  }
}

// dist[i] = sum_k (x_ik - mean_k)^2 (non-negative doubles, so their bit
// patterns order like their values); best[0] = the smallest bit pattern.
__global__ __launch_bounds__(256) void k_mdist(const float* __restrict__ X, int64_t n, int d,
                                              const double* __restrict__ mean,
                                              double* __restrict__ dist,
                                              unsigned long long* __restrict__ best) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long b = ~0ull;
  if (i < n) {
    double s = 0.0;
    const float* x = X + i * d;
    for (int k = 0; k < d; ++k) {
      const double t = (double)x[k] - mean[k];
      const double t2 = t * t;
      s = s + t2;
    }
    dist[i] = s;
    b = (unsigned long long)__double_as_longlong(s);
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = shfl_xor_u64(b, o);
    b = y < b ? y : b;
  }
  if ((threadIdx.x & 63) == 0 && b != ~0ull) atomicMin(best, b);
}

// The smallest id whose distance is the minimum.
__global__ __launch_bounds__(256) void k_mpick(const double* __restrict__ dist, int64_t n,
                                              const unsigned long long* __restrict__ best,
                                              int64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (unsigned long long)__double_as_longlong(dist[i]) == *best)
    atomicMin(reinterpret_cast<unsigned long long*>(out), (unsigned long long)i);
}

MedoidLayout medoid_layout(int64_t n, int32_t d) {
  MedoidLayout m;
  m.nb = (int)(n < 256 ? n : 256);
  m.chunk = (n + m.nb - 1) / m.nb;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  m.part_off = 0;
  m.mean_off = al((size_t)m.nb * d * 8);
  m.dist_off = m.mean_off + al((size_t)d * 8);
  m.best_off = m.dist_off + al((size_t)n * 8);
  m.total = m.best_off + 256;
  return m;
}

hipError_t launch_medoid(const float* X, int64_t n, int32_t d, void* scratch, int64_t* out,
                         hipStream_t s) {
  const MedoidLayout m = medoid_layout(n, d);
  char* base = static_cast<char*>(scratch);
  double* part = reinterpret_cast<double*>(base + m.part_off);
  double* mean = reinterpret_cast<double*>(base + m.mean_off);
  double* dist = reinterpret_cast<double*>(base + m.dist_off);
  unsigned long long* best = reinterpret_cast<unsigned long long*>(base + m.best_off);
  hipLaunchKernelGGL(k_colsum64, dim3((unsigned)m.nb), dim3(256), 0, s, X, n, d, m.chunk, part);
  hipLaunchKernelGGL(k_mean64, dim3(1), dim3(256), 0, s, part, m.nb, n, d, mean, best, out);
  const unsigned grid = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_mdist, dim3(grid), dim3(256), 0, s, X, n, d, mean, dist, best);
  hipLaunchKernelGGL(k_mpick, dim3(grid), dim3(256), 0, s, dist, n, best, out);
  return hipGetLastError();
}

size_t search_lds_bytes(int R, int d) {
  return (size_t)search_lds(R, (d + 3) / 4).total * sizeof(float);
}

template <int METRIC, int LJ>
static hipError_t launch_search_t(const SearchArgs& a, hipStream_t s) {
  const size_t lds = (size_t)search_lds(a.R, a.d4).total * sizeof(float);
  hipLaunchKernelGGL((k_search<METRIC, LJ>), dim3((unsigned)a.nq), dim3(64), lds, s, a);
  return hipGetLastError();
}

template <int METRIC>
static hipError_t launch_search_m(const SearchArgs& a, hipStream_t s) {
  switch ((a.L + 63) / 64) {
    case 1: return launch_search_t<METRIC, 1>(a, s);
    case 2: return launch_search_t<METRIC, 2>(a, s);
    case 3: return launch_search_t<METRIC, 3>(a, s);
    default: return launch_search_t<METRIC, 4>(a, s);
  }
}

hipError_t launch_search(const SearchArgs& a, hipStream_t s) {
  return a.metric == 0 ? launch_search_m<0>(a, s) : launch_search_m<1>(a, s);
}

}  // namespace grnnd
