// round.hip -- the round kernels with FP32 tiles for the L2 metric, the
// classification pass and the launch entry (kernels in round_impl.hpp; the
// FP32 inner-product instances in round_ip.hip, narrow-tile instances in
// round_bf16.hip, round_fp16.hip, round_fp8.hip).
#include "round_impl.hpp"

namespace grnnd {

hipError_t launch_round_fp32_ip(const RoundArgs& a, bool final_pass, bool compact_pools,
                                hipStream_t s);

hipError_t launch_round_bf16(const RoundArgs& a, int metric, bool final_pass, bool compact_pools,
                             hipStream_t s);
hipError_t launch_round_fp16(const RoundArgs& a, int metric, bool final_pass, bool compact_pools,
                             hipStream_t s);
hipError_t launch_round_fp8(const RoundArgs& a, int metric, bool final_pass, bool compact_pools,
                            hipStream_t s);
hipError_t launch_probe_bf16(const RoundArgs& a, int metric, const int32_t* ids, int64_t nv,
                             float* t, float* b, float* c, hipStream_t s);
hipError_t launch_probe_fp16(const RoundArgs& a, int metric, const int32_t* ids, int64_t nv,
                             float* t, float* b, float* c, hipStream_t s);
hipError_t launch_probe_fp8(const RoundArgs& a, int metric, const int32_t* ids, int64_t nv,
                            float* t, float* b, float* c, hipStream_t s);

namespace {
// ------------------------------------------------------- classification
// Splits the vertices into four lists by pool class: 0, 1, 2 = compact
// (valid entries first) with at most 16, 32, 64 valid entries, 3 = any other
// pool; counts[0..3] must be zero. The vertices are visited in the locality
// order when one is given (else by id); each block takes 1024 consecutive
// positions (4 per thread) and reserves its list ranges with one atomic per
// list, so the lists keep the order within each 1024-vertex run. The classes
// come from pool_cls (set by the merge that wrote the pools; its rows are
// compact) when given, else from the rows.
constexpr int kClassPer = 4;
constexpr int kLists = 4;

__device__ __forceinline__ int row_class(const int32_t* __restrict__ ids, int64_t v, int64_t n,
                                         int32_t R) {
  const int32_t* row = ids + v * R;
  int32_t e[kMaxR];
#pragma unroll
  for (int j = 0; j < kMaxR; ++j) e[j] = (j < R) ? row[j] : -1;
  uint64_t vmask = 0;
#pragma unroll
  for (int j = 0; j < kMaxR; ++j)
    if (e[j] >= 0 && (int64_t)e[j] < n) vmask |= 1ull << j;
  const int K = __popcll(vmask);
  if (vmask != (K == 64 ? ~0ull : ((1ull << K) - 1ull))) return 3;  // holes
  return K <= 16 ? 0 : (K <= 32 ? 1 : 2);
}

__global__ __launch_bounds__(256) void k_classify(const int32_t* __restrict__ ids,
                                                  const uint8_t* __restrict__ pool_cls,
                                                  const int32_t* __restrict__ order,
                                                  int64_t n, int32_t R, int32_t* __restrict__ l0,
                                                  int32_t* __restrict__ l1,
                                                  int32_t* __restrict__ l2,
                                                  int32_t* __restrict__ l3,
                                                  uint32_t* __restrict__ counts) {
  __shared__ uint32_t wsum[kLists][4];
  __shared__ uint32_t base[kLists];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * kClassPer;
  uint32_t f[kLists] = {0u, 0u, 0u, 0u};  // per-class flags, bit k for position i0 + k
  int32_t vk[kClassPer];
#pragma unroll
  for (int k = 0; k < kClassPer; ++k) {
    const int64_t i = i0 + k;
    vk[k] = 0;
    if (i < n) {
      const int64_t v = order ? (int64_t)order[i] : i;
      vk[k] = (int32_t)v;
      const int c = pool_cls ? (int)pool_cls[v] : row_class(ids, v, n, R);
      f[c > 3 ? 3 : c] |= 1u << k;
    }
  }
  // exclusive scan of the per-thread counts over the block, per list
  uint32_t incl[kLists], own[kLists];
#pragma unroll
  for (int l = 0; l < kLists; ++l) incl[l] = own[l] = (uint32_t)__popc(f[l]);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
    for (int l = 0; l < kLists; ++l) {
      const uint32_t y = __shfl_up(incl[l], o);
      if (lane >= o) incl[l] += y;
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int l = 0; l < kLists; ++l) wsum[l][wv] = incl[l];
  }
  __syncthreads();
  if (threadIdx.x < kLists) {
    const int l = threadIdx.x;
    const uint32_t tot = wsum[l][0] + wsum[l][1] + wsum[l][2] + wsum[l][3];
    base[l] = tot ? atomicAdd(&counts[l], tot) : 0u;
  }
  __syncthreads();
  int32_t* lists[kLists] = {l0, l1, l2, l3};
#pragma unroll
  for (int l = 0; l < kLists; ++l) {
    uint32_t pos = base[l] + incl[l] - own[l];
    for (int k = 0; k < wv; ++k) pos += wsum[l][k];
#pragma unroll
    for (int k = 0; k < kClassPer; ++k) {
      if ((f[l] >> k) & 1u) {
        if (pos < (uint64_t)n) lists[l][pos] = vk[k];
        ++pos;
      }
    }
  }
}

}  // namespace

size_t round_lds_bytes(int R, int /*d*/) {
  const int nb = (R + 15) / 16;
  size_t b = (size_t)round3_lds(16 * nb).total;
  // the FP8 layout is the largest of the group kernels'
  constexpr size_t g16 = GroupLds<16, GRNND_PREC_FP8_E4M3>::total;
  constexpr size_t g32 = GroupLds<32, GRNND_PREC_FP8_E4M3>::total;
  constexpr size_t g64 = GroupLds<64, GRNND_PREC_FP8_E4M3, 64>::total;
  b = b > g16 ? b : g16;
  b = b > g32 ? b : g32;
  b = b > g64 ? b : g64;
  return b * sizeof(float);
}

hipError_t launch_classify(const int32_t* ids, const uint8_t* pool_cls, const int32_t* order,
                           int64_t n, int32_t R, int32_t* const (&lists)[4], uint32_t* counts,
                           hipStream_t s) {
  const int64_t per_block = 256 * kClassPer;
  hipLaunchKernelGGL(k_classify, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(256), 0,
                     s, ids, pool_cls, order, n, R, lists[0], lists[1], lists[2], lists[3],
                     counts);
  return hipGetLastError();
}

hipError_t launch_round(const RoundArgs& a, int metric, bool final_pass, bool compact_pools,
                        hipStream_t s) {
  switch (a.prec) {
    case GRNND_PREC_BF16: return launch_round_bf16(a, metric, final_pass, compact_pools, s);
    case GRNND_PREC_FP16: return launch_round_fp16(a, metric, final_pass, compact_pools, s);
    case GRNND_PREC_FP8_E4M3: return launch_round_fp8(a, metric, final_pass, compact_pools, s);
    default:
      return metric == 0 ? launch_round_pm<GRNND_PREC_FP32, 0>(a, final_pass, compact_pools, s)
                         : launch_round_fp32_ip(a, final_pass, compact_pools, s);
  }
}

hipError_t launch_tile_probe(const RoundArgs& a, int metric, const int32_t* ids, int64_t nv,
                             float* t, float* b, float* c, hipStream_t s) {
  switch (a.prec) {
    case GRNND_PREC_BF16: return launch_probe_bf16(a, metric, ids, nv, t, b, c, s);
    case GRNND_PREC_FP16: return launch_probe_fp16(a, metric, ids, nv, t, b, c, s);
    case GRNND_PREC_FP8_E4M3: return launch_probe_fp8(a, metric, ids, nv, t, b, c, s);
    default: return launch_tile_probe_prec<GRNND_PREC_FP32>(a, metric, ids, nv, t, b, c, s);
  }
}

}  // namespace grnnd
