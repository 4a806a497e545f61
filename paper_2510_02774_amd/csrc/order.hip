// order.hip -- a locality order of the vertices for the round kernels.
//
// The rounds gather the rows of every vertex's candidates. Candidates are
// near their vertex, so vertices that are near each other share many of
// them; processing such vertices together on one XCD lets its L2 serve the
// shared rows. The order groups the points by Voronoi cell of kOrderPivots
// pivot points (drawn with the counter-based hash the method uses for its
// random choices, tag 0x4000), using the first (up to) 32 coordinates -- a
// coarse cell is all the locality needs. The order only decides which
// vertices run together; it never changes a result.
#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {
constexpr uint64_t kTagOrder = 0x4000;
constexpr int kOrderDims = 32;

// Nearest pivot (by |p|^2 - 2 <x, p> over the sampled coordinates) of each
// point; pivots staged in LDS once per block of 256 points.
__global__ __launch_bounds__(256) void k_cell(const float* __restrict__ X, int64_t n, int32_t ld,
                                              int32_t ds, uint64_t seed,
                                              uint8_t* __restrict__ cell) {
  __shared__ float4 piv[kOrderPivots][kOrderDims / 4];
  __shared__ float pn[kOrderPivots];
  const int tid = threadIdx.x;
  const int d4 = ds >> 2;
  for (int p = tid; p < kOrderPivots; p += blockDim.x) {
    const int64_t id = (int64_t)(hash4(seed, kTagOrder, 0, (uint64_t)p) % (uint64_t)n);
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < kOrderDims / 4; ++q) {
      const float4 x = (q < d4) ? *reinterpret_cast<const float4*>(X + id * ld + 4 * q)
                                : make_float4(0.f, 0.f, 0.f, 0.f);
      piv[p][q] = x;
      s += x.x * x.x + x.y * x.y + x.z * x.z + x.w * x.w;
    }
    pn[p] = s;
  }
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + tid;
  if (v >= n) return;
  float4 xv[kOrderDims / 4];
#pragma unroll
  for (int q = 0; q < kOrderDims / 4; ++q)
    xv[q] = (q < d4) ? *reinterpret_cast<const float4*>(X + v * ld + 4 * q)
                     : make_float4(0.f, 0.f, 0.f, 0.f);
  float best = INFINITY;
  int bp = 0;
  for (int p = 0; p < kOrderPivots; ++p) {
    float dot = 0.0f;
#pragma unroll
    for (int q = 0; q < kOrderDims / 4; ++q) {
      const float4 y = piv[p][q];
      dot = fmaf(xv[q].x, y.x, dot);
      dot = fmaf(xv[q].y, y.y, dot);
      dot = fmaf(xv[q].z, y.z, dot);
      dot = fmaf(xv[q].w, y.w, dot);
    }
    const float sc = pn[p] - 2.0f * dot;
    if (sc < best) {
      best = sc;
      bp = p;
    }
  }
  cell[v] = (uint8_t)bp;
}

// Per-cell counts (hist[0..kOrderPivots), zeroed beforehand).
__global__ __launch_bounds__(256) void k_cell_hist(const uint8_t* __restrict__ cell, int64_t n,
                                                   uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kOrderPivots];
  for (int i = threadIdx.x; i < kOrderPivots; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const int64_t v0 = (int64_t)blockIdx.x * 4096;
  for (int k = threadIdx.x; k < 4096; k += blockDim.x)
    if (v0 + k < n) atomicAdd(&h[cell[v0 + k]], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderPivots; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Exclusive prefix of the counts into cursors (one block).
__global__ __launch_bounds__(kOrderPivots) void k_cell_scan(uint32_t* __restrict__ hist) {
  __shared__ uint32_t s[kOrderPivots];
  const int i = threadIdx.x;
  s[i] = hist[i];
  __syncthreads();
  for (int o = 1; o < kOrderPivots; o <<= 1) {
    const uint32_t y = i >= o ? s[i - o] : 0u;
    __syncthreads();
    s[i] += y;
    __syncthreads();
  }
  hist[i] = s[i] - hist[i];
}

// Places every vertex at its cell's range: each block reserves its share of
// every cell with one atomic, then ranks its vertices within the share.
__global__ __launch_bounds__(256) void k_cell_place(const uint8_t* __restrict__ cell, int64_t n,
                                                    uint32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ order) {
  __shared__ uint32_t h[kOrderPivots];
  __shared__ uint32_t base[kOrderPivots];
  for (int i = threadIdx.x; i < kOrderPivots; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const int64_t v0 = (int64_t)blockIdx.x * 4096;
  for (int k = threadIdx.x; k < 4096; k += blockDim.x)
    if (v0 + k < n) atomicAdd(&h[cell[v0 + k]], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kOrderPivots; i += blockDim.x) {
    base[i] = h[i] ? atomicAdd(&cursor[i], h[i]) : 0u;
    h[i] = 0u;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 4096; k += blockDim.x) {
    const int64_t v = v0 + k;
    if (v < n) {
      const int c = cell[v];
      const uint32_t pos = base[c] + atomicAdd(&h[c], 1u);
      if (pos < (uint64_t)n) order[pos] = (int32_t)v;
    }
  }
}
}  // namespace

hipError_t launch_locality_order(const float* X, int64_t n, int32_t ld, uint64_t seed,
                                 uint8_t* cell, uint32_t* hist, int32_t* order, hipStream_t s) {
  const int32_t ds = (ld < kOrderDims ? ld : kOrderDims) & ~3;
  hipLaunchKernelGGL(k_cell, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n, ld, ds,
                     seed, cell);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_clear(hist, kOrderPivots, nullptr, nullptr, nullptr, s)) != hipSuccess) return e;
  const unsigned nb = (unsigned)((n + 4095) / 4096);
  hipLaunchKernelGGL(k_cell_hist, dim3(nb), dim3(256), 0, s, cell, n, hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(kOrderPivots), 0, s, hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_place, dim3(nb), dim3(256), 0, s, cell, n, hist, order);
  return hipGetLastError();
}

}  // namespace grnnd
