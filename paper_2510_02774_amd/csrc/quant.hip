// quant.hip -- reduced-precision copies of the points for the distance tile.
//
// For a BF16, FP16 or FP8-e4m3 tile the round kernels gather a narrow copy of
// the points instead of the FP32 rows: y = x - c (c = the column means rounded
// to integers for L2, which keeps integer-valued data exact; c = 0 for the
// inner product, which is not translation invariant), stored as q with y ~ s q
// (s = 1 for BF16/FP16; for FP8 a power of two per row, so that max |y| / s
// <= 448). For every row the conversion also records upper bounds, in FP32,
//   eps >= || s q - (x - c) ||_2   and   nrm >= || x - c ||_2,
// from exact per-element differences (two-sum) and FP32 sums whose rounding
// the bound absorbs; no step needs FP64. The tile's error against
// the exact distance is then bounded per pair by these two numbers (plus the
// FP32 accumulation term), which is what lets the round kernels re-decide
// every comparison inside the bound with the canonical FP32 distance and so
// reach exactly the decisions of the FP32 tile.
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

namespace {

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// An upper bound on sqrt(S_true) from S, an FP32 sum of m non-negative
// rounded terms taken over at most 2^12 / 64 + 6 additions per lane and tree
// level: |S - S_true| <= (m + 2) u S_true with u = 2^-24, so inflating the
// root by 1e-5 (more than (m + 2) u for every row length allowed) and
// rounding up covers it.
__device__ __forceinline__ float root_upper(float S) {
  return S == 0.0f ? 0.0f : nextafterf(sqrtf(S) * 1.00001f, INFINITY);  // 0 stays exact
}

// Column sums of X in FP32 in a fixed order, one partial row per block (rows
// split evenly): the centre only needs to be the same on every run.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ X, int64_t n, int32_t d,
                                                int32_t ld, float* __restrict__ part) {
  const int64_t r0 = n * blockIdx.x / gridDim.x, r1 = n * (blockIdx.x + 1) / gridDim.x;
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += X[r * ld + j];
    part[(int64_t)blockIdx.x * d + j] = s;
  }
}

// c_j = the column mean rounded to the nearest integer.
__global__ __launch_bounds__(256) void k_center(const float* __restrict__ part, int nparts,
                                                int64_t n, int32_t d, float* __restrict__ c) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d; j += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * d + j];
    c[j] = nearbyintf(s / (float)n);
  }
}

// One wave per row: narrow copy (ldr elements, zero padded), scale, eps, nrm.
template <int PREC>
__global__ __launch_bounds__(64) void k_quantize(const float* __restrict__ X, int64_t n, int32_t d,
                                                 int32_t ld, const float* __restrict__ c,
                                                 void* __restrict__ Xr, int32_t ldr,
                                                 float* __restrict__ rscale,
                                                 float2* __restrict__ rinfo) {
  const int64_t v = blockIdx.x;
  const int lane = threadIdx.x;
  const float* x = X + v * ld;
  float s = 1.0f;
  if (PREC == GRNND_PREC_FP8_E4M3) {
    float amax = 0.0f;
    for (int e = lane; e < d; e += kWave) amax = fmaxf(amax, fabsf(x[e] - (c ? c[e] : 0.0f)));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
    if (amax > 0.0f) {
      int ex;
      frexpf(amax / 448.0f, &ex);  // amax / 448 < 2^ex
      s = ldexpf(1.0f, ex);
    }
    if (lane == 0) rscale[v] = s;
  }
  // eps: the element's error against the exact x - c is (back - y) + (y -
  // (x - c)); back - y is exact (back is y rounded to fewer bits, within a
  // factor of two of it, or 0), and y - (x - c) is the exact rounding error of
  // the subtraction (two-sum). Squares and sums are FP32, covered by
  // root_upper.
  float err = 0.0f, nrm = 0.0f;
  for (int e = lane; e < ldr; e += kWave) {
    const float xv = e < d ? x[e] : 0.0f;
    const float cv = (e < d && c) ? -c[e] : 0.0f;
    const float y = xv + cv;
    const float bb = y - xv;
    const float re = (xv - (y - bb)) + (cv - bb);  // (x - c) - y, exactly
    float back;
    if (PREC == GRNND_PREC_BF16) {
      const uint16_t q = to_bf16(y);
      static_cast<uint16_t*>(Xr)[v * ldr + e] = q;
      back = from_bf16(q);
    } else if (PREC == GRNND_PREC_FP16) {
      const _Float16 q = (_Float16)y;
      static_cast<_Float16*>(Xr)[v * ldr + e] = q;
      back = (float)q;
    } else {
      const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(y / s, 0.0f, 0, false);
      static_cast<uint8_t*>(Xr)[v * ldr + e] = (uint8_t)(pk & 0xFF);
      back = __builtin_amdgcn_cvt_f32_fp8(pk, 0) * s;
    }
    const float df = fabsf(back - y) + fabsf(re);  // >= |back - (x - c)|
    err += df * df;
    const float ay = fabsf(y) + fabsf(re);  // >= |x - c|
    nrm += ay * ay;
  }
  err = wave_sum(err);
  nrm = wave_sum(nrm);
  if (lane == 0) rinfo[v] = make_float2(root_upper(err), root_upper(nrm));
}

template <int PREC>
hipError_t launch_quantize_t(const float* X, int64_t n, int32_t d, int32_t ld, const float* c,
                             void* Xr, int32_t ldr, float* rscale, float2* rinfo, hipStream_t s) {
  hipLaunchKernelGGL((k_quantize<PREC>), dim3((unsigned)n), dim3(64), 0, s, X, n, d, ld, c, Xr,
                     ldr, rscale, rinfo);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_quantize(const float* X, int64_t n, int32_t d, int32_t ld, int metric, int prec,
                           float* part, float* center, void* Xr, int32_t ldr, float* rscale,
                           float2* rinfo, hipStream_t s) {
  const float* c = nullptr;
  if (metric == GRNND_METRIC_L2) {
    constexpr int kParts = 256;
    hipLaunchKernelGGL(k_colsum, dim3(kParts), dim3(256), 0, s, X, n, d, ld, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_center, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s, part, kParts,
                       n, d, center);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    c = center;
  }
  switch (prec) {
    case GRNND_PREC_BF16:
      return launch_quantize_t<GRNND_PREC_BF16>(X, n, d, ld, c, Xr, ldr, rscale, rinfo, s);
    case GRNND_PREC_FP16:
      return launch_quantize_t<GRNND_PREC_FP16>(X, n, d, ld, c, Xr, ldr, rscale, rinfo, s);
    default:
      return launch_quantize_t<GRNND_PREC_FP8_E4M3>(X, n, d, ld, c, Xr, ldr, rscale, rinfo, s);
  }
}

}  // namespace grnnd
