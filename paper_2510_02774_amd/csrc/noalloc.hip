// noalloc.hip -- grnnd_build_noalloc: a construction whose scratch memory is
// a static device array of the library instead of a caller workspace.
//
// In host code the name `scratch` stands for a host-side shadow, not for the
// device memory: its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per GPU and kept in g_scratch; only that
// address is ever passed on.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "grnnd.h"

namespace grnnd {
int set_error(int code, const char* msg);  // api.cpp: the thread's last-error text
}

static __device__ __align__(256) unsigned char scratch[GRNND_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` per GPU

int nfail(int code, const char* fmt, long long a, long long b) {
  char buf[256];
  snprintf(buf, sizeof buf, fmt, a, b);
  return grnnd::set_error(code, buf);
}

// Device address of the scratch array on the current GPU (looked up on the
// first call on that GPU, with it current).
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return nfail(GRNND_EDEVICE, "hipGetDevice failed (%lld)%lld", (long long)e, 0);
  if (dev < 0 || dev >= kMaxDevices)
    return nfail(GRNND_ENOTSUP, "device %lld beyond the %lld the scratch table holds", dev,
                 kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return nfail(GRNND_EDEVICE, "hipGetSymbolAddress(scratch) failed (%lld) on device %lld",
                   (long long)e, dev);
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GRNND_OK;
}

}  // namespace

extern "C" int grnnd_build_noalloc(const float* points, int64_t n, int32_t d, int32_t metric,
                                   int32_t R, const grnnd_params* p, uint64_t seed,
                                   int32_t* out_adj, float* out_keys, uint64_t* dev_stats,
                                   void* stream) {
  size_t need = 0;
  int rc = grnnd_workspace_size(n, d, R, p, &need);
  if (rc) return rc;
  if (need > GRNND_NOALLOC_SCRATCH_BYTES)
    return nfail(GRNND_ENOSPACE,
                 "this build needs %lld B of scratch; the allocation-free entry point holds %lld B "
                 "(use grnnd_build_ex with a workspace)",
                 (long long)need, (long long)GRNND_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((rc = scratch_ptr(&ws))) return rc;
  return grnnd_build_ex(points, n, d, metric, R, p, seed, out_adj, out_keys, dev_stats, ws,
                        GRNND_NOALLOC_SCRATCH_BYTES, stream);
}
