// round_bf16.hip -- the round kernels with BF16 distance tiles.
#include "round_impl.hpp"

namespace grnnd {

hipError_t launch_round_bf16(const RoundArgs& a, int metric, bool final_pass, bool compact_pools,
                              hipStream_t s) {
  return launch_round_prec<GRNND_PREC_BF16>(a, metric, final_pass, compact_pools, s);
}

hipError_t launch_probe_bf16(const RoundArgs& a, int metric, const int32_t* ids, int64_t nv,
                              float* t, float* b, float* c, hipStream_t s) {
  return launch_tile_probe_prec<GRNND_PREC_BF16>(a, metric, ids, nv, t, b, c, s);
}

}  // namespace grnnd
