// round_bf16.hip -- the round kernels with BF16 distance tiles.
#include "round_impl.hpp"

namespace grnnd {

hipError_t launch_round_bf16(const RoundArgs& a, int metric, bool final_pass, bool compact_pools,
                              hipStream_t s) {
  return launch_round_prec<GRNND_PREC_BF16>(a, metric, final_pass, compact_pools, s);
}

}  // namespace grnnd
