// round_ip.hip -- the round kernels with FP32 tiles for the inner-product
// metric (a unit of its own so that the FP32 instances compile in parallel).
#include "round_impl.hpp"

namespace grnnd {

hipError_t launch_round_fp32_ip(const RoundArgs& a, bool final_pass, bool compact_pools,
                                hipStream_t s) {
  return launch_round_pm<GRNND_PREC_FP32, 1>(a, final_pass, compact_pools, s);
}

}  // namespace grnnd
