// items.hpp -- device side of the item sink shared by the update round and
// the reverse pass (the layout is described with ItemSink in launch.hpp).
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace grnnd {

// A redirected candidate whose key is left to the destination's merge is
// sent with this key word, a NaN that no distance between finite rows
// produces; the merge gives it the canonical distance d(destination,
// candidate) unless the destination already holds the candidate with a key.
constexpr uint32_t kDeferredKey = 0x7FFFFFFFu;

__device__ __forceinline__ uint2 item_pack(int cand, float key) {
  return make_uint2((uint32_t)cand, __float_as_uint(key));
}

// Every lane with `send` set delivers (cand, key) to vertex dst, whose slot
// counter it has already advanced (slot = the value before its increment).
// Slots below bcap land in dst's bucket; the rest are appended to the
// overflow list with one counter update per wave.
__device__ __forceinline__ void send_items(const ItemSink& S, bool send, int dst, uint32_t slot,
                                           int cand, float key, int lane) {
  const bool over = send && slot >= (uint32_t)S.bcap;
  if (send && !over) S.bkt[(int64_t)dst * S.bcap + slot] = item_pack(cand, key);
  const uint64_t om = ballot(over);
  if (om) {
    const int lead = __ffsll((long long)om) - 1;
    uint32_t base = 0;
    if (lane == lead) base = atomicAdd(S.ovf_n, (uint32_t)__popcll(om));
    base = (uint32_t)__shfl((int)base, lead);
    if (over)
      S.ovf[base + (uint32_t)__popcll(om & lanemask_lt(lane))] =
          make_uint4((uint32_t)dst, slot - (uint32_t)S.bcap, (uint32_t)cand, __float_as_uint(key));
  }
}

}  // namespace grnnd
