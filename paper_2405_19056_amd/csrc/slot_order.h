// Canonical per-pixel order of the transparency slots (device helpers).
//
// Eq. (5) pools h over the slots with a sum, a symmetric function, so the
// method's result does not depend on the order of the transparency buffers
// (Sec. 3.3; the order-inversion table of Sec. 4.3 reports no difference at
// all).  A floating-point sum does depend on the order its terms are added
// in, by a rounding.  Every path that pools in canonical order therefore
// adds a pixel's slots in an order that depends only on the multiset of its
// slot records, which makes the result bitwise the same under any
// permutation of the slots, in every precision.
//
// The order: active slots (alpha > 0) first, by the bits of alpha as an
// unsigned integer (positive floats order like their bit patterns); equal
// alphas by the bit patterns of planes 0, 1, ..., 11 in turn; bitwise equal
// records by index (their terms are identical, so swapping them cannot
// change the sum).  Inactive slots follow, by index: their terms are
// exactly zero wherever they sit.
#pragma once

#include "gn_internal.h"

namespace gn {

constexpr uint32_t kInactiveKey = 0xFFFFFFFFu;

// Sort key of a slot from its alpha (NaN and alpha <= 0: inactive).
__device__ __forceinline__ uint32_t slot_key(float alpha) {
  return alpha > 0.0f ? __float_as_uint(alpha) : kInactiveKey;
}

// Whether slot j precedes slot i in the canonical order.  L points at the
// pixel's plane 0 of slot 0; plane c of slot s is L[(s * kNL + c) * hw].
// The records are read only when two active slots have the same alpha.
template <class P>
__device__ __forceinline__ bool slot_before(P L, size_t hw, int j, int i, uint32_t kj,
                                            uint32_t ki) {
  if (kj != ki) return kj < ki;
  if (ki != kInactiveKey) {
    for (int c = 0; c < kNL; ++c) {
      const uint32_t a = __float_as_uint(L[((size_t)j * kNL + c) * hw]);
      const uint32_t b = __float_as_uint(L[((size_t)i * kNL + c) * hw]);
      if (a != b) return a < b;
    }
  }
  return j < i;
}

// Whether slot i of the pixel takes part in the pool (alpha > 0).
template <class P>
__device__ __forceinline__ bool slot_active(P L, int hw, int i) {
  return slot_key(L[((size_t)i * kNL + kAlpha) * (size_t)hw]) != kInactiveKey;
}

// Position of slot i in the canonical order among the pixel's k slots.
template <class P>
__device__ __forceinline__ int slot_rank(P L, size_t hw, int k, int i) {
  const uint32_t ki = slot_key(L[((size_t)i * kNL + kAlpha) * hw]);
  int r = 0;
  for (int j = 0; j < k; ++j)
    if (j != i) r += slot_before(L, hw, j, i, slot_key(L[((size_t)j * kNL + kAlpha) * hw]), ki);
  return r;
}

}  // namespace gn
