// Block-wide OR of a per-thread flag for the cost of one barrier, for the
// network's z-marching kernels (their per-plane "is this neighbourhood all
// zero" test rides on the barrier that already follows each plane store).
#pragma once

#include "common.h"

namespace fs {

// The __syncthreads_or builtin takes three barriers with LDS atomics between
// them.  Here each wave posts its vote in its word of `slot` (kBlock / kWave
// ints, 16-byte aligned), one barrier follows, then every thread reads the
// words back.  A slot is read only between its barrier and the next one, so
// callers that use two or more slots in turn never write a slot that a
// slower wave still reads.
__device__ inline int barrier_or(int v, int* slot) {
  static_assert(kBlock / kWave == 4, "one int4 of votes");
  const bool any = __ballot(v != 0) != 0ull;
  if ((threadIdx.x & (kWave - 1)) == 0) slot[threadIdx.x / kWave] = any;
  __syncthreads();
  const int4 w = *reinterpret_cast<const int4*>(slot);
  return w.x | w.y | w.z | w.w;
}

}  // namespace fs
