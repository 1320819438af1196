// Batched launches: one launch runs a kernel for several same-shape members
// of a batch plan (continuous batching of simulations).  Member m's
// workspace is member 0's shifted by m * stride bytes, so every workspace
// pointer of a member is member 0's plus one offset; blockIdx.z selects the
// descriptor, and a descriptor whose member is negative makes its blocks
// return at once.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "pm.h"

namespace pmk {

struct BatchArg {
  const pm_req_desc* d = nullptr;   // device descriptors, one per blockIdx.z; null: unbatched
  long stride = 0;                  // bytes between consecutive members' workspaces
  int n = 1;                        // descriptors (the grid's z extent)
};

// Byte offset of the workspace of this block's member, or -1 when its
// descriptor is skipped.  Uniform over the block.
__device__ __forceinline__ long batch_bytes(const BatchArg& b) {
  if (!b.d) return 0;
  const int m = b.d[blockIdx.z].member;
  return m < 0 ? -1L : (long)m * b.stride;
}

// p shifted by `bytes`, through char pointer arithmetic: a round trip
// through an integer would hide from the compiler that p points to global
// memory and turn every access through the result into a (slower) flat one.
template <class T>
__host__ __device__ __forceinline__ T* byte_adv(T* p, long bytes) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<C*>(p) + bytes) : p;
}

}  // namespace pmk
