// counts.hpp — counts of weighted points for stars of equal weights.
//
// When every point of nonzero weight carries the same fixed-point weight u, the
// exclusive prefix sum of the weights is CW[n] = u c[n], c[n] the number of such
// points before n (c < 2^31).  The search kernels then accumulate c in 32 bits
// (cheaper LDS atomics; differences of counts are exact modulo 2^32) and multiply
// bin or window totals back by u, which gives the same integers as the prefixes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mi355bls {

// Exact division of a weight prefix v = c u by u (c < 2^32): with u = 2^shift odd,
// v >> shift = c odd, and multiplying by the inverse of odd modulo 2^32 leaves c
// modulo 2^32, which is c.  The inverse comes from Newton's iteration
// x <- x (2 - odd x), which doubles the number of correct low bits from the 3 of
// x = odd.
struct CountDiv {
  uint32_t shift, inv;
};

__device__ __forceinline__ CountDiv count_div(int64_t unit) {
  const uint64_t u = static_cast<uint64_t>(unit);
  const uint32_t t = static_cast<uint32_t>(__builtin_ctzll(u));
  const uint32_t odd = static_cast<uint32_t>(u >> t);
  uint32_t x = odd;
  for (int i = 0; i < 4; ++i) x *= 2u - odd * x;
  return CountDiv{t, x};
}

__device__ __forceinline__ uint32_t count_of(long long v, CountDiv c) {
  return static_cast<uint32_t>(static_cast<uint64_t>(v) >> c.shift) * c.inv;
}

}  // namespace mi355bls
