// Sorting one window of block descriptors in LDS (unplanned block lists).
#pragma once

#include "common.hpp"

namespace ta {

// Ascending bitonic sort of the W keys in skey by the 256 threads of the
// workgroup (W a power of two, at least 512).  The caller makes every key
// distinct (position in the low bits), so equal configurations keep list
// order.  Starts with a barrier and ends without one: the caller
// synchronises before reading the result.
template <int W>
TA_DEV void bitonic_sort_window(uint32_t* skey, int tid) {
#pragma unroll 1
  for (int k = 2; k <= W; k <<= 1)
#pragma unroll 1
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < W / 512; ++r) {
        const int pr = tid + r * 256;                        // pair index
        const int lo = ((pr & ~(j - 1)) << 1) | (pr & (j - 1)), hi = lo + j;
        const uint32_t x = skey[lo], y = skey[hi];
        if ((x > y) == ((lo & k) == 0)) {
          skey[lo] = y;
          skey[hi] = x;
        }
      }
    }
}

}  // namespace ta
