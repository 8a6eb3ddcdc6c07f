// select.hpp — workgroup-wide exact order statistics and argmax on doubles
// (device code shared by the S/N and resampling kernels).
//
// Medians are exact order statistics found by an 8-bit radix select on the FP64
// bit patterns (an order-preserving integer key), with the counting done in an
// LDS histogram; a wave whose lanes fall into one bucket adds its count once.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace mi355bls {
namespace {

// Order-preserving 64-bit keys of doubles (NaN excluded by construction).
__device__ __forceinline__ unsigned long long key_of(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double value_of(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double(static_cast<long long>(b));
}

struct SelShared {
  unsigned int hist[256];
  unsigned long long prefix;
  long long rank;
  int digit;
};

// The rank-th smallest (0-based) of v(i) for i in [lo, hi), exact.
template <typename F>
__device__ double block_select(F v, int64_t lo, int64_t hi, int64_t rank, SelShared& sh) {
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63;
  unsigned long long prefix = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int q = tid; q < 256; q += T) sh.hist[q] = 0;
    __syncthreads();
    const unsigned long long hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
    for (int64_t i0 = lo; i0 < hi; i0 += T) {
      const int64_t i = i0 + tid;
      bool take = false;
      int dg = 0;
      if (i < hi) {
        const unsigned long long k = key_of(v(i));
        take = (k & hmask) == (prefix & hmask);
        dg = static_cast<int>((k >> shift) & 255ull);
      }
      // Aggregate the common case where a whole wave falls into one bucket.
      const unsigned long long m = __ballot(take);
      if (m) {
        const int leader = __ffsll(static_cast<long long>(m)) - 1;
        const int ld = __shfl(dg, leader, 64);
        const unsigned long long same = __ballot(take && dg == ld);
        if (same == m) {
          if (lane == leader) atomicAdd(&sh.hist[ld], static_cast<unsigned>(__popcll(m)));
        } else if (take) {
          atomicAdd(&sh.hist[dg], 1u);
        }
      }
    }
    __syncthreads();
    if (tid < 64) {
      unsigned int c0 = sh.hist[4 * tid], c1 = sh.hist[4 * tid + 1], c2 = sh.hist[4 * tid + 2],
                   c3 = sh.hist[4 * tid + 3];
      long long mine = static_cast<long long>(c0) + c1 + c2 + c3;
      long long incl = mine;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      const long long excl = incl - mine;
      const long long r = rank;
      if (r >= excl && r < incl) {
        long long acc = excl;
        int dsel = 4 * tid;
        if (r >= acc + c0) { acc += c0; dsel++;
          if (r >= acc + c1) { acc += c1; dsel++;
            if (r >= acc + c2) { acc += c2; dsel++; } } }
        sh.digit = dsel;
        sh.rank = r - acc;
      }
    }
    __syncthreads();
    prefix |= static_cast<unsigned long long>(sh.digit) << shift;
    rank = sh.rank;
    __syncthreads();
  }
  return value_of(prefix);
}

template <typename F>
__device__ double block_median(F v, int64_t lo, int64_t hi, SelShared& sh) {
  const int64_t c = hi - lo;
  if (c & 1) return block_select(v, lo, hi, c / 2, sh);
  const double a = block_select(v, lo, hi, c / 2 - 1, sh);
  const double b = block_select(v, lo, hi, c / 2, sh);
  return (a + b) * 0.5;
}

struct ArgMax {
  double v;
  int64_t i;
};

__device__ __forceinline__ ArgMax amax(ArgMax a, ArgMax b) {
  return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}

__device__ ArgMax block_argmax(ArgMax x, ArgMax* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ArgMax y;
    y.v = __shfl_xor(x.v, o, 64);
    y.i = __shfl_xor(x.i, o, 64);
    x = amax(x, y);
  }
  __syncthreads();
  if (lane == 0) scratch[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    ArgMax r = scratch[0];
    for (int q = 1; q < (blockDim.x >> 6); ++q) r = amax(r, scratch[q]);
    scratch[0] = r;
  }
  __syncthreads();
  const ArgMax r = scratch[0];
  __syncthreads();
  return r;
}

}  // namespace
}  // namespace mi355bls
