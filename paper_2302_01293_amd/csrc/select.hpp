// select.hpp — workgroup-wide exact order statistics and argmax on doubles
// (device code shared by the S/N and resampling kernels).
//
// Medians are exact order statistics of the FP64 values through an order-preserving
// integer key: histogram passes over the remaining key range (up to 2048 buckets
// each) narrow it down until the bucket that holds the rank is small, and that
// bucket is ranked exactly in LDS.
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

constexpr int kSelBuckets = 2048;  // histogram buckets per pass (11 bits of key range)
constexpr int kSelUnroll = 4;      // values loaded per thread before any is used (loads in flight)
constexpr int kSelCap = 1024;      // candidates finished in LDS

struct SelShared {
  unsigned int hist[kSelBuckets];
  unsigned long long cand[kSelCap];
  unsigned long long red[32];
  long long wsum[16];
  unsigned long long kmin, kmax, lo_key, key_a, key_b;
  long long rank;
  unsigned int ncand, bcount;
  int bucket, shift;
};

// The bucket (of hist[0, nb)) holding rank r, the rank within it and its count, by
// a block-wide prefix sum: thread t owns buckets [t B, t B + B).
__device__ __forceinline__ void find_bucket(int nb, long long r, SelShared& sh) {
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int B = (nb + T - 1) / T;
  const int b0 = tid * B;
  long long mine = 0;
  for (int q = 0; q < B; ++q)
    if (b0 + q < nb) mine += sh.hist[b0 + q];
  long long incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) sh.wsum[wave] = incl;
  __syncthreads();
  long long before = 0;
  for (int w = 0; w < wave; ++w) before += sh.wsum[w];
  const long long excl = before + incl - mine;
  if (mine > 0 && r >= excl && r < excl + mine) {
    long long acc = excl;
    int b = b0;
    while (acc + static_cast<long long>(sh.hist[b]) <= r) acc += sh.hist[b++];
    sh.bucket = b;
    sh.rank = r - acc;
    sh.bcount = sh.hist[b];
  }
  if (tid == 0) sh.ncand = 0;
  __syncthreads();
}

// Keys of v(base + u T + tid), u < kSelUnroll, for the indices below hi (ok[u]); all
// loads are issued before the first key is formed, so a pass waits on its loads once
// per kSelUnroll values instead of once per value.
template <typename F>
__device__ __forceinline__ void load_keys(F v, int64_t base, int64_t hi, unsigned long long (&k)[kSelUnroll],
                                          bool (&ok)[kSelUnroll]) {
  const int64_t T = blockDim.x, tid = threadIdx.x;
  double x[kSelUnroll];
#pragma unroll
  for (int u = 0; u < kSelUnroll; ++u) {
    const int64_t i = base + u * T + tid;
    ok[u] = i < hi;
    x[u] = ok[u] ? v(i) : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kSelUnroll; ++u) k[u] = key_of(x[u]);
}

// Block-wide minimum and maximum of the keys of v(i), i in [lo, hi).
template <typename F>
__device__ void block_key_range(F v, int64_t lo, int64_t hi, SelShared& sh) {
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, wave = tid >> 6;
  unsigned long long mn = ~0ull, mx = 0ull;
  for (int64_t b0 = lo; b0 < hi; b0 += static_cast<int64_t>(kSelUnroll) * T) {
    unsigned long long k[kSelUnroll];
    bool ok[kSelUnroll];
    load_keys(v, b0, hi, k, ok);
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u) {
      if (ok[u]) {
        mn = k[u] < mn ? k[u] : mn;
        mx = k[u] > mx ? k[u] : mx;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (lane == 0) {
    sh.red[wave] = mn;
    sh.red[16 + wave] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long a = ~0ull, b = 0ull;
    for (int q = 0; q < (T >> 6); ++q) {
      a = sh.red[q] < a ? sh.red[q] : a;
      b = sh.red[16 + q] > b ? sh.red[16 + q] : b;
    }
    sh.kmin = a;
    sh.kmax = b;
  }
  __syncthreads();
}

// The rank-th smallest (0-based) of v(i) for i in [lo, hi), exact, and with `pair`
// also the (rank+1)-th.  Keys are the order-preserving integer images of the
// doubles.  A pass histograms the keys inside the current key range [base, base +
// span] into 64-2048 buckets of equal width (about one per two keys: the range's
// top bits); the bucket that holds the rank becomes the range.  As soon as that
// bucket is small (at most 64 keys, or few enough that ranking them all pairwise
// costs about as much as a pass over the data, and never more than kSelCap) its keys
// are gathered into LDS and ranked there exactly (ties by LDS slot).
// A value range of 2^64 keys needs at most six histogram passes; typical spectra
// take one (min/max, histogram, gather: three passes over the data).
template <typename F>
__device__ void block_select_keys(F v, int64_t lo, int64_t hi, int64_t rank, bool pair, SelShared& sh,
                                  unsigned long long& out_a, unsigned long long& out_b) {
  const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63;
  block_key_range(v, lo, hi, sh);
  unsigned long long base = sh.kmin;
  unsigned long long span = sh.kmax - sh.kmin;  // keys in [base, base + span]
  long long r = rank;
  long long cnt_in = hi - lo;                   // keys inside the range
  for (;;) {
    if (span == 0) {  // every remaining key is equal
      out_a = out_b = base;
      return;
    }
    // buckets: about one per two remaining keys, 64 to 2048 (the range's top bits)
    int lbk = 6;
    while (lbk < 11 && (1ll << (lbk + 1)) < 2 * static_cast<long long>(cnt_in)) ++lbk;
    const int bits = 64 - __clzll(static_cast<long long>(span));
    const int shift = bits > lbk ? bits - lbk : 0;
    const int nb = static_cast<int>(span >> shift) + 1;
    for (int q = tid; q < nb; q += T) sh.hist[q] = 0;
    __syncthreads();
    for (int64_t b0 = lo; b0 < hi; b0 += static_cast<int64_t>(kSelUnroll) * T) {
      unsigned long long kk[kSelUnroll];
      bool ok[kSelUnroll];
      load_keys(v, b0, hi, kk, ok);
#pragma unroll
      for (int u = 0; u < kSelUnroll; ++u) {
        const unsigned long long k = kk[u];
        const bool take = ok[u] && k >= base && k - base <= span;
        const int bk = take ? static_cast<int>((k - base) >> shift) : 0;
        // a wave whose keys share one bucket adds its count once
        const unsigned long long m = __ballot(take);
        if (m) {
          const int leader = __ffsll(static_cast<long long>(m)) - 1;
          const int lb = __shfl(bk, leader, 64);
          if (__ballot(take && bk == lb) == m) {
            if (lane == leader) atomicAdd(&sh.hist[lb], static_cast<unsigned>(__popcll(m)));
          } else if (take) {
            atomicAdd(&sh.hist[bk], 1u);
          }
        }
      }
    }
    __syncthreads();
    find_bucket(nb, r, sh);
    const int b = sh.bucket;
    r = sh.rank;
    const unsigned int cnt = sh.bcount;
    const unsigned long long blo = base + (static_cast<unsigned long long>(b) << shift);
    const unsigned long long bspan =
        shift == 0 ? 0ull : ((static_cast<unsigned long long>(b) + 1 == static_cast<unsigned long long>(nb))
                                 ? (base + span) - blo
                                 : ((1ull << shift) - 1ull));
    __syncthreads();
    // gather when ranking the bucket in LDS (cnt^2 / T compares per thread) costs
    // no more than a few passes over the data (n / T reads per thread)
    const bool gather = cnt <= static_cast<unsigned>(kSelCap) &&
                        (cnt <= 64u || static_cast<long long>(cnt) * cnt <= 8 * (hi - lo));
    if (gather || shift == 0) {
      if (shift == 0) {  // one key value per bucket: the rank lies in it
        out_a = blo;
        if (pair) {
          if (r + 1 < static_cast<long long>(cnt)) {
            out_b = blo;
          } else {  // the next key above this bucket
            unsigned long long mnx = ~0ull;
            for (int64_t b0 = lo; b0 < hi; b0 += static_cast<int64_t>(kSelUnroll) * T) {
              unsigned long long kk[kSelUnroll];
              bool ok[kSelUnroll];
              load_keys(v, b0, hi, kk, ok);
#pragma unroll
              for (int u = 0; u < kSelUnroll; ++u)
                if (ok[u] && kk[u] > blo && kk[u] < mnx) mnx = kk[u];
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
              const unsigned long long a2 = __shfl_xor(mnx, o, 64);
              mnx = a2 < mnx ? a2 : mnx;
            }
            if (lane == 0) sh.red[tid >> 6] = mnx;
            __syncthreads();
            if (tid == 0) {
              unsigned long long a2 = ~0ull;
              for (int q = 0; q < (T >> 6); ++q) a2 = sh.red[q] < a2 ? sh.red[q] : a2;
              sh.key_b = a2;
            }
            __syncthreads();
            out_b = sh.key_b;
          }
        }
        __syncthreads();
        return;
      }
      // gather the bucket's keys into LDS
      for (int64_t b0 = lo; b0 < hi; b0 += static_cast<int64_t>(kSelUnroll) * T) {
        unsigned long long kk[kSelUnroll];
        bool ok[kSelUnroll];
        load_keys(v, b0, hi, kk, ok);
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
          if (ok[u] && kk[u] >= blo && kk[u] - blo <= bspan) {
            const unsigned int slot = atomicAdd(&sh.ncand, 1u);
            sh.cand[slot] = kk[u];
          }
        }
      }
      __syncthreads();
      const int nc = static_cast<int>(sh.ncand);
      // rank every candidate: smaller keys, and equal keys at lower slots
      for (int c = tid; c < nc; c += T) {
        const unsigned long long k = sh.cand[c];
        int less = 0;
        for (int e = 0; e < nc; ++e) {
          const unsigned long long x = sh.cand[e];
          less += (x < k || (x == k && e < c)) ? 1 : 0;
        }
        if (less == r) sh.key_a = k;
        if (pair && less == r + 1) sh.key_b = k;
      }
      __syncthreads();
      out_a = sh.key_a;
      if (pair) {
        if (r + 1 < nc) {
          out_b = sh.key_b;
        } else {  // the next key above this bucket
          unsigned long long mnx = ~0ull;
          const unsigned long long top = blo + bspan;
          for (int64_t b0 = lo; b0 < hi; b0 += static_cast<int64_t>(kSelUnroll) * T) {
            unsigned long long kk[kSelUnroll];
            bool ok[kSelUnroll];
            load_keys(v, b0, hi, kk, ok);
#pragma unroll
            for (int u = 0; u < kSelUnroll; ++u)
              if (ok[u] && kk[u] > top && kk[u] < mnx) mnx = kk[u];
          }
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long a2 = __shfl_xor(mnx, o, 64);
            mnx = a2 < mnx ? a2 : mnx;
          }
          if (lane == 0) sh.red[tid >> 6] = mnx;
          __syncthreads();
          if (tid == 0) {
            unsigned long long a2 = ~0ull;
            for (int q = 0; q < (T >> 6); ++q) a2 = sh.red[q] < a2 ? sh.red[q] : a2;
            sh.key_b = a2;
          }
          __syncthreads();
          out_b = sh.key_b;
        }
      }
      __syncthreads();
      return;
    }
    base = blo;
    span = bspan;
    cnt_in = cnt;
  }
}

template <typename F>
__device__ double block_select(F v, int64_t lo, int64_t hi, int64_t rank, SelShared& sh) {
  unsigned long long a, b;
  block_select_keys(v, lo, hi, rank, false, sh, a, b);
  return value_of(a);
}

template <typename F>
__device__ double block_median(F v, int64_t lo, int64_t hi, SelShared& sh) {
  const int64_t c = hi - lo;
  unsigned long long a, b;
  if (c & 1) {
    block_select_keys(v, lo, hi, c / 2, false, sh, a, b);
    return value_of(a);
  }
  block_select_keys(v, lo, hi, c / 2 - 1, true, sh, a, b);
  return (value_of(a) + value_of(b)) * 0.5;
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
