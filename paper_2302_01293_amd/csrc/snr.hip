// snr.hip — spectroscopic S/N of QLP Data Release Notes 003, Sec. 2.2 item 1:
// Eq. 1, S/N(f) = (SR(f) - trend) / sigma_SR, with its two changes:
//   * the trend is the spectrum median-binned into N = round(1 + 3.322 log10 n)
//     bins (Sturges' rule, footnote) and interpolated to every frequency;
//   * sigma_SR = 1.4826 x the median absolute deviation.
// Readings (where the note is silent): equal-width bins in frequency between the
// first and last grid frequency, knot at each non-empty bin's centre, linear
// interpolation held constant beyond the first/last knot, MAD of the detrended
// residual about its median, even counts take the mean of the middle two, first
// index wins ties of the maximum.
//
// One workgroup per star.  Medians are exact order statistics found by an 8-bit
// radix select on the FP64 bit patterns (an order-preserving integer key), with
// the counting done in an LDS histogram.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "plan.hpp"

namespace mi355bls {

namespace {

__device__ __forceinline__ void grid_point_s(const StarDesc& d, int64_t i, int32_t noverlap, double& f,
                                             int32_t& nb) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  const double uu = u * u;
  f = uu * u;
  nb = static_cast<int32_t>(ceil(static_cast<double>(noverlap) / (d.kq * uu)));
}

__device__ __forceinline__ double freq_s(const StarDesc& d, int64_t i) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  return (u * u) * u;
}

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

__global__ void __launch_bounds__(kThreads) k_snr(const StarDesc* __restrict__ stars, const double* __restrict__ sr_all,
                                                  const bls_best* __restrict__ best_all, double* __restrict__ snr_all,
                                                  double* __restrict__ rho_all, bls_result* __restrict__ res_all,
                                                  Consts c) {
  __shared__ SelShared sh;
  __shared__ int64_t s_start[kMaxSturges + 1];
  __shared__ double s_kx[kMaxSturges], s_ky[kMaxSturges];
  __shared__ int s_nk;
  __shared__ ArgMax s_red[16];
  const int tid = threadIdx.x, T = blockDim.x;
  const StarDesc d = stars[blockIdx.x];
  const int64_t nf = d.nf;
  const double* __restrict__ sr = sr_all + d.f_off;
  double* __restrict__ rho = rho_all + d.f_off;
  const int nbins = d.sturges;
  const double f0 = freq_s(d, 0);
  const double span = freq_s(d, nf - 1) - f0;
  auto bin_of = [&](int64_t i) -> int {
    int k = 0;
    if (span > 0.0) k = static_cast<int>(floor(((freq_s(d, i) - f0) / span) * static_cast<double>(nbins)));
    if (k >= nbins) k = nbins - 1;
    if (k < 0) k = 0;
    return k;
  };
  // Bin b covers indices [s_start[b], s_start[b+1]) (bins are monotone in i).
  for (int b = tid; b <= nbins; b += T) s_start[b] = nf;
  __syncthreads();
  for (int64_t i = tid; i < nf; i += T) {
    const int k = bin_of(i);
    const int kp = i > 0 ? bin_of(i - 1) : -1;
    for (int b = kp + 1; b <= k; ++b) s_start[b] = i;
  }
  __syncthreads();
  if (tid == 0) s_nk = 0;
  __syncthreads();
  auto srv = [&](int64_t i) { return sr[i]; };
  for (int b = 0; b < nbins; ++b) {
    const int64_t lo = s_start[b], hi = s_start[b + 1];
    if (hi <= lo) continue;
    const double med = block_median(srv, lo, hi, sh);
    if (tid == 0) {
      s_kx[s_nk] = f0 + ((static_cast<double>(b) + 0.5) * span) / static_cast<double>(nbins);
      s_ky[s_nk] = med;
      s_nk = s_nk + 1;
    }
    __syncthreads();
  }
  const int nk = s_nk;
  // Trend by linear interpolation, residual rho = SR - trend.
  auto trend_at = [&](double f) -> double {
    if (f <= s_kx[0]) return s_ky[0];
    if (f >= s_kx[nk - 1]) return s_ky[nk - 1];
    int q = 0;
    while (q + 1 < nk && s_kx[q + 1] <= f) ++q;
    const double slope = (s_ky[q + 1] - s_ky[q]) / (s_kx[q + 1] - s_kx[q]);
    return slope * (f - s_kx[q]) + s_ky[q];
  };
  for (int64_t i = tid; i < nf; i += T) rho[i] = sr[i] - trend_at(freq_s(d, i));
  __syncthreads();
  auto rhov = [&](int64_t i) { return rho[i]; };
  double med, sigma;
  if (c.mad_of_raw) {
    med = block_median(srv, 0, nf, sh);
    auto dev = [&](int64_t i) { return fabs(sr[i] - med); };
    sigma = 1.4826 * block_median(dev, 0, nf, sh);
  } else {
    med = block_median(rhov, 0, nf, sh);
    auto dev = [&](int64_t i) { return fabs(rho[i] - med); };
    sigma = 1.4826 * block_median(dev, 0, nf, sh);
  }
  const int status = (!(sigma > 0.0) || isinf(sigma)) ? 1 : 0;
  ArgMax bs{-INFINITY, 0}, bsr{-INFINITY, 0};
  for (int64_t i = tid; i < nf; i += T) {
    const double v = status ? 0.0 : rho[i] / sigma;
    if (snr_all) snr_all[d.f_off + i] = v;
    bs = amax(bs, ArgMax{v, i});
    bsr = amax(bsr, ArgMax{sr[i], i});
  }
  bs = block_argmax(bs, s_red);
  bsr = block_argmax(bsr, s_red);
  if (tid == 0) {
    bls_result r;
    const int64_t i = bs.i;
    double f;
    int32_t nb;
    grid_point_s(d, i, c.noverlap, f, nb);
    r.i_snr = i;
    r.i_sr = bsr.i;
    r.period = 1.0 / f;
    r.sr = sr[i];
    r.snr = bs.v;
    r.trend = trend_at(f);
    r.sigma = sigma;
    r.status = status;
    r.nbins = nbins;
    r.t0 = r.duration = r.depth = NAN;
    if (best_all) {
      const bls_best b = best_all[d.f_off + i];
      if (b.j >= 0) {
        double ph = (static_cast<double>(b.j) + 0.5 * static_cast<double>(b.m)) / static_cast<double>(nb);
        ph = ph - floor(ph);
        r.t0 = d.t0 + ph / f;
        r.duration = (static_cast<double>(b.m) / static_cast<double>(nb)) / f;
        r.depth = -b.s / (b.r * (1.0 - b.r));
      }
    }
    res_all[blockIdx.x] = r;
  }
}

}  // namespace mi355bls

using namespace mi355bls;

extern "C" bls_status bls_snr(bls_plan* plan, void* ws, const double* d_sr, const bls_best* d_best,
                              double* d_snr, bls_result* d_result, bls_stream_t stream) {
  if (!plan || !d_sr || !d_result) return BLS_E_ARG;
  if (!ws || plan->uploaded_to != ws) return BLS_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const Layout& L = plan->layout;
  hipLaunchKernelGGL(k_snr, dim3(plan->n_stars), dim3(kThreads), 0, st,
                     reinterpret_cast<const StarDesc*>(base + L.stars), d_sr, d_best, d_snr,
                     reinterpret_cast<double*>(base + L.rho), d_result, plan->consts);
  if (hipGetLastError() != hipSuccess) return BLS_E_HIP;
  return BLS_OK;
}
