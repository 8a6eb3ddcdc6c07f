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
// One workgroup per star: 256 threads when every spectrum of the batch is short
// (the selections are bound by their barriers, so several small groups per CU beat
// one large one), else 1024.  Medians are exact order statistics on an
// order-preserving integer key of the FP64 values (select.hpp): a key-range pass,
// histogram passes (buckets sized to the keys left) until the rank's bucket is
// small, and a gather of that bucket, ranked in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "plan.hpp"
#include "select.hpp"

namespace mi355bls {

namespace {

// Frequency i of a star's grid and the window geometry of its best-window record:
// the fine-bin count and the window length for bls_best.m (with the per-duration
// rebinning, m holds the duration index k: noverlap bins of the k-th set).
__device__ __forceinline__ void window_geometry(const StarDesc& d, int64_t i, const Consts& c, int32_t m_rec,
                                                double& f, int32_t& nb, int32_t& m) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  const double uu = u * u;
  f = uu * u;
  if (c.rebin) {
    const int32_t k = m_rec < 0 ? 0 : (m_rec >= c.n_rebin ? c.n_rebin - 1 : m_rec);
    nb = rebin_bins(qlo_at(d, c, uu), c.rebin_g[k], c.noverlap);
    m = c.noverlap;
  } else {
    nb = fine_bins(d, c, uu);
    m = m_rec;
  }
}

__device__ __forceinline__ double freq_s(const StarDesc& d, int64_t i) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  return (u * u) * u;
}

}  // namespace

// Median-binned trend of one star's SR spectrum: Sturges bins in frequency, a knot
// at the centre of every non-empty bin holding the bin's median SR.
struct TrendLds {
  SelShared sh;
  int64_t start[kMaxSturges + 1];
  double kx[kMaxSturges], ky[kMaxSturges];
  double slope[kMaxSturges];  // (ky[q+1] - ky[q]) / (kx[q+1] - kx[q]), once per knot pair
  int nk;
  ArgMax red[16];
};

__device__ void build_knots(const StarDesc& d, const double* __restrict__ sr, TrendLds& L) {
  const int tid = threadIdx.x, T = blockDim.x;
  const int64_t nf = d.nf;
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
  // Bin b covers indices [start[b], start[b+1]) (bins are monotone in i): start[b]
  // is the first index whose bin is b or more, found by a binary search over i (the
  // same bin_of as a pass over every frequency would evaluate).
  for (int b = tid; b <= nbins; b += T) {
    int64_t lo = 0, hi = nf;
    if (b == 0) {
      hi = 0;
    } else if (b == nbins) {
      lo = nf;
    } else {
      while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (bin_of(m) < b) lo = m + 1; else hi = m;
      }
    }
    L.start[b] = lo;
  }
  __syncthreads();
  if (tid == 0) L.nk = 0;
  __syncthreads();
  auto srv = [&](int64_t i) { return sr[i]; };
  for (int b = 0; b < nbins; ++b) {
    const int64_t lo = L.start[b], hi = L.start[b + 1];
    if (hi <= lo) continue;
    const double med = block_median(srv, lo, hi, L.sh);
    if (tid == 0) {
      L.kx[L.nk] = f0 + ((static_cast<double>(b) + 0.5) * span) / static_cast<double>(nbins);
      L.ky[L.nk] = med;
      L.nk = L.nk + 1;
    }
    __syncthreads();
  }
  for (int q = tid; q + 1 < L.nk; q += T) L.slope[q] = (L.ky[q + 1] - L.ky[q]) / (L.kx[q + 1] - L.kx[q]);
  __syncthreads();
}

// Linear interpolation through the knots, constant beyond the first and last.
__device__ double trend_at(const TrendLds& L, double f) {
  const int nk = L.nk;
  if (f <= L.kx[0]) return L.ky[0];
  if (f >= L.kx[nk - 1]) return L.ky[nk - 1];
  int q = 0;
  while (q + 1 < nk && L.kx[q + 1] <= f) ++q;
  return L.slope[q] * (f - L.kx[q]) + L.ky[q];
}

// Residual rho = SR - trend into the scratch array, and sigma = 1.4826 MAD.
__device__ double residual_sigma(const StarDesc& d, const double* __restrict__ sr, double* __restrict__ rho,
                                 TrendLds& L, int mad_of_raw) {
  const int tid = threadIdx.x, T = blockDim.x;
  const int64_t nf = d.nf;
  for (int64_t i = tid; i < nf; i += T) rho[i] = sr[i] - trend_at(L, freq_s(d, i));
  __syncthreads();
  auto srv = [&](int64_t i) { return sr[i]; };
  auto rhov = [&](int64_t i) { return rho[i]; };
  if (mad_of_raw) {
    const double med = block_median(srv, 0, nf, L.sh);
    auto dev = [&](int64_t i) { return fabs(sr[i] - med); };
    return 1.4826 * block_median(dev, 0, nf, L.sh);
  }
  const double med = block_median(rhov, 0, nf, L.sh);
  auto dev = [&](int64_t i) { return fabs(rho[i] - med); };
  return 1.4826 * block_median(dev, 0, nf, L.sh);
}

// Summary of the chosen frequency i of a star (period, T0, duration, depth).
__device__ bls_result make_result(const StarDesc& d, const double* sr, const bls_best* best_all, const TrendLds& L,
                                  int64_t i, int64_t i_sr, double snr, double sigma, int status, int nbins,
                                  const Consts& c) {
  bls_result r;
  double f;
  int32_t nb;
  int32_t m;
  window_geometry(d, i, c, best_all ? best_all[d.f_off + i].m : 0, f, nb, m);
  r.i_snr = i;
  r.i_sr = i_sr;
  r.period = 1.0 / f;
  r.sr = sr[i];
  r.snr = snr;
  r.trend = trend_at(L, f);
  r.sigma = sigma;
  r.status = status;
  r.nbins = nbins;
  r.t0 = r.duration = r.depth = NAN;
  if (best_all) {
    const bls_best b = best_all[d.f_off + i];
    if (b.j >= 0) {
      double ph = (static_cast<double>(b.j) + 0.5 * static_cast<double>(m)) / static_cast<double>(nb);
      ph = ph - floor(ph);
      r.t0 = d.t0 + ph / f;
      r.duration = (static_cast<double>(m) / static_cast<double>(nb)) / f;
      r.depth = -b.s / (b.r * (1.0 - b.r));
    }
  }
  return r;
}

// Plain S/N of one star over its full grid.
__device__ void snr_full(const StarDesc& d, const double* __restrict__ sr_all, const bls_best* __restrict__ best_all,
                         double* __restrict__ snr_all, double* __restrict__ rho_all, bls_result* out, const Consts& c,
                         TrendLds& L) {
  const int tid = threadIdx.x, T = blockDim.x;
  const int64_t nf = d.nf;
  const double* __restrict__ sr = sr_all + d.f_off;
  double* __restrict__ rho = rho_all + d.f_off;
  build_knots(d, sr, L);
  const double sigma = residual_sigma(d, sr, rho, L, c.mad_of_raw);
  const int status = (!(sigma > 0.0) || isinf(sigma)) ? 1 : 0;
  ArgMax bs{-INFINITY, 0}, bsr{-INFINITY, 0};
  for (int64_t i = tid; i < nf; i += T) {
    const double v = status ? 0.0 : rho[i] / sigma;
    if (snr_all) snr_all[d.f_off + i] = v;
    bs = amax(bs, ArgMax{v, i});
    bsr = amax(bsr, ArgMax{sr[i], i});
  }
  bs = block_argmax(bs, L.red);
  bsr = block_argmax(bsr, L.red);
  if (tid == 0) *out = make_result(d, sr, best_all, L, bs.i, bsr.i, bs.v, sigma, status, d.sturges, c);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_snr(const StarDesc* __restrict__ stars, const double* __restrict__ sr_all,
                                                  const bls_best* __restrict__ best_all, double* __restrict__ snr_all,
                                                  double* __restrict__ rho_all, bls_result* __restrict__ res_all,
                                                  Consts c) {
  __shared__ TrendLds L;
  const StarDesc d = stars[blockIdx.x];
  snr_full(d, sr_all, best_all, snr_all, rho_all, res_all + blockIdx.x, c, L);
}

// S/N restricted to frequency windows: trend and sigma come from a coarse spectrum
// of the same star (a grid with fewer samples per peak), and S/N = (SR - trend) /
// sigma is evaluated only at the fine frequencies inside the star's windows.  A
// star flagged for fallback has its full fine spectrum and gets the plain S/N.
template <int NT>
__global__ void __launch_bounds__(NT) k_snr_windows(
    const StarDesc* __restrict__ fine, const StarDesc* __restrict__ coarse, const double* __restrict__ sr_all,
    const bls_best* __restrict__ best_all, double* __restrict__ rho_fine, const double* __restrict__ sr_coarse_all,
    double* __restrict__ rho_coarse, const int64_t* __restrict__ windows, int32_t per_star,
    const uint8_t* __restrict__ fallback, bls_result* __restrict__ res_all, Consts c) {
  __shared__ TrendLds L;
  const int s = blockIdx.x;
  const int tid = threadIdx.x, T = blockDim.x;
  const StarDesc d = fine[s];
  if (fallback[s]) {
    snr_full(d, sr_all, best_all, nullptr, rho_fine, res_all + s, c, L);
    return;
  }
  const StarDesc dc = coarse[s];
  const double* __restrict__ src = sr_coarse_all + dc.f_off;
  build_knots(dc, src, L);
  const double sigma = residual_sigma(dc, src, rho_coarse + dc.f_off, L, c.mad_of_raw);
  const int status = (!(sigma > 0.0) || isinf(sigma)) ? 1 : 0;
  const double* __restrict__ sr = sr_all + d.f_off;
  ArgMax bs{-INFINITY, -1}, bsr{-INFINITY, -1};
  for (int q = 0; q < per_star; ++q) {
    const int64_t* w = windows + 3 * (static_cast<int64_t>(s) * per_star + q);
    if (w[0] != s) continue;
    const int64_t i0 = max<int64_t>(0, w[1]), i1 = min<int64_t>(d.nf, w[2]);
    for (int64_t i = i0 + tid; i < i1; i += T) {
      const double v = status ? 0.0 : (sr[i] - trend_at(L, freq_s(d, i))) / sigma;
      bs = amax(bs, ArgMax{v, i});
      bsr = amax(bsr, ArgMax{sr[i], i});
    }
  }
  bs = block_argmax(bs, L.red);
  bsr = block_argmax(bsr, L.red);
  if (tid == 0) {
    if (bs.i < 0) {  // no window frequency: nothing searched
      bls_result r = make_result(d, sr, nullptr, L, 0, 0, 0.0, sigma, 2, dc.sturges, c);
      r.sr = 0.0;
      res_all[s] = r;
    } else {
      res_all[s] = make_result(d, sr, best_all, L, bs.i, bsr.i, bs.v, sigma, status, dc.sturges, c);
    }
  }
}

}  // namespace mi355bls

using namespace mi355bls;

namespace {
// The selections of the S/N step are bound by their barriers: small workgroups (more
// of them per CU) suit batches of short spectra, large ones long spectra.
bool snr_small_groups(const bls_plan* plan) {
  int64_t nf_max = 0;
  for (const StarDesc& d : plan->stars) nf_max = std::max<int64_t>(nf_max, d.nf);
  return nf_max <= kSnrSmallMaxFreqs;
}
}  // namespace

extern "C" bls_status bls_snr(bls_plan* plan, void* ws, const double* d_sr, const bls_best* d_best,
                              double* d_snr, bls_result* d_result, bls_stream_t stream) {
  if (!plan || !d_sr || !d_result) return BLS_E_ARG;
  if (!ws || plan->uploaded_to != ws) return BLS_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const Layout& L = plan->layout;
  const StarDesc* sd = reinterpret_cast<const StarDesc*>(base + L.stars);
  double* rho = reinterpret_cast<double*>(base + L.rho);
  if (snr_small_groups(plan))
    hipLaunchKernelGGL(k_snr<kSnrThreads>, dim3(plan->n_stars), dim3(kSnrThreads), 0, st, sd, d_sr, d_best, d_snr,
                       rho, d_result, plan->consts);
  else
    hipLaunchKernelGGL(k_snr<kThreads>, dim3(plan->n_stars), dim3(kThreads), 0, st, sd, d_sr, d_best, d_snr, rho,
                       d_result, plan->consts);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

extern "C" bls_status pp_snr_windows(const bls_plan* fine, void* fine_ws, const double* d_sr, const bls_best* d_best,
                                     const bls_plan* coarse, void* coarse_ws, const double* d_coarse_sr,
                                     const int64_t* d_windows, int32_t windows_per_star, const uint8_t* d_fallback,
                                     bls_result* d_result, bls_stream_t stream) {
  if (!fine || !coarse || !d_sr || !d_coarse_sr || !d_windows || !d_fallback || !d_result) return BLS_E_ARG;
  if (windows_per_star < 1 || fine->n_stars != coarse->n_stars) return BLS_E_ARG;
  if (!fine_ws || fine->uploaded_to != fine_ws || !coarse_ws || coarse->uploaded_to != coarse_ws) return BLS_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* fb = static_cast<char*>(fine_ws);
  char* cb = static_cast<char*>(coarse_ws);
  const StarDesc* fd = reinterpret_cast<const StarDesc*>(fb + fine->layout.stars);
  const StarDesc* cd = reinterpret_cast<const StarDesc*>(cb + coarse->layout.stars);
  double* rf = reinterpret_cast<double*>(fb + fine->layout.rho);
  double* rc = reinterpret_cast<double*>(cb + coarse->layout.rho);
  if (snr_small_groups(fine))
    hipLaunchKernelGGL(k_snr_windows<kSnrThreads>, dim3(fine->n_stars), dim3(kSnrThreads), 0, st, fd, cd, d_sr, d_best,
                       rf, d_coarse_sr, rc, d_windows, windows_per_star, d_fallback, d_result, fine->consts);
  else
    hipLaunchKernelGGL(k_snr_windows<kThreads>, dim3(fine->n_stars), dim3(kThreads), 0, st, fd, cd, d_sr, d_best, rf,
                       d_coarse_sr, rc, d_windows, windows_per_star, d_fallback, d_result, fine->consts);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}
