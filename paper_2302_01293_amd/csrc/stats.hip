// stats.hip — the other statistics of a detection (QLP Data Release Notes 003,
// Sec. 2.2 item 5) and the detection criteria of the paragraph after the list:
// points in, before and after transit, the number of transits (a transit counts
// only when data lie within half a duration of its expected mid-transit time),
// the out-of-transit level, and the candidate flag (at least two transits and
// S/N above the threshold, 9 in the note).
//
// Each star is described by the best window of its detection frequency i_snr (from
// bls_snr and the per-frequency best windows of bls_search_batch): m fine bins
// starting at bin j of the fold at f_i with nb_i bins.  A point with w > 0 and
// p = (t - t0) f, ip = floor(p), bin b = min(nb - 1, floor((p - ip) nb)) -- the
// search's own fold, so the same points are "in" the window -- sits at offset
// o = (b - j) mod nb from the window start:
//   in transit      o < m                      (within half a duration of mid-transit)
//   after transit   m <= o < 2m                (the duration after egress)
//   before transit  o >= 2m and o >= nb - m    (the duration before ingress)
// Its transit number is k = floor((ip nb + b - j) / nb), the cycle in which its
// window starts.  ip nb + b never decreases along a star's time-ordered points, so
// k never decreases either, and the transits with data are the in-transit points
// whose k exceeds that of every earlier in-transit point: an exclusive running
// maximum per tile of points, carried across tiles.
//
// One 1024-thread workgroup per star; points are read tile by tile (coalesced).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "plan.hpp"

namespace mi355bls {

namespace {

constexpr int kStatThreads = 1024;
constexpr long long kNoK = -(1ll << 62);  // below every transit number

struct StatLds {
  long long wmax[kStatThreads / 64];
  unsigned long long cnt[kStatThreads / 64][4];
  double sw[kStatThreads / 64][2], swy[kStatThreads / 64][2];
  long long carry;
  double f;
  int32_t nb, m, j, ok;
};

__device__ __forceinline__ long long wave_max_excl(long long v, long long* total) {
  const int lane = threadIdx.x & 63;
  long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o, 64);
    if (lane >= o) x = x > y ? x : y;
  }
  *total = __shfl(x, 63, 64);
  const long long e = __shfl_up(x, 1, 64);
  return lane == 0 ? kNoK : e;
}

// Neumaier addition, so the level does not depend on the reduction order beyond
// the last bits.
__device__ __forceinline__ void nsum(double& s, double& c, double v) {
  const double t = s + v;
  c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
  s = t;
}

}  // namespace

__global__ void __launch_bounds__(kStatThreads) k_stats(const StarDesc* __restrict__ stars, const double* __restrict__ t,
                                                        const double* __restrict__ y, const double* __restrict__ w,
                                                        const bls_best* __restrict__ best,
                                                        const bls_result* __restrict__ res, Consts c,
                                                        double snr_min, bls_star_stats* __restrict__ out) {
  __shared__ StatLds L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const StarDesc d = stars[blockIdx.x];
  if (tid == 0) {
    const bls_result r = res[blockIdx.x];
    L.ok = 0;
    if (r.i_snr >= 0 && r.i_snr < d.nf) {
      const bls_best bb = best[d.f_off + r.i_snr];
      const double u = d.umin + static_cast<double>(r.i_snr) * d.A;
      const double uu = u * u;
      L.f = uu * u;
      if (c.rebin) {  // m holds the duration index k: noverlap bins of the k-th set
        const bool kok = bb.m >= 0 && bb.m < c.n_rebin;
        L.nb = kok ? rebin_bins(qlo_at(d, c, uu), c.rebin_g[bb.m], c.noverlap) : 1;
        L.m = kok ? c.noverlap : 0;
      } else {
        L.nb = fine_bins(d, c, uu);
        L.m = bb.m;
      }
      L.j = bb.j;
      L.ok = (bb.m >= 1 && bb.m < L.nb && bb.j >= 0 && bb.j < L.nb) ? 1 : 0;
    }
    L.carry = kNoK;
  }
  __syncthreads();
  bls_star_stats st;
  st.n_in = st.n_before = st.n_after = st.n_transits = 0;
  st.oot_level = NAN;
  st.candidate = 0;
  st.status = 1;
  if (!L.ok) {
    if (tid == 0) out[blockIdx.x] = st;
    return;
  }
  const double f = L.f, nbd = static_cast<double>(L.nb);
  const int32_t nb = L.nb, m = L.m, j = L.j;
  const double t0 = d.t0;
  const int64_t n = d.n, off = d.p_off;
  unsigned long long n_in = 0, n_before = 0, n_after = 0, n_tr = 0;
  double sw = 0.0, cw = 0.0, swy = 0.0, cwy = 0.0;
  for (int64_t base = 0; base < n; base += kStatThreads) {
    const int64_t q = base + tid;
    long long k = kNoK;
    bool in = false;
    if (q < n) {
      const double wq = w ? w[off + q] : 1.0;
      if (wq > 0.0) {
        const double p = (t[off + q] - t0) * f;
        const double ip = floor(p);
        int32_t b = static_cast<int32_t>(floor((p - ip) * nbd));
        if (b >= nb) b = nb - 1;
        int32_t o = b - j;
        if (o < 0) o += nb;
        if (o < m) {
          in = true;
          ++n_in;
          const long long num = static_cast<long long>(ip) * nb + b - j;
          // floor division by nb > 0
          k = num >= 0 ? num / nb : -((-num + nb - 1) / nb);
        } else {
          if (o < 2 * m)
            ++n_after;
          else if (o >= nb - m)
            ++n_before;
          nsum(sw, cw, wq);
          nsum(swy, cwy, wq * y[off + q]);
        }
      }
    }
    // exclusive running maximum of k over the in-transit points of the tile
    long long wtot;
    const long long ex = wave_max_excl(k, &wtot);
    if (lane == 63) L.wmax[wave] = wtot;
    __syncthreads();
    long long before = L.carry;
    for (int v = 0; v < wave; ++v) before = before > L.wmax[v] ? before : L.wmax[v];
    before = before > ex ? before : ex;
    if (in && k > before) ++n_tr;
    __syncthreads();
    if (tid == 0) {
      long long cm = L.carry;
      for (int v = 0; v < kStatThreads / 64; ++v) cm = cm > L.wmax[v] ? cm : L.wmax[v];
      L.carry = cm;
    }
    __syncthreads();
  }
  // block reductions
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    n_in += __shfl_xor(n_in, o, 64);
    n_before += __shfl_xor(n_before, o, 64);
    n_after += __shfl_xor(n_after, o, 64);
    n_tr += __shfl_xor(n_tr, o, 64);
  }
  // compensated sums: exchange (s, c) pairs and merge in a fixed order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double s1 = __shfl_xor(sw, o, 64), c1 = __shfl_xor(cw, o, 64);
    const double s2 = __shfl_xor(swy, o, 64), c2 = __shfl_xor(cwy, o, 64);
    nsum(sw, cw, s1);
    cw += c1;
    nsum(swy, cwy, s2);
    cwy += c2;
  }
  if (lane == 0) {
    L.cnt[wave][0] = n_in;
    L.cnt[wave][1] = n_before;
    L.cnt[wave][2] = n_after;
    L.cnt[wave][3] = n_tr;
    L.sw[wave][0] = sw;
    L.sw[wave][1] = cw;
    L.swy[wave][0] = swy;
    L.swy[wave][1] = cwy;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long a = 0, b = 0, e = 0, tr = 0;
    double s = 0.0, sc = 0.0, s2 = 0.0, sc2 = 0.0;
    for (int v = 0; v < kStatThreads / 64; ++v) {
      a += L.cnt[v][0];
      b += L.cnt[v][1];
      e += L.cnt[v][2];
      tr += L.cnt[v][3];
      nsum(s, sc, L.sw[v][0]);
      sc += L.sw[v][1];
      nsum(s2, sc2, L.swy[v][0]);
      sc2 += L.swy[v][1];
    }
    st.n_in = static_cast<int64_t>(a);
    st.n_before = static_cast<int64_t>(b);
    st.n_after = static_cast<int64_t>(e);
    st.n_transits = static_cast<int64_t>(tr);
    const double W = s + sc;
    st.oot_level = W > 0.0 ? (s2 + sc2) / W : NAN;
    st.candidate = (tr >= 2 && res[blockIdx.x].snr > snr_min) ? 1 : 0;
    st.status = 0;
    out[blockIdx.x] = st;
  }
}

}  // namespace mi355bls

using namespace mi355bls;

extern "C" bls_status bls_stats(bls_plan* plan, void* ws, const double* d_t, const double* d_y, const double* d_w,
                                const bls_best* d_best, const bls_result* d_result, double snr_min,
                                bls_star_stats* d_stats, bls_stream_t stream) {
  if (!plan || !d_t || !d_y || !d_best || !d_result || !d_stats) return BLS_E_ARG;
  if (!(snr_min == snr_min)) return BLS_E_ARG;
  if (!ws || plan->uploaded_to != ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return BLS_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const StarDesc* sd = reinterpret_cast<const StarDesc*>(static_cast<char*>(ws) + plan->layout.stars);
  hipLaunchKernelGGL(k_stats, dim3(plan->n_stars), dim3(kStatThreads), 0, st, sd, d_t, d_y, d_w, d_best, d_result,
                     plan->consts, snr_min, d_stats);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}
