// rebin.hip — the BLS search with one bin set per searched duration (the
// per-duration rebinning variant, rebin = 1).
//
// QLP Data Release Notes 003, Sec. 2.1 footnote, gives cuvarbase's noverlap = 3.
// Read literally, every duration q_k of a continuous ladder (q_k = g_k q_lo, g_k =
// min(e^(k dlogq), qmax/qmin)) gets its own phase binning of nb_k =
// ceil(noverlap / q_k) bins, and a transit window is noverlap consecutive bins
// (cyclic) starting at any bin: noverlap shifted bin sets of width about q_k.  The
// plain search instead bins once per frequency at q_lo / noverlap and scans windows
// of the integer ladder m_k; both give SR of Kovacs et al. (2002).
//
// One workgroup per work item (a frequency range of one star), static round-robin.
// Per frequency and duration: every point's bin from the FP64 phase (one multiply
// and an exact fract, then one multiply by nb_k, as the plain path's fold), its
// fixed-point weight and weighted residual (differences of the prepared exclusive
// prefix sums) added to int64 LDS accumulators, then each thread scans the windows
// of its start bins with exact int64 window sums.  Bin sets wider than the LDS are
// searched in passes over ranges of start bins.  The best window over (k, j) has
// the largest power; ties go to the smallest (k, j).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "plan.hpp"

namespace mi355bls {

namespace {

constexpr int kRebinThreads = 512;
constexpr int kRebinSlots = 4096;      // int64 accumulator pairs per pass (64 KiB)
constexpr int kRebinGroupsPerCu = 2;
constexpr double kUnitW = 2.168404344971008868e-19;  // 2^-62: one fixed-point weight unit

struct RebinArgs {
  const StarDesc* stars;
  const StarRt* rt;
  const WorkItem* items;
  const int64_t* windows;  // optional (star, i0, i1) triples replacing items
  const double* dt;
  const int64_t* cw;       // exclusive prefix sums of the fixed-point weights
  const int64_t* cs;       // and of the fixed-point weighted residuals
  double* sr;
  bls_best* best;
  int32_t n_items;
  int32_t n_stars;
  Consts c;
};

struct RebinLds {
  long long gw[kRebinSlots];
  long long gs[kRebinSlots];
  unsigned long long wkey[kRebinThreads / 64];
  uint32_t wkj[kRebinThreads / 64];
  double wr[kRebinThreads / 64];
  double ws[kRebinThreads / 64];
};

struct Cand {
  unsigned long long key;  // bits of the power + 1 (0: none); powers are >= 0
  uint32_t kj;             // (k << 20) | j
  double r, s;
};

__device__ __forceinline__ bool cand_better(const Cand& a, const Cand& b) {
  return a.key > b.key || (a.key == b.key && a.key != 0ull && a.kj < b.kj);
}

template <bool DIP>
__global__ void __launch_bounds__(kRebinThreads) k_search_rebin(RebinArgs a) {
  __shared__ RebinLds L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, T = kRebinThreads;
  const int32_t nov = a.c.noverlap;
  for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    int64_t star, i0, i1;
    if (a.windows) {
      star = a.windows[3 * item];
      i0 = a.windows[3 * item + 1];
      i1 = a.windows[3 * item + 2];
    } else {
      const WorkItem it = a.items[item];
      star = it.star;
      i0 = it.i0;
      i1 = it.i1;
    }
    if (star < 0 || star >= a.n_stars) continue;
    const StarDesc d = a.stars[star];
    i0 = max<int64_t>(0, min<int64_t>(i0, d.nf));
    i1 = max<int64_t>(0, min<int64_t>(i1, d.nf));
    const StarRt rt = a.rt[star];
    const int64_t n = d.n;
    const double* __restrict__ dt = a.dt + d.p_off;
    const int64_t* __restrict__ cw = a.cw + d.p_off;
    const int64_t* __restrict__ cs = a.cs + d.p_off;
    for (int64_t fi = i0; fi < i1; ++fi) {
      const double u = d.umin + static_cast<double>(fi) * d.A;
      const double uu = u * u;
      const double f = uu * u;
      const double qlo = qlo_at(d, a.c, uu);
      Cand mine{0ull, ~0u, 0.0, 0.0};
      for (int k = 0; k < a.c.n_rebin; ++k) {
        const int32_t nb = rebin_bins(qlo, a.c.rebin_g[k], nov);
        if (nov >= nb) continue;  // a window would cover every point
        const double nbd = static_cast<double>(nb);
        // one pass when the set fits; else ranges of `span` start bins, each with the
        // noverlap - 1 bins after it (nslot <= nb, so no two slots alias one bin)
        const int passes = nb <= kRebinSlots ? 1 : (nb + kRebinSlots - nov) / (kRebinSlots - nov + 1);
        const int span = passes == 1 ? nb : (nb + passes - 1) / passes;
        const int nslot = passes == 1 ? nb : span + nov - 1;
        for (int p = 0; p < passes; ++p) {
          const int32_t b0 = p * span;
          for (int i = tid; i < nslot; i += T) {
            L.gw[i] = 0;
            L.gs[i] = 0;
          }
          __syncthreads();
          for (int64_t q = tid; q < n; q += T) {
            const double x = dt[q] * f;
            const double ph = __builtin_amdgcn_fract(x);  // x - floor(x), exact for x >= 0
            int32_t b = static_cast<int32_t>(ph * nbd);
            b = b < nb - 1 ? b : nb - 1;
            int32_t slot = b - b0;
            if (slot < 0) slot += nb;
            if (slot < nslot) {
              const long long w1 = q + 1 < n ? cw[q + 1] : rt.cw_total;
              const long long s1 = q + 1 < n ? cs[q + 1] : rt.cs_total;
              const unsigned long long ew = static_cast<unsigned long long>(w1) - static_cast<unsigned long long>(cw[q]);
              const unsigned long long es = static_cast<unsigned long long>(s1) - static_cast<unsigned long long>(cs[q]);
              atomicAdd(reinterpret_cast<unsigned long long*>(&L.gw[slot]), ew);
              atomicAdd(reinterpret_cast<unsigned long long*>(&L.gs[slot]), es);
            }
          }
          __syncthreads();
          for (int j = tid; j < span && b0 + j < nb; j += T) {
            unsigned long long rw = 0ull, rs = 0ull;
            for (int v = 0; v < nov; ++v) {
              int idx = j + v;
              if (idx >= nb) idx -= nb;  // one pass: slots are bins (cyclic)
              rw += static_cast<unsigned long long>(L.gw[idx]);
              rs += static_cast<unsigned long long>(L.gs[idx]);
            }
            const double r = static_cast<double>(static_cast<long long>(rw)) * kUnitW;
            const double s = static_cast<double>(static_cast<long long>(rs)) * rt.s_scale;
            if (r > 0.0 && r < 1.0 && (!DIP || s < 0.0)) {
              const double pw = (s * s) / (r * (1.0 - r));
              const unsigned long long key = static_cast<unsigned long long>(__double_as_longlong(pw)) + 1ull;
              if (key > mine.key) {  // k, then j, ascend within a thread: ties keep the first
                mine.key = key;
                mine.kj = (static_cast<uint32_t>(k) << 20) | static_cast<uint32_t>(b0 + j);
                mine.r = r;
                mine.s = s;
              }
            }
          }
          __syncthreads();
        }
      }
      // block argmax: largest power, then smallest (k, j)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        Cand other;
        other.key = __shfl_xor(mine.key, o, 64);
        other.kj = __shfl_xor(mine.kj, o, 64);
        other.r = __shfl_xor(mine.r, o, 64);
        other.s = __shfl_xor(mine.s, o, 64);
        if (cand_better(other, mine)) mine = other;
      }
      if (lane == 0) {
        L.wkey[wave] = mine.key;
        L.wkj[wave] = mine.kj;
        L.wr[wave] = mine.r;
        L.ws[wave] = mine.s;
      }
      __syncthreads();
      if (tid == 0) {
        Cand b{L.wkey[0], L.wkj[0], L.wr[0], L.ws[0]};
        for (int v = 1; v < T / 64; ++v) {
          const Cand o{L.wkey[v], L.wkj[v], L.wr[v], L.ws[v]};
          if (cand_better(o, b)) b = o;
        }
        const int64_t out = d.f_off + fi;
        bls_best bb;
        double sr = 0.0;
        if (b.key != 0ull) {
          sr = sqrt((b.s * b.s) / (b.r * (1.0 - b.r)));
          bb.m = static_cast<int32_t>(b.kj >> 20);
          bb.j = static_cast<int32_t>(b.kj & 0xFFFFFu);
          bb.r = b.r;
          bb.s = b.s;
        } else {
          bb.m = 0;
          bb.j = -1;
          bb.r = 0.0;
          bb.s = 0.0;
        }
        a.sr[out] = sr;
        if (a.best) a.best[out] = bb;
      }
      __syncthreads();
    }
  }
}

}  // namespace

// The rebinning search over the plan's work items or a caller's window list (see
// bls_search_batch); the workspace must hold the prepared arrays.
bls_status rebin_search(const bls_plan* plan, const char* base, const int64_t* d_windows, int64_t n_items,
                        double* d_sr, bls_best* d_best, hipStream_t st) {
  const Layout& Ly = plan->layout;
  RebinArgs a;
  a.stars = reinterpret_cast<const StarDesc*>(base + Ly.stars);
  a.rt = reinterpret_cast<const StarRt*>(base + Ly.rt);
  a.items = reinterpret_cast<const WorkItem*>(base + Ly.items);
  a.windows = d_windows;
  a.dt = reinterpret_cast<const double*>(base + Ly.dt);
  a.cw = reinterpret_cast<const int64_t*>(base + Ly.cw);
  a.cs = reinterpret_cast<const int64_t*>(base + Ly.cs);
  a.sr = d_sr;
  a.best = d_best;
  a.n_items = static_cast<int32_t>(n_items);
  a.n_stars = plan->n_stars;
  a.c = plan->consts;
  if (a.c.n_rebin < 1 || a.c.n_rebin > kRebinMax || a.c.packed) return BLS_E_STATE;
  int dev = 0, cus = 0;
  BLS_HIP_TRY(hipGetDevice(&dev));
  BLS_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (cus < 1) return BLS_E_HIP;
  const int64_t grid = std::min<int64_t>(n_items, kRebinGroupsPerCu * static_cast<int64_t>(cus));
  if (a.c.dip_only)
    hipLaunchKernelGGL(k_search_rebin<true>, dim3(static_cast<unsigned>(grid)), dim3(kRebinThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_search_rebin<false>, dim3(static_cast<unsigned>(grid)), dim3(kRebinThreads), 0, st, a);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

}  // namespace mi355bls
