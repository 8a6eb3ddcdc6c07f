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
// One 1024-thread workgroup per CU takes work items (a frequency range of one
// star) round-robin.  A point's bin in a set is the plain path's: FP64 phase (one
// multiply and an exact fract) times nb_k, truncated; its fixed-point weight and
// weighted residual (differences of the prepared exclusive prefix sums) are added
// to int64 LDS accumulators, and windows are scanned with exact int64 sums.  When
// every set of a frequency fits the 8192 accumulator pairs together, up to 32
// frequencies are binned in one pass over the points (the phase once per point and
// frequency, then one multiply and two LDS adds per set); otherwise one set at a
// time, in passes over start-bin ranges beyond 8192 bins.  Stars of equal weights
// add 32-bit counts of weighted points in place of weight prefixes (counts.hpp).
// The best window over (k, j) has the largest power; ties go to the smallest (k, j).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "counts.hpp"
#include "plan.hpp"

namespace mi355bls {

namespace {

constexpr int kRebinThreads = 1024;
constexpr int kRebinSlots = 8192;      // int64 accumulator pairs (128 KiB)
constexpr int kRebinF = 32;            // most frequencies binned together
constexpr int kScanIter = kRebinSlots / kRebinThreads;
static_assert((kRebinF & (kRebinF - 1)) == 0 && (kRebinMax & (kRebinMax - 1)) == 0 && kRebinMax <= 64 && kRebinF <= 64,
              "rows of the set tables are read one entry per lane");
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
  int2 nbo[kRebinF][kRebinMax];     // set k at the group's frequency fi: bins (0: no window),
                                    // first slot
  int32_t off[kRebinMax + 1];       // slot offset of set k within one frequency's stride
  double f[kRebinF];
  unsigned long long key[kRebinF];
  uint32_t kj[kRebinF];
  int32_t n_ok;                     // leading frequencies whose sets fit the stride
  unsigned long long wkey[kRebinThreads / 64];
  uint32_t wkj[kRebinThreads / 64];
  double wr[kRebinThreads / 64];
  double ws[kRebinThreads / 64];
};

__device__ __forceinline__ double readlane_f64(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

struct Cand {
  unsigned long long key;  // bits of the power + 1 (0: none); powers are >= 0
  uint32_t kj;             // (k << 20) | j
  double r, s;
};

__device__ __forceinline__ bool cand_better(const Cand& a, const Cand& b) {
  return a.key > b.key || (a.key == b.key && a.key != 0ull && a.kj < b.kj);
}

// The weight side of a star: prefixes of the fixed-point weights, or (equal
// weights, cnt) counts of weighted points, the prefixes divided by `unit`.
struct WeightForm {
  bool cnt;
  CountDiv cd;
  int64_t unit;
  long long total;  // the star's total in the form's units
};

__device__ __forceinline__ WeightForm weight_form(const StarRt& rt) {
  WeightForm wf;
  wf.cnt = rt.w_unit != 0;
  wf.unit = rt.w_unit;
  wf.cd = wf.cnt ? count_div(rt.w_unit) : CountDiv{0u, 0u};
  wf.total = wf.cnt ? static_cast<long long>(count_of(rt.cw_total, wf.cd)) : rt.cw_total;
  return wf;
}

// Time of point q and the exclusive prefix sums of the weights (in the form's
// units) and weighted residuals at q and q + 1 (the star's totals after its last
// point).
__device__ __forceinline__ void point_prefix(const double* __restrict__ dt, const int64_t* __restrict__ cw,
                                             const int64_t* __restrict__ cs, const StarRt& rt, const WeightForm& wf,
                                             int64_t q, int64_t n, double& x, long long& p0, long long& p1,
                                             long long& s0, long long& s1) {
  x = dt[q];
  p0 = cw[q];
  s0 = cs[q];
  p1 = q + 1 < n ? cw[q + 1] : rt.cw_total;
  s1 = q + 1 < n ? cs[q + 1] : rt.cs_total;
  if (wf.cnt) {
    p0 = count_of(p0, wf.cd);
    p1 = q + 1 < n ? static_cast<long long>(count_of(p1, wf.cd)) : wf.total;
  }
}

// A window's weight total in fixed-point units from the sum of its slots (counts:
// each slot's low word is its bin's count, the high word stays zero).
__device__ __forceinline__ unsigned long long weight_units(unsigned long long rw, const WeightForm& wf) {
  return wf.cnt ? rw * static_cast<unsigned long long>(wf.unit) : rw;
}

// Adds one wave's 64 consecutive points (one set of one frequency) to the LDS
// accumulators.  A point's contribution is P[q+1] - P[q] of the exclusive prefix
// sums P; over a run of consecutive points in one bin these telescope to P[end+1] -
// P[start], so only a run's first point (-P[q]) and last point (+P[q+1]) add, each
// into its own bin: one atomic per value and lane, and no more than the two ends of
// a run on one address.  The chunk's first and last points close their runs, so
// chunks are independent.  The neighbours' bins come by DPP wave shifts.
// slot < 0: the point's bin is not held.
__device__ __forceinline__ void add_chunk(RebinLds& L, bool cnt, int lane, int last, bool valid, int32_t b, int slot,
                                          long long p0, long long p1, long long s0, long long s1) {
  const int32_t bp = __builtin_amdgcn_update_dpp(b, b, 0x138, 0xf, 0xf, false);  // lane - 1 (wave_shr:1)
  const int32_t bn = __builtin_amdgcn_update_dpp(b, b, 0x130, 0xf, 0xf, false);  // lane + 1 (wave_shl:1)
  const bool start = valid && (lane == 0 || b != bp);
  const bool end = valid && (lane == last || b != bn);
  if ((start || end) && slot >= 0) {
    const unsigned long long vw = (end ? static_cast<unsigned long long>(p1) : 0ull) -
                                  (start ? static_cast<unsigned long long>(p0) : 0ull);
    const unsigned long long vs = (end ? static_cast<unsigned long long>(s1) : 0ull) -
                                  (start ? static_cast<unsigned long long>(s0) : 0ull);
    if (cnt)  // the low word of the slot
      atomicAdd(reinterpret_cast<unsigned int*>(&L.gw[slot]), static_cast<unsigned int>(vw));
    else
      atomicAdd(reinterpret_cast<unsigned long long*>(&L.gw[slot]), vw);
    atomicAdd(reinterpret_cast<unsigned long long*>(&L.gs[slot]), vs);
  }
}

// Power key of a window from its exact int64 sums (0 when the window is invalid).
template <bool DIP>
__device__ __forceinline__ unsigned long long window_key(unsigned long long rw, unsigned long long rs, double s_scale,
                                                         double& r, double& s) {
  r = static_cast<double>(static_cast<long long>(rw)) * kUnitW;
  s = static_cast<double>(static_cast<long long>(rs)) * s_scale;
  if (!(r > 0.0 && r < 1.0) || (DIP && !(s < 0.0))) return 0ull;
  const double pw = (s * s) / (r * (1.0 - r));
  return static_cast<unsigned long long>(__double_as_longlong(pw)) + 1ull;
}

__device__ __forceinline__ void write_best(const RebinArgs& a, int64_t out, unsigned long long key, uint32_t kj,
                                           double r, double s) {
  bls_best bb;
  double sr = 0.0;
  if (key != 0ull) {
    sr = sqrt((s * s) / (r * (1.0 - r)));
    bb.m = static_cast<int32_t>(kj >> 20);
    bb.j = static_cast<int32_t>(kj & 0xFFFFFu);
    bb.r = r;
    bb.s = s;
  } else {
    bb.m = 0;
    bb.j = -1;
    bb.r = 0.0;
    bb.s = 0.0;
  }
  a.sr[out] = sr;
  if (a.best) a.best[out] = bb;
}

// One frequency whose bin sets do not fit together: one set at a time, in passes
// over ranges of start bins when a set exceeds the accumulators.
template <bool DIP>
__device__ void rebin_one(const RebinArgs& a, RebinLds& L, const StarDesc& d, const StarRt& rt,
                          const WeightForm& wf, int64_t fi, const double* __restrict__ dt,
                          const int64_t* __restrict__ cw, const int64_t* __restrict__ cs) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, T = kRebinThreads;
  const int32_t nov = a.c.noverlap;
  const int64_t n = d.n;
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
      for (int64_t c0 = static_cast<int64_t>(wave) * 64; c0 < n; c0 += static_cast<int64_t>(T)) {
        const int64_t q = c0 + lane;
        const bool valid = q < n;
        const int last = static_cast<int>(min<int64_t>(63, n - 1 - c0));
        long long p0 = 0, p1 = 0, s0 = 0, s1 = 0;
        double x = 0.0;
        if (valid) point_prefix(dt, cw, cs, rt, wf, q, n, x, p0, p1, s0, s1);
        const double ph = __builtin_amdgcn_fract(x * f);  // x - floor(x)
        int32_t b = static_cast<int32_t>(ph * nbd);
        b = b < nb - 1 ? b : nb - 1;
        int32_t slot = b - b0;
        if (slot < 0) slot += nb;
        add_chunk(L, wf.cnt, lane, last, valid, b, slot < nslot ? slot : -1, p0, p1, s0, s1);
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
        double r, s;
        const unsigned long long key = window_key<DIP>(weight_units(rw, wf), rs, rt.s_scale, r, s);
        if (key > mine.key) {  // k, then j, ascend within a thread: ties keep the first
          mine.key = key;
          mine.kj = (static_cast<uint32_t>(k) << 20) | static_cast<uint32_t>(b0 + j);
          mine.r = r;
          mine.s = s;
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
    write_best(a, d.f_off + fi, b.key, b.kj, b.r, b.s);
  }
  __syncthreads();
}

// Up to kRebinF consecutive frequencies starting at g0 whose bin sets fit the
// accumulators together: every set of a frequency gets room for its count at g0
// (counts fall with frequency) plus, with exact durations, one bin for the device
// asin's last place; a frequency whose counts exceed that room ends the group.
// One pass over the points bins each point's phase into every set.  Returns the
// number of frequencies searched (0: the first does not fit; use rebin_one).
template <bool DIP>
__device__ int rebin_group(const RebinArgs& a, RebinLds& L, const StarDesc& d, const StarRt& rt,
                           const WeightForm& wf, int64_t g0, int64_t g_end, const double* __restrict__ dt,
                           const int64_t* __restrict__ cw, const int64_t* __restrict__ cs) {
  const int tid = threadIdx.x, T = kRebinThreads;
  const int32_t nov = a.c.noverlap, K = a.c.n_rebin;
  const int64_t n = d.n;
  if (tid == 0) {
    const double u = d.umin + static_cast<double>(g0) * d.A;
    const double qlo = qlo_at(d, a.c, u * u);
    int32_t acc = 0;
    for (int k = 0; k < K; ++k) {
      const int32_t nb = rebin_bins(qlo, a.c.rebin_g[k], nov);
      const int32_t room = nb + a.c.exact_q;
      L.off[k] = acc;
      acc += room > nov ? room : 0;
      if (acc > kRebinSlots) acc = kRebinSlots + 1;  // does not fit (and cannot overflow)
    }
    L.off[K] = acc;
  }
  __syncthreads();
  const int32_t S = L.off[K];
  if (S > kRebinSlots) return 0;
  const int fmax = static_cast<int>(min<int64_t>(min(kRebinF, S > 0 ? kRebinSlots / S : kRebinF), g_end - g0));
  if (tid == 0) L.n_ok = fmax;
  __syncthreads();
  if (tid < fmax) {
    const double u = d.umin + static_cast<double>(g0 + tid) * d.A;
    const double uu = u * u;
    const double qlo = qlo_at(d, a.c, uu);
    L.f[tid] = uu * u;
    bool fits = true;
    for (int k = 0; k < K; ++k) {
      const int32_t nb = rebin_bins(qlo, a.c.rebin_g[k], nov);
      const bool live = nb > nov;
      L.nbo[tid][k] = make_int2(live ? nb : 0, tid * S + L.off[k]);
      if (live && nb > L.off[k + 1] - L.off[k]) fits = false;
    }
    L.key[tid] = 0ull;
    L.kj[tid] = ~0u;
    if (!fits) atomicMin(&L.n_ok, tid);
  }
  __syncthreads();
  const int F = L.n_ok;  // >= 1: the first frequency's counts define the room
  for (int i = tid; i < F * S; i += T) {
    L.gw[i] = 0;
    L.gs[i] = 0;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  // The group's frequencies and, per frequency, its sets' bins and first slots are
  // read from LDS once per 64-point chunk as a row across the lanes (lane i holds
  // entry i; entries past F or K are in bounds and unused), then taken lane by lane
  // into scalar registers: one LDS read per frequency instead of one per set.
  const double f_row = L.f[lane & (kRebinF - 1)];
  for (int64_t c0 = static_cast<int64_t>(wave) * 64; c0 < n; c0 += static_cast<int64_t>(T)) {
    const int64_t q = c0 + lane;
    const bool valid = q < n;
    const int last = static_cast<int>(min<int64_t>(63, n - 1 - c0));
    long long p0 = 0, p1 = 0, s0 = 0, s1 = 0;
    double x = 0.0;
    if (valid) point_prefix(dt, cw, cs, rt, wf, q, n, x, p0, p1, s0, s1);
    for (int fi = 0; fi < F; ++fi) {
      const double ph = __builtin_amdgcn_fract(x * readlane_f64(f_row, fi));  // x - floor(x)
      const int2 row = L.nbo[fi][lane & (kRebinMax - 1)];
      for (int k = 0; k < K; ++k) {
        const int32_t nb = __builtin_amdgcn_readlane(row.x, k);
        if (nb == 0) continue;
        const int32_t slot0 = __builtin_amdgcn_readlane(row.y, k);
        int32_t b = static_cast<int32_t>(ph * static_cast<double>(nb));
        b = b < nb - 1 ? b : nb - 1;
        add_chunk(L, wf.cnt, lane, last, valid, b, slot0 + b, p0, p1, s0, s1);
      }
    }
  }
  __syncthreads();
  // windows: one per slot (frequency fi, set k, start j < nb)
  unsigned long long ckey[kScanIter];
  uint32_t ckj[kScanIter];
  int cfi[kScanIter];
#pragma unroll
  for (int it = 0; it < kScanIter; ++it) {
    const int x = tid + it * T;
    ckey[it] = 0ull;
    ckj[it] = ~0u;
    cfi[it] = 0;
    if (x < F * S) {
      const int fi = x / S;
      const int rem = x - fi * S;
      int k = 0;
      while (k + 1 < K && L.off[k + 1] <= rem) ++k;
      const int32_t nb = L.nbo[fi][k].x;
      const int j = rem - L.off[k];
      if (nb > 0 && j < nb) {
        const int sb = fi * S + L.off[k];
        unsigned long long rw = 0ull, rs = 0ull;
        for (int v = 0; v < nov; ++v) {
          int idx = j + v;
          if (idx >= nb) idx -= nb;
          rw += static_cast<unsigned long long>(L.gw[sb + idx]);
          rs += static_cast<unsigned long long>(L.gs[sb + idx]);
        }
        double r, s;
        const unsigned long long key = window_key<DIP>(weight_units(rw, wf), rs, rt.s_scale, r, s);
        if (key != 0ull) {
          ckey[it] = key;
          ckj[it] = (static_cast<uint32_t>(k) << 20) | static_cast<uint32_t>(j);
          cfi[it] = fi;
          atomicMax(&L.key[fi], key);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kScanIter; ++it)
    if (ckey[it] != 0ull && ckey[it] == L.key[cfi[it]]) atomicMin(&L.kj[cfi[it]], ckj[it]);
  __syncthreads();
  if (tid < F) {
    const unsigned long long key = L.key[tid];
    const uint32_t kj = L.kj[tid];
    double r = 0.0, s = 0.0;
    if (key != 0ull) {  // the winner's sums again (exact, so the same r and s)
      const int k = static_cast<int>(kj >> 20), j = static_cast<int>(kj & 0xFFFFFu);
      const int32_t nb = L.nbo[tid][k].x;
      const int sb = tid * S + L.off[k];
      unsigned long long rw = 0ull, rs = 0ull;
      for (int v = 0; v < nov; ++v) {
        int idx = j + v;
        if (idx >= nb) idx -= nb;
        rw += static_cast<unsigned long long>(L.gw[sb + idx]);
        rs += static_cast<unsigned long long>(L.gs[sb + idx]);
      }
      (void)window_key<DIP>(weight_units(rw, wf), rs, rt.s_scale, r, s);
    }
    write_best(a, d.f_off + g0 + tid, key, kj, r, s);
  }
  __syncthreads();
  return F;
}

template <bool DIP>
__global__ void __launch_bounds__(kRebinThreads) k_search_rebin(RebinArgs a) {
  __shared__ RebinLds L;
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
    const WeightForm wf = weight_form(rt);
    const double* __restrict__ dt = a.dt + d.p_off;
    const int64_t* __restrict__ cw = a.cw + d.p_off;
    const int64_t* __restrict__ cs = a.cs + d.p_off;
    for (int64_t g0 = i0; g0 < i1;) {
      const int F = rebin_group<DIP>(a, L, d, rt, wf, g0, i1, dt, cw, cs);
      if (F > 0) {
        g0 += F;
      } else {
        rebin_one<DIP>(a, L, d, rt, wf, g0, dt, cw, cs);
        g0 += 1;
      }
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
  const int64_t grid = std::min<int64_t>(n_items, static_cast<int64_t>(cus));  // one group per CU (133 KiB LDS)
  if (a.c.dip_only)
    hipLaunchKernelGGL(k_search_rebin<true>, dim3(static_cast<unsigned>(grid)), dim3(kRebinThreads), 0, st, a);
  else
    hipLaunchKernelGGL(k_search_rebin<false>, dim3(static_cast<unsigned>(grid)), dim3(kRebinThreads), 0, st, a);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

}  // namespace mi355bls
