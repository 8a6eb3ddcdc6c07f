// search.hip — gfx950 kernels of the BLS search: preparation (normalise, fixed-point
// prefix sums) and the fused fold -> bin accumulation -> duration/phase scan.
//
// The statistic is Kovacs, Zucker & Mazeh (2002), which QLP Data Release Notes 003
// adopts (Introduction; Sec. 2.2 item 1 calls it the signal residue SR):
//   wt = w / sum w,  x = y - sum wt y,  for a window of phase bins:
//   r = sum wt,  s = sum wt x,  SR = max sqrt(s^2 / (r (1 - r))),
// on the Keplerian grid of Sec. 2.1: durations between 0.5 and 2.0 times the
// circular-orbit duration, fine bins of width <= q_lo / noverlap, durations of
// m fine bins for m in the dlogq ladder, windows starting at every fine bin.
//
// Design (MI355X): the bin sums are built without per-point atomics.
//  * The preparation kernel quantises wt and wt x to int64 fixed point (2^-62 and a
//    per-star power of two) and stores their exclusive prefix sums CW, CS.
//  * Along the time-ordered points the phase bin only changes at "boundaries".  If
//    every boundary at point n adds (CW[n], CS[n]) into G[b] for each bin b it
//    enters, the telescoping sum gives the exact bin totals
//        H[b] = G[b+1] - G[b] + [b == bin of the last point] * total.
//    Whole cycles skipped between two points add the same value to every G and
//    cancel; a point that skips bins inside a cycle (data gaps) adds its values
//    to a range of G, which changes H only at the range ends (the D slots).
//    Integer sums are exact, so the result does not depend on order.
//  * Points stay in registers (dt, CW, CS) across all frequencies of a work item;
//    only boundaries touch LDS (one 64-bit integer atomic pair per boundary).
//  * The phase frac((t - t0) f) is computed in FP64 with the same IEEE operations
//    as the grid (this file is compiled with -ffp-contract=off), so the bin of
//    every point is bit-identical to a sequential FP64 evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "plan.hpp"

namespace mi355bls {

__device__ __forceinline__ void grid_point(const StarDesc& d, int64_t i, int32_t noverlap, double& f,
                                           int32_t& nb) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  const double uu = u * u;
  f = uu * u;
  nb = static_cast<int32_t>(ceil(static_cast<double>(noverlap) / (d.kq * uu)));
}

// Fine bin of a point: b = min(nb-1, floor(frac(dt f) nb)).
__device__ __forceinline__ int32_t fold_bin(double dt, double f, double nbd, int32_t nbm1) {
  const double p = dt * f;
  const double ph = __builtin_amdgcn_fract(p);  // p - floor(p), exact for finite p >= 0
  const int32_t b = static_cast<int32_t>(ph * nbd);
  return b < nbm1 ? b : nbm1;
}

// ----------------------------------------------------------------------------
// Block reductions (1024 threads).
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ T block_sum(T v, T* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T r = 0;
  if (wave == 0) {
    r = lane < (blockDim.x >> 6) ? scratch[lane] : T(0);
    r = wave_sum(r);
    if (lane == 0) scratch[0] = r;
  }
  __syncthreads();
  r = scratch[0];
  __syncthreads();
  return r;
}

// Exclusive block scan of one int64 per thread; returns the total through *total.
__device__ int64_t block_exscan(int64_t v, int64_t* scratch, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  if (wave == 0) {
    const int nw = blockDim.x >> 6;
    int64_t s = lane < nw ? scratch[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < nw) scratch[lane] = s;  // inclusive per wave
  }
  __syncthreads();
  const int64_t wave_off = wave > 0 ? scratch[wave - 1] : 0;
  *total = scratch[(blockDim.x >> 6) - 1];
  __syncthreads();
  return wave_off + x - v;
}

// ----------------------------------------------------------------------------
// Compensated (Neumaier) block sum: the weighted mean must be accurate in absolute
// terms because s = sum_in wt (y - ybar) moves by r times the error of ybar while the
// flux level is ~10^3 times the signal.
// ----------------------------------------------------------------------------
struct CSum {
  double s, c;
};

__device__ __forceinline__ void csum_add(CSum& a, double v) {
  const double t = a.s + v;
  if (fabs(a.s) >= fabs(v))
    a.c += (a.s - t) + v;
  else
    a.c += (v - t) + a.s;
  a.s = t;
}

__device__ __forceinline__ CSum csum_merge(CSum a, CSum b) {
  CSum r = a;
  csum_add(r, b.s);
  r.c += b.c;
  return r;
}

__device__ double block_csum(CSum v, CSum* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    CSum y;
    y.s = __shfl_xor(v.s, o, 64);
    y.c = __shfl_xor(v.c, o, 64);
    v = csum_merge(v, y);
  }
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    CSum r = scratch[0];
    for (int q = 1; q < (blockDim.x >> 6); ++q) r = csum_merge(r, scratch[q]);
    scratch[0] = r;
  }
  __syncthreads();
  const CSum r = scratch[0];
  __syncthreads();
  return r.s + r.c;
}

// ----------------------------------------------------------------------------
// Preparation: one workgroup per star.
//   W = sum w, wt = w / W, ybar = sum wt y (both compensated), x = y - ybar,
//   a = sum |wt x|.  Fixed point: Wq = rint(wt 2^62), Sq = rint(wt x 2^e) with
//   2^e a <= 2^62, so every window sum fits in int64.  Outputs dt = t - t0 and the
//   exclusive prefix sums CW, CS.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_prepare(const StarDesc* __restrict__ stars, StarRt* __restrict__ rt,
                                                      const double* __restrict__ t, const double* __restrict__ y,
                                                      const double* __restrict__ w, double* __restrict__ dt_out,
                                                      int64_t* __restrict__ cw_out, int64_t* __restrict__ cs_out) {
  __shared__ CSum sc[16];
  __shared__ double sd[16];
  __shared__ int64_t si[32];
  const StarDesc d = stars[blockIdx.x];
  const int64_t n = d.n, off = d.p_off;
  const int tid = threadIdx.x, T = blockDim.x;

  CSum acc{0.0, 0.0};
  for (int64_t i = tid; i < n; i += T) csum_add(acc, w ? w[off + i] : 1.0);
  const double W = block_csum(acc, sc);

  acc = CSum{0.0, 0.0};
  for (int64_t i = tid; i < n; i += T) csum_add(acc, ((w ? w[off + i] : 1.0) / W) * y[off + i]);
  const double ybar = block_csum(acc, sc);

  double aacc = 0.0;
  for (int64_t i = tid; i < n; i += T) {
    const double wt = (w ? w[off + i] : 1.0) / W;
    aacc += fabs(wt * (y[off + i] - ybar));
  }
  const double absum = block_sum(aacc, sd);
  int e = 0;
  if (absum > 0.0) {
    frexp(absum, &e);  // absum < 2^e
  }
  const int es = 62 - e;

  // Contiguous runs per thread for the scans.
  const int64_t run = (n + T - 1) / T;
  const int64_t a = min<int64_t>(n, tid * run), b = min<int64_t>(n, a + run);
  int64_t lw = 0, ls = 0;
  for (int64_t i = a; i < b; ++i) {
    const double wt = (w ? w[off + i] : 1.0) / W;
    lw += static_cast<int64_t>(rint(ldexp(wt, 62)));
    ls += static_cast<int64_t>(rint(ldexp(wt * (y[off + i] - ybar), es)));
  }
  int64_t tw, ts;
  int64_t pw = block_exscan(lw, si, &tw);
  int64_t ps = block_exscan(ls, si, &ts);
  for (int64_t i = a; i < b; ++i) {
    const double wt = (w ? w[off + i] : 1.0) / W;
    cw_out[off + i] = pw;
    cs_out[off + i] = ps;
    pw += static_cast<int64_t>(rint(ldexp(wt, 62)));
    ps += static_cast<int64_t>(rint(ldexp(wt * (y[off + i] - ybar), es)));
    dt_out[off + i] = t[off + i] - d.t0;
  }
  if (tid == 0) {
    StarRt r;
    r.cw_total = tw;
    r.cs_total = ts;
    r.s_scale = ldexp(1.0, -es);
    r.pad = 0.0;
    rt[blockIdx.x] = r;
  }
}

// ----------------------------------------------------------------------------
// Fused fold -> boundary accumulation -> H -> duration/phase scan.
// One workgroup per work item (a frequency range of one star).  LDS layout for the
// F frequencies of the current group, nb_cap bins each (k-major):
//   [  0, 32K)  GW  int64 G of the weights     -> after conversion HW (FP64 H_W)
//   [32K, 64K)  GS  int64 G of the residuals   -> after conversion HS (FP64 H_S)
//   [64K, 96K)  DW  int64 range-add ends at data gaps (weights)
//   [96K,128K)  DS  int64 range-add ends at data gaps (residuals)
// Separate 8-byte arrays keep the boundary atomics of a wave on distinct banks,
// and GS sits at a fixed offset from GW (one address per atomic pair).
// ----------------------------------------------------------------------------
constexpr int kArrBytes = kGBytes / 4;   // 32 KB per array
constexpr int kUGroup = 4;               // points whose bins are computed together
constexpr int kArrElems = kArrBytes / 8; // F * nb_cap <= 4096

struct SearchArgs {
  const StarDesc* stars;
  const StarRt* rt;
  const WorkItem* items;
  const double* dt;
  const int64_t* cw;
  const int64_t* cs;
  const int32_t* gaps;     // per-star lists of points whose step can skip bins
  const int64_t* windows;  // optional (star, i0, i1) triples replacing items
  double* sr;
  bls_best* best;
  Consts c;
};

// Best window of a lane or wave: power s^2 / d kept as the pair (s^2, d) so that
// comparisons need no division; mj = (m << 20) | j orders ties lexicographically.
// The empty state is (-1, 1, ~0): every valid window beats it.
struct ScanBest {
  double ss, d;
  uint32_t mj;
  uint32_t pad;
};

__device__ __forceinline__ bool better(double ssa, double da, uint32_t mja, double ssb, double db, uint32_t mjb) {
  const double x = ssa * db, y = ssb * da;
  return x > y || (x == y && mja < mjb);
}

constexpr int kScanUnroll = 16;  // durations up to this length run fully unrolled

constexpr double kW62 = 2.168404344971008868e-19;  // 2^-62

// Fine bin without the clamp: fract() returns at most 1 - 2^-53, and for any
// integer nb >= 1, (1 - 2^-53) nb rounds to a value below nb, so the truncation
// is at most nb - 1 (the same bin as min(nb-1, floor(frac nb))).
__device__ __forceinline__ int32_t fold_bin_nc(double dt, double f, double nbd) {
  return static_cast<int32_t>(__builtin_amdgcn_fract(dt * f) * nbd);
}

__device__ __forceinline__ void lds_add64(unsigned char* base, uint32_t byte_off, long long v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(base + byte_off), static_cast<unsigned long long>(v));
}

// One pass of the fold over the wave's block for frequencies k0 and, when TWO,
// k0 + 1: a point whose bin differs from its predecessor's is a boundary and adds
// its prefix values into G of its bin.
template <bool TWO>
__device__ __forceinline__ void fold_pass(unsigned char* smem, int stride, int k0, const double* s_f,
                                          const int32_t* s_nb, const double (&dtr)[kUMax],
                                          const long long (&cwr)[kUMax], const long long (&csr)[kUMax],
                                          double dt_before, int run, int lane) {
  const int k1 = TWO ? k0 + 1 : k0;
  const double fa = s_f[k0], fb = s_f[k1];
  const double na = static_cast<double>(s_nb[k0]), nbv = static_cast<double>(s_nb[k1]);
  const uint32_t ga = static_cast<uint32_t>(k0 * stride) * 8u;
  const uint32_t gb = static_cast<uint32_t>(k1 * stride) * 8u;
  // Bin of the point before the block: the predecessor of lane 0 at step 0.
  int32_t carry_a = fold_bin_nc(dt_before, fa, na);
  int32_t carry_b = TWO ? fold_bin_nc(dt_before, fb, nbv) : 0;
#pragma unroll
  for (int u0 = 0; u0 < kUMax; u0 += kUGroup) {
    if (u0 >= run) break;
    // Bins of a group of steps for both frequencies, stage by stage so the
    // independent FP64 chains overlap (the empty asm statements pin the order;
    // without them the compiler sinks each chain into its branch).
    double xa[kUGroup], xb[kUGroup];
    int32_t ba[kUGroup], bb[kUGroup];
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      xa[v] = dtr[u0 + v] * fa;
      if (TWO) xb[v] = dtr[u0 + v] * fb;
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      asm volatile("" : "+v"(xa[v]));
      if (TWO) asm volatile("" : "+v"(xb[v]));
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      xa[v] = __builtin_amdgcn_fract(xa[v]);
      if (TWO) xb[v] = __builtin_amdgcn_fract(xb[v]);
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      asm volatile("" : "+v"(xa[v]));
      if (TWO) asm volatile("" : "+v"(xb[v]));
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      xa[v] = xa[v] * na;
      if (TWO) xb[v] = xb[v] * nbv;
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      asm volatile("" : "+v"(xa[v]));
      if (TWO) asm volatile("" : "+v"(xb[v]));
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      ba[v] = static_cast<int32_t>(xa[v]);
      bb[v] = TWO ? static_cast<int32_t>(xb[v]) : 0;
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) asm volatile("" ::"v"(ba[v]), "v"(bb[v]));
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      const int u = u0 + v;
      // Predecessor bins: lane l-1 of this step (DPP wave shift right by one);
      // lane 0 takes lane 63 of the previous step.
      const int32_t la = v == 0 ? carry_a : __builtin_amdgcn_readlane(ba[v - 1], 63);
      const int32_t pa = __builtin_amdgcn_update_dpp(la, ba[v], 0x138, 0xf, 0xf, false);
      if (ba[v] != pa) {
        const uint32_t o = ga + 8u * static_cast<uint32_t>(ba[v]);
        lds_add64(smem, o, cwr[u]);
        lds_add64(smem, o + kArrBytes, csr[u]);
      }
      if (TWO) {
        const int32_t lb = v == 0 ? carry_b : __builtin_amdgcn_readlane(bb[v - 1], 63);
        const int32_t pb = __builtin_amdgcn_update_dpp(lb, bb[v], 0x138, 0xf, 0xf, false);
        if (bb[v] != pb) {
          const uint32_t o = gb + 8u * static_cast<uint32_t>(bb[v]);
          lds_add64(smem, o, cwr[u]);
          lds_add64(smem, o + kArrBytes, csr[u]);
        }
      }
    }
    carry_a = __builtin_amdgcn_readlane(ba[kUGroup - 1], 63);
    if (TWO) carry_b = __builtin_amdgcn_readlane(bb[kUGroup - 1], 63);
  }
}

__global__ void __launch_bounds__(kSearchThreads) k_search(SearchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  long long* GW = reinterpret_cast<long long*>(smem);
  long long* GS = reinterpret_cast<long long*>(smem + kArrBytes);
  long long* DW = reinterpret_cast<long long*>(smem + 2 * kArrBytes);
  long long* DS = reinterpret_cast<long long*>(smem + 3 * kArrBytes);
  double* HW = reinterpret_cast<double*>(smem);
  double* HS = reinterpret_cast<double*>(smem + kArrBytes);
  double* s_f = reinterpret_cast<double*>(smem + kGBytes);
  int32_t* s_nb = reinterpret_cast<int32_t*>(s_f + kFMax);
  int32_t* s_blast = s_nb + kFMax;
  long long* s_g0w = reinterpret_cast<long long*>(s_blast + kFMax);
  long long* s_g0s = s_g0w + kFMax;
  ScanBest* s_res = reinterpret_cast<ScanBest*>(s_g0s + kFMax);  // [kFMax][16]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  WorkItem it;
  if (a.windows) {
    const int64_t* wv = a.windows + 3 * static_cast<int64_t>(blockIdx.x);
    it.star = static_cast<int32_t>(wv[0]);
    it.i0 = static_cast<int32_t>(wv[1]);
    it.i1 = static_cast<int32_t>(wv[2]);
  } else {
    it = a.items[blockIdx.x];
  }
  const StarDesc d = a.stars[it.star];
  const StarRt rt = a.rt[it.star];
  if (it.i0 < 0) it.i0 = 0;
  if (it.i1 > d.nf) it.i1 = static_cast<int32_t>(d.nf);
  if (it.i1 <= it.i0) return;
  const int64_t n = d.n;
  const double* __restrict__ dt = a.dt + d.p_off;
  const int64_t* __restrict__ cw = a.cw + d.p_off;
  const int64_t* __restrict__ cs = a.cs + d.p_off;
  const int32_t noverlap = a.c.noverlap;

  double f_first;
  int32_t nb_cap;
  grid_point(d, it.i0, noverlap, f_first, nb_cap);
  if (nb_cap > kNbLimit || nb_cap < 1) return;  // rejected by the plan
  // Slot stride: nb_cap bins plus room to replicate the first bins after the
  // last, so windows that wrap past bin nb-1 read contiguously.
  const int stride = nb_cap + kMCap;
  const int F_act = min(kFMax, kArrElems / stride);

  // Points: wave w owns a contiguous block of 64 * run points per chunk; lane l holds
  // points block + 64 u + l, so a point's predecessor is in the previous lane of the
  // same step (lane 0: lane 63 of the previous step).  Loads are coalesced and the
  // boundaries of one step fall on consecutive bins.
  const int T = blockDim.x;
  const int run = static_cast<int>(min<int64_t>(kUMax, (n + T - 1) / T));
  const int64_t chunk_pts = static_cast<int64_t>(run) * T;
  const int nchunks = static_cast<int>((n + chunk_pts - 1) / chunk_pts);
  double dtr[kUMax];
  long long cwr[kUMax], csr[kUMax];
  double dt_before = 0.0;  // time of the point before the wave's block (its first if none)
  bool active = false;
  auto load_chunk = [&](int c) {
    const int64_t wbase = static_cast<int64_t>(c) * chunk_pts + static_cast<int64_t>(wave) * 64 * run;
    active = wbase < n;
    if (!active) return;
    const int64_t wend = min<int64_t>(n, wbase + static_cast<int64_t>(64) * run);
    // Points past the block's end repeat its last point: same bin, no boundary.
#pragma unroll
    for (int u = 0; u < kUMax; ++u) {
      const int64_t q = min<int64_t>(wbase + u * 64 + lane, wend - 1);
      dtr[u] = dt[q];
      cwr[u] = cw[q];
      csr[u] = cs[q];
    }
    dt_before = dt[wbase > 0 ? wbase - 1 : 0];
  };
  if (nchunks == 1) load_chunk(0);
  const double dt_last = dt[n - 1];

  const int waves = T >> 6;
  for (int g0 = it.i0; g0 < it.i1; g0 += F_act) {
    const int F = min(F_act, it.i1 - g0);
    if (tid < F) {
      double f;
      int32_t nb;
      grid_point(d, g0 + tid, noverlap, f, nb);
      s_f[tid] = f;
      s_nb[tid] = nb;
      s_blast[tid] = fold_bin_nc(dt_last, f, static_cast<double>(nb));
    }
    for (int idx = tid; idx < F * stride; idx += T) {
      GW[idx] = 0;
      GS[idx] = 0;
      DW[idx] = 0;
      DS[idx] = 0;
    }
    __syncthreads();

    // ---- fold: a point whose bin differs from its predecessor's is a boundary
    // and adds its prefix values into G of its bin.  Two frequencies per pass give
    // the scheduler two independent chains per point.
    for (int c = 0; c < nchunks; ++c) {
      if (nchunks > 1) load_chunk(c);
      if (!active) continue;
      for (int k0 = 0; k0 < F; k0 += 2) {
        if (k0 + 1 < F)
          fold_pass<true>(smem, stride, k0, s_f, s_nb, dtr, cwr, csr, dt_before, run, lane);
        else
          fold_pass<false>(smem, stride, k0, s_f, s_nb, dtr, cwr, csr, dt_before, run, lane);
      }
    }
    // A point whose time step crosses more than one fine bin (a data gap) belongs
    // to every bin in (bp, b]: G[b] has its prefix values from the fold; adding them
    // to the skipped bins (bp, b-1] changes H = G[b+1] - G[b] only at the two ends
    // of that range, recorded in D: D[bp] += E, D[b-1] -= E.  Only points in the
    // star's gap list can do this (their step is large compared with the bin width
    // at the top of the grid).
    if (d.n_gaps > 0) {
      const int32_t* gl = a.gaps + d.g_off;
      const int total_g = F * d.n_gaps;
      for (int idx = tid; idx < total_g; idx += T) {
        const int k = idx / d.n_gaps;
        const int32_t q = gl[idx - k * d.n_gaps];
        const double f = s_f[k];
        const int32_t nb = s_nb[k];
        const double nbd = static_cast<double>(nb);
        const int32_t bq = fold_bin_nc(dt[q - 1], f, nbd);
        const int32_t bu = fold_bin_nc(dt[q], f, nbd);
        int32_t steps = bu - bq;
        if (steps < 0) steps += nb;
        if (steps > 1) {
          const int32_t bm1 = bu == 0 ? nb - 1 : bu - 1;
          const uint32_t kb = static_cast<uint32_t>(k * stride);
          const long long ew = cw[q], es = cs[q];
          atomicAdd(reinterpret_cast<unsigned long long*>(&DW[kb + bq]), static_cast<unsigned long long>(ew));
          atomicAdd(reinterpret_cast<unsigned long long*>(&DS[kb + bq]), static_cast<unsigned long long>(es));
          atomicAdd(reinterpret_cast<unsigned long long*>(&DW[kb + bm1]), 0ull - static_cast<unsigned long long>(ew));
          atomicAdd(reinterpret_cast<unsigned long long*>(&DS[kb + bm1]), 0ull - static_cast<unsigned long long>(es));
        }
      }
    }
    __syncthreads();

    // ---- G -> H in place, in chunks of T bins (all reads of a chunk precede its
    // writes; the wrap value G[k][0] is saved first) ----
    if (tid < F) {
      s_g0w[tid] = GW[tid * stride];
      s_g0s[tid] = GS[tid * stride];
    }
    __syncthreads();
    const int total = F * stride;
    for (int base = 0; base < total; base += T) {
      const int idx = base + tid;
      bool act = false;
      double hw = 0.0, hs = 0.0;
      if (idx < total) {
        const int k = idx / stride;
        const int b = idx - k * stride;
        const int32_t nb = s_nb[k];
        if (b < nb) {
          act = true;
          const unsigned long long w0 = static_cast<unsigned long long>(GW[idx] - DW[idx]);
          const unsigned long long s0 = static_cast<unsigned long long>(GS[idx] - DS[idx]);
          const unsigned long long w1 = static_cast<unsigned long long>(b + 1 < nb ? GW[idx + 1] : s_g0w[k]);
          const unsigned long long s1 = static_cast<unsigned long long>(b + 1 < nb ? GS[idx + 1] : s_g0s[k]);
          unsigned long long dw = w1 - w0, ds = s1 - s0;
          if (b == s_blast[k]) {
            dw += static_cast<unsigned long long>(rt.cw_total);
            ds += static_cast<unsigned long long>(rt.cs_total);
          }
          hw = static_cast<double>(static_cast<long long>(dw)) * kW62;
          hs = static_cast<double>(static_cast<long long>(ds)) * rt.s_scale;
        }
      }
      __syncthreads();
      if (act) {
        HW[idx] = hw;
        HS[idx] = hs;
      }
      __syncthreads();
    }

    // Replicate the first bins after the last one (windows wrap past nb - 1).
    const int m_max = a.c.m_max;
    for (int idx = tid; idx < F * kMCap; idx += T) {
      const int k = idx / kMCap;
      const int i = idx - k * kMCap;
      const int32_t nb = s_nb[k];
      if (i < min(m_max, nb - 1)) {
        HW[k * stride + nb + i] = HW[k * stride + i];
        HS[k * stride + nb + i] = HS[k * stride + i];
      }
    }
    __syncthreads();

    // ---- scan: every start bin j, durations m of the ladder.  Branch-free running
    // maximum of s^2 / (r (1 - r)) compared as cross products. ----
    const int wpk = F <= waves ? waves / F : 1;  // waves per frequency
    const int kstep = waves / wpk;
    const uint32_t m_mask = a.c.m_mask;
    const bool dip = a.c.dip_only != 0;
    for (int k = wave / wpk; k < F; k += kstep) {
      const int sub = wave - (wave / wpk) * wpk;
      const int32_t nb = s_nb[k];
      const double* hwk = HW + k * stride;
      const double* hsk = HS + k * stride;
      double bss = -1.0, bd = 1.0;
      uint32_t bmj = ~0u;
      const int mlim = min(m_max, nb - 1);
      auto window = [&](int m, int j, double r, double s) {
        const double dd = fma(-r, r, r);  // r (1 - r) > 0  <=>  0 < r < 1
        const double ss = s * s;
        const uint32_t mj = (static_cast<uint32_t>(m) << 20) | static_cast<uint32_t>(j);
        const bool ok = dd > 0.0 && (!dip || s < 0.0);
        if (ok && better(ss, dd, mj, bss, bd, bmj)) {
          bss = ss;
          bd = dd;
          bmj = mj;
        }
      };
      for (int j = sub * 64 + lane; j < nb; j += wpk * 64) {
        double r = 0.0, s = 0.0;
#pragma unroll
        for (int m = 1; m <= kScanUnroll; ++m) {
          if (m <= mlim) {
            r += hwk[j + m - 1];
            s += hsk[j + m - 1];
            if (m_mask & (1u << (m - 1))) window(m, j, r, s);
          }
        }
        for (int m = kScanUnroll + 1; m <= mlim; ++m) {
          r += hwk[j + m - 1];
          s += hsk[j + m - 1];
          if (m_mask & (1u << (m - 1))) window(m, j, r, s);
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double qss = __shfl_xor(bss, o, 64);
        const double qd = __shfl_xor(bd, o, 64);
        const uint32_t qmj = __shfl_xor(bmj, o, 64);
        if (better(qss, qd, qmj, bss, bd, bmj)) {
          bss = qss;
          bd = qd;
          bmj = qmj;
        }
      }
      if (lane == 0) s_res[k * 16 + sub] = ScanBest{bss, bd, bmj, 0u};
    }
    __syncthreads();
    if (tid < F) {
      const int k = tid;
      ScanBest bsel = s_res[k * 16];
      for (int q = 1; q < wpk; ++q) {
        const ScanBest o = s_res[k * 16 + q];
        if (better(o.ss, o.d, o.mj, bsel.ss, bsel.d, bsel.mj)) bsel = o;
      }
      const int64_t fi = d.f_off + g0 + k;
      bls_best bb;
      bb.m = 0;
      bb.j = -1;
      bb.r = 0.0;
      bb.s = 0.0;
      double sr = 0.0;
      if (bsel.mj != ~0u) {
        const int m = static_cast<int>(bsel.mj >> 20), j = static_cast<int>(bsel.mj & 0xFFFFFu);
        const double* hwk = HW + k * stride;
        const double* hsk = HS + k * stride;
        double r = 0.0, s = 0.0;
        for (int u = 0; u < m; ++u) {
          r += hwk[j + u];
          s += hsk[j + u];
        }
        sr = sqrt((s * s) / (r * (1.0 - r)));
        bb.m = m;
        bb.j = j;
        bb.r = r;
        bb.s = s;
      }
      a.sr[fi] = sr;
      if (a.best) a.best[fi] = bb;
    }
    __syncthreads();
  }
}

}  // namespace mi355bls

using namespace mi355bls;

namespace {
bool ws_ok(const bls_plan* plan, const void* ws) {
  return plan && ws && plan->uploaded_to == ws &&
         (reinterpret_cast<uintptr_t>(ws) & 255) == 0;
}
}  // namespace

extern "C" bls_status bls_plan_upload(bls_plan* plan, void* ws, int64_t bytes, bls_stream_t stream) {
  if (!plan || !ws) return BLS_E_ARG;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return BLS_E_ARG;
  if (bytes < plan->layout.total) return BLS_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  if (hipMemcpyAsync(base + plan->layout.stars, plan->stars.data(), sizeof(StarDesc) * plan->stars.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return BLS_E_HIP;
  if (!plan->items.empty() &&
      hipMemcpyAsync(base + plan->layout.items, plan->items.data(), sizeof(WorkItem) * plan->items.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return BLS_E_HIP;
  if (!plan->gaps.empty() &&
      hipMemcpyAsync(base + plan->layout.gaps, plan->gaps.data(), sizeof(int32_t) * plan->gaps.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return BLS_E_HIP;
  plan->uploaded_to = ws;
  return BLS_OK;
}

extern "C" bls_status bls_prepare(bls_plan* plan, void* ws, const double* d_t, const double* d_y,
                                  const double* d_w, bls_stream_t stream) {
  if (!plan || !d_t || !d_y) return BLS_E_ARG;
  if (!ws_ok(plan, ws)) return BLS_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const Layout& L = plan->layout;
  hipLaunchKernelGGL(k_prepare, dim3(plan->n_stars), dim3(kThreads), 0, st,
                     reinterpret_cast<const StarDesc*>(base + L.stars), reinterpret_cast<StarRt*>(base + L.rt),
                     d_t, d_y, d_w, reinterpret_cast<double*>(base + L.dt), reinterpret_cast<int64_t*>(base + L.cw),
                     reinterpret_cast<int64_t*>(base + L.cs));
  if (hipGetLastError() != hipSuccess) return BLS_E_HIP;
  return BLS_OK;
}

extern "C" bls_status bls_search_batch(bls_plan* plan, void* ws, const int64_t* d_windows, int64_t n_windows,
                                       double* d_sr, bls_best* d_best, bls_stream_t stream) {
  if (!plan || !d_sr) return BLS_E_ARG;
  if (!ws_ok(plan, ws)) return BLS_E_STATE;
  if (d_windows && n_windows < 0) return BLS_E_ARG;
  if (n_windows > 0x7fffffff) return BLS_E_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const Layout& L = plan->layout;
  SearchArgs a;
  a.stars = reinterpret_cast<const StarDesc*>(base + L.stars);
  a.rt = reinterpret_cast<const StarRt*>(base + L.rt);
  a.items = reinterpret_cast<const WorkItem*>(base + L.items);
  a.dt = reinterpret_cast<const double*>(base + L.dt);
  a.cw = reinterpret_cast<const int64_t*>(base + L.cw);
  a.cs = reinterpret_cast<const int64_t*>(base + L.cs);
  a.gaps = reinterpret_cast<const int32_t*>(base + L.gaps);
  a.windows = d_windows;
  a.sr = d_sr;
  a.best = d_best;
  a.c = plan->consts;
  const int64_t n_items = d_windows ? n_windows : static_cast<int64_t>(plan->items.size());
  if (n_items == 0) return BLS_OK;
  const size_t lds = kGBytes + kFMax * (8 + 4 + 4 + 8 + 8) + kFMax * 16 * sizeof(ScanBest);
  static_assert(kGBytes + kFMax * 32 + kFMax * 16 * sizeof(ScanBest) <= 160 * 1024, "LDS budget");
  hipLaunchKernelGGL(k_search, dim3(static_cast<unsigned>(n_items)), dim3(kSearchThreads), lds, st, a);
  if (hipGetLastError() != hipSuccess) return BLS_E_HIP;
  return BLS_OK;
}
