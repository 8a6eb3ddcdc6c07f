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
//    cancel; a point that skips bins inside a cycle (a data gap) changes H at two
//    bins, the one it leaves and the one before the one it enters.  Stars where
//    most steps skip bins (cadence coarser than the finest bins) fold in
//    difference form: each boundary adds its values to the bin it enters and
//    subtracts them from the bin it leaves.  Integer sums are exact, so the
//    result does not depend on order.
//  * Points stay in registers (dt, CW, CS) across all frequencies of a work item;
//    only boundaries touch LDS (one 64-bit integer atomic pair per boundary, or,
//    for stars of equal weights, a 32-bit count of weighted points in place of the
//    weight prefix: counts.hpp).
//  * The phase frac((t - t0) f) is computed in FP64 with the same IEEE operations
//    as the grid (this file is compiled with -ffp-contract=off), so the bin of
//    every point is bit-identical to a sequential FP64 evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "counts.hpp"
#include "plan.hpp"

namespace mi355bls {

// EXQ: the exact circular duration (its arcsine only in the kernels that need it,
// so that the others' register allocation does not carry it).
template <bool EXQ>
__device__ __forceinline__ void grid_point(const StarDesc& d, int64_t i, const Consts& c, double& f, int32_t& nb) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  const double uu = u * u;
  f = uu * u;
  if constexpr (EXQ)
    nb = fine_bins(d, c, uu);
  else
    nb = static_cast<int32_t>(ceil(static_cast<double>(c.noverlap) / (d.kq * uu)));
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

// Block reduction of one value per thread with an associative, commutative op.
template <typename T, typename Op>
__device__ T block_reduce(T v, T* scratch, Op op) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T r = scratch[0];
  for (int q = 1; q < static_cast<int>(blockDim.x >> 6); ++q) r = op(r, scratch[q]);
  __syncthreads();
  return r;
}

// Exclusive block scan of one integer per thread (unsigned: wraps modulo 2^64);
// returns the total through *total.
template <typename I>
__device__ I block_exscan(I v, I* scratch, I* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  I x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const I y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  if (wave == 0) {
    const int nw = blockDim.x >> 6;
    I s = lane < nw ? scratch[lane] : I(0);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const I y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < nw) scratch[lane] = s;  // inclusive per wave
  }
  __syncthreads();
  const I wave_off = wave > 0 ? scratch[wave - 1] : I(0);
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

// Kinds of star in a prepared batch (precision 0), or-ed into one flags word.
constexpr unsigned kHasEqualWeights = 1u, kHasUnequalWeights = 2u;

// ----------------------------------------------------------------------------
// Preparation: one workgroup per star.
//   W = sum w, wt = w / W, ybar = sum wt y (both compensated), x = y - ybar,
//   a = sum |wt x|.  Fixed point (precision 0): Wq = rint(wt 2^62), Sq = rint(wt x
//   2^es) with 2^-es a <= 2^62, so every window sum fits in int64; outputs the
//   exclusive prefix sums CW, CS.  Packed (precision 1): Wq = rint(wt 2^27) in the
//   high 28 bits and Sq = rint(wt x 2^es) with a 2^es <= 2^34 in the low 36 bits of
//   one integer, one prefix sum modulo 2^64 in CW.  Also dt = t - t0.  The scans run
//   tile by tile over the star (coalesced), carrying the running total.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_prepare(const StarDesc* __restrict__ stars, StarRt* __restrict__ rt,
                                                      const double* __restrict__ t, const double* __restrict__ y,
                                                      const double* __restrict__ w, double* __restrict__ dt_out,
                                                      int64_t* __restrict__ cw_out, int64_t* __restrict__ cs_out,
                                                      int32_t packed, unsigned int* __restrict__ flags) {
  __shared__ CSum sc[16];
  __shared__ double sd[16];
  __shared__ unsigned long long si[32];
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
  const int es = (packed ? 34 : 62) - e;

  unsigned long long carry_w = 0, carry_s = 0;
  unsigned long long qmin = ~0ull, qmax = 0ull;  // nonzero fixed-point weights (precision 0)
  for (int64_t base = 0; base < n; base += T) {
    const int64_t i = base + tid;
    unsigned long long qw = 0, qs = 0;
    if (i < n) {
      const double wt = (w ? w[off + i] : 1.0) / W;
      const long long sq = static_cast<long long>(rint(ldexp(wt * (y[off + i] - ybar), es)));
      if (packed) {
        qw = (static_cast<unsigned long long>(rint(ldexp(wt, kPackWBits))) << kPackShift) +
             static_cast<unsigned long long>(sq);
      } else {
        qw = static_cast<unsigned long long>(static_cast<long long>(rint(ldexp(wt, 62))));
        qs = static_cast<unsigned long long>(sq);
        if (qw != 0ull) {
          qmin = min(qmin, qw);
          qmax = max(qmax, qw);
        }
      }
    }
    unsigned long long tw, ts = 0;
    const unsigned long long pw = block_exscan<unsigned long long>(qw, si, &tw);
    unsigned long long ps = 0;
    if (!packed) ps = block_exscan<unsigned long long>(qs, si, &ts);
    if (i < n) {
      cw_out[off + i] = static_cast<int64_t>(carry_w + pw);
      if (!packed) cs_out[off + i] = static_cast<int64_t>(carry_s + ps);
      dt_out[off + i] = t[off + i] - d.t0;
    }
    carry_w += tw;
    carry_s += ts;
  }
  // One fixed-point weight for every weighted point (equal weights, zeros aside):
  // the search may then accumulate counts of points instead of weight prefixes.
  int64_t w_unit = 0;
  if (!packed) {
    qmin = block_reduce(qmin, si, [](unsigned long long x, unsigned long long z) { return min(x, z); });
    qmax = block_reduce(qmax, si, [](unsigned long long x, unsigned long long z) { return max(x, z); });
    if (qmax != 0ull && qmin == qmax && n < (int64_t{1} << 31)) w_unit = static_cast<int64_t>(qmax);
  }
  if (tid == 0) {
    StarRt r;
    r.cw_total = static_cast<int64_t>(carry_w);
    r.cs_total = static_cast<int64_t>(carry_s);
    r.s_scale = ldexp(1.0, -es);
    r.w_unit = w_unit;
    rt[blockIdx.x] = r;
    if (!packed) atomicOr(flags, w_unit != 0 ? kHasEqualWeights : kHasUnequalWeights);
  }
}

// ----------------------------------------------------------------------------
// Fused fold -> boundary accumulation -> H -> duration/phase scan.
// A persistent grid pulls work items (a frequency range of one star) from a
// counter.  Common shape: 48 KB of accumulators (plus the group's scalars) per
// workgroup and at most 80 registers per lane let three workgroups share a CU (six
// waves per SIMD), so some fold (LDS-atomic bound) while others scan (VALU bound).
// Large shape: 72 KB and 128 registers, two per CU.  LDS layout for the F
// frequencies of the current group, `stride` slots each (k-major):
//   [0, W/2)  GW  int64 G of the weights   -> FP64 H_W
//   [W/2, W)  GS  int64 G of the residuals -> FP64 H_S     (W = 48 KB or 72 KB)
// GS sits at a fixed offset from GW, so one address serves each atomic pair.
// ----------------------------------------------------------------------------
constexpr int kUGroup = 4;                // points whose bins are computed together

// LDS window of a workgroup shape (BIG: the large one).  A group searches the
// frequencies whose fine-bin count lies in (nb_lo, nb_hi].
template <bool BIG>
struct Win {
  static constexpr int bytes = BIG ? kGBytesBig : kGBytes;
  static constexpr int arr_bytes = bytes / 2;                // per array (G_W, G_S)
  static constexpr int elems = arr_bytes / 8;                // F * stride <= elems
  static constexpr int threads = BIG ? kSearchThreadsBig : kSearchThreads;
  static constexpr int slot_iter = (elems + threads - 1) / threads;  // slots per thread (scan)
  static constexpr int nb_lo = BIG ? kNbLimit : 0;
  static constexpr int nb_hi = BIG ? kNbLimitBig : kNbLimit;
  static constexpr int groups = BIG ? kSearchGroupsPerCuBig : kSearchGroupsPerCu;
  static constexpr int um = BIG ? kUMaxBig : kUMaxSmall;     // register points per thread
};
static_assert(kUMax % kUGroup == 0 && kUMaxSmall % kUGroup == 0 && kUMaxBig % kUGroup == 0,
              "the folds take whole groups of steps");
// A large-shape group of a star that is not long holds one frequency (two with
// more than kNbLimit bins do not fit), so it never reaches frequencies of the
// common shape.
static_assert(2 * (kNbLimit + 1) > Win<true>::elems, "one frequency per large-shape group");
// Scan slots per thread of k_search_wide (512 threads over the large window).
constexpr int kWideSlotIter = (Win<true>::elems + kSearchThreads - 1) / kSearchThreads;

struct SearchArgs {
  const StarDesc* stars;
  const StarRt* rt;
  const WorkItem* items;
  const double* dt;
  const int64_t* cw;
  const int64_t* cs;
  const int32_t* gaps;     // per-star lists of points whose step can skip bins
  const double* gap_steps; // their time steps (each list ordered largest first)
  const int64_t* windows;  // optional (star, i0, i1) triples replacing items
  double* sr;
  bls_best* best;
  unsigned int* next;      // per-XCD work counters, kCounterStride apart (zeroed by k_reset)
  int32_t n_items;
  int32_t n_stars;
  Consts c;
};

// Per-group scalars after the two accumulator arrays.
// Gap points of a work item (up to one per lane) are kept in LDS for the whole
// item; stars with more fold in difference form.
constexpr int kGapCache = kGapLanes;
struct GroupLds {
  double f[kFMax];
  int32_t nb[kFMax];
  int32_t blast[kFMax];               // bin of the last point (receives the totals)
  unsigned long long key[kFMax];      // 1 + bits of the best power (0: no valid window)
  uint32_t mj[kFMax];                 // smallest (m << 20 | j) reaching that power
  int32_t item[2];
  double gdt0[kGapCache], gdt1[kGapCache];   // dt of the point before each gap point, and its own
  long long gcw[kGapCache], gcs[kGapCache];  // prefix values at each gap point
};
template <bool BIG>
constexpr size_t search_lds() {
  return Win<BIG>::bytes + sizeof(GroupLds);
}
static_assert(kSearchGroupsPerCu * search_lds<false>() <= 160 * 1024, "common search workgroups per CU");
static_assert(kSearchGroupsPerCuBig * search_lds<true>() <= 160 * 1024, "large search workgroups per CU");

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int src) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), src));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), src));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ bool better(double ssa, double da, uint32_t mja, double ssb, double db, uint32_t mjb) {
  const double x = ssa * db, y = ssb * da;
  return x > y || (x == y && mja < mjb);
}

constexpr double kW62 = 2.168404344971008868e-19;  // 2^-62

// Fine bin without the clamp: fract() returns at most 1 - 2^-53, and for any
// integer nb >= 1, (1 - 2^-53) nb rounds to a value below nb, so the truncation
// is at most nb - 1 (the same bin as min(nb-1, floor(frac nb))).
__device__ __forceinline__ int32_t fold_bin_nc(double dt, double f, double nbd) {
  return static_cast<int32_t>(__builtin_amdgcn_fract(dt * f) * nbd);
}

// Predecessor bins of step v (see the point layout in k_search): even steps shift
// right by one lane, odd steps left; the lane without a source keeps `old`, the
// same lane's bin one step earlier.
__device__ __forceinline__ int32_t pred_bin(int v, int32_t old, int32_t src) {
  return (v & 1) ? __builtin_amdgcn_update_dpp(old, src, 0x130, 0xf, 0xf, false)
                 : __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ void lds_add64(unsigned char* base, uint32_t byte_off, long long v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(base + byte_off), static_cast<unsigned long long>(v));
}

__device__ __forceinline__ void lds_sub64(unsigned char* base, uint32_t byte_off, long long v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(base + byte_off), 0ull - static_cast<unsigned long long>(v));
}

// Counts of weighted points (equal weights): a 32-bit add into the low word of the
// bin's 8-byte slot.  A 32-bit LDS atomic issues in about two thirds of the time of
// a 64-bit one on gfx950, and telescoped differences of counts are exact modulo 2^32.
__device__ __forceinline__ void lds_add64(unsigned char* base, uint32_t byte_off, uint32_t v) {
  atomicAdd(reinterpret_cast<unsigned int*>(base + byte_off), v);
}

__device__ __forceinline__ void lds_sub64(unsigned char* base, uint32_t byte_off, uint32_t v) {
  atomicAdd(reinterpret_cast<unsigned int*>(base + byte_off), 0u - v);
}

// Slot index -> (frequency k, bin b) for idx < F * stride <= 4096: a float
// estimate of idx / stride corrected by one step either way.
__device__ __forceinline__ void slot_of(int idx, int stride, float inv_stride, int& k, int& b) {
  k = static_cast<int>(static_cast<float>(idx) * inv_stride);
  b = idx - k * stride;
  if (b < 0) {
    --k;
    b += stride;
  } else if (b >= stride) {
    ++k;
    b -= stride;
  }
}

// Accumulation forms of the fold (uniform per launch).
//  kTelescope: a boundary adds its prefix values to G of the bin it enters;
//              H[b] = G[b+1] - G[b] (+ corrections at data gaps).
//  kDiff:      a boundary subtracts its prefix values from the bin it enters and
//              adds them to the bin it leaves, so G holds each bin's sums (exits
//              minus entries of every visit) apart from the last visit's exit.
constexpr int kTelescope = 0, kDiff = 1;

// One pass of the fold over the wave's block for frequencies k0 and, when TWO,
// k0 + 1: a point whose bin differs from its predecessor's is a boundary.
// WV: the weight values held per point (long long: prefixes CW; uint32_t: counts of
// weighted points, equal weights).
template <bool TWO, bool PACKED, int UM, int ARR, typename WV>
__device__ __forceinline__ void fold_pass(unsigned char* smem, int stride, int k0, const GroupLds* g,
                                          const double (&dtr)[UM], const WV (&cwr)[UM],
                                          const long long (&csr)[UM], double dt_before, int run, int form) {
  const int k1 = TWO ? k0 + 1 : k0;
  const double fa = g->f[k0], fb = g->f[k1];
  const double na = static_cast<double>(g->nb[k0]), nbv = static_cast<double>(g->nb[k1]);
  uint32_t ga = static_cast<uint32_t>(k0 * stride) * 8u;
  uint32_t gb = static_cast<uint32_t>(k1 * stride) * 8u;
  asm volatile("" : "+s"(ga), "+s"(gb));  // keep base + 8 b as one shift-add
  // Bins of the previous step; lane 0 of the first step takes the bin of the point
  // before the block (uniform).
  int32_t prev_a = fold_bin_nc(dt_before, fa, na);
  int32_t prev_b = TWO ? fold_bin_nc(dt_before, fb, nbv) : 0;
#pragma unroll
  for (int u0 = 0; u0 < UM; u0 += kUGroup) {
    if (u0 >= run) break;
    // Bins of a group of steps for both frequencies, stage by stage so the
    // independent FP64 chains overlap (the compiler's own schedule of these
    // stages measured faster than one pinned with empty asm statements).
    double xa[kUGroup], xb[kUGroup];
    int32_t ba[kUGroup], bb[kUGroup];
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      xa[v] = dtr[u0 + v] * fa;
      if (TWO) xb[v] = dtr[u0 + v] * fb;
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      xa[v] = __builtin_amdgcn_fract(xa[v]);
      if (TWO) xb[v] = __builtin_amdgcn_fract(xb[v]);
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      xa[v] = xa[v] * na;
      if (TWO) xb[v] = xb[v] * nbv;
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      ba[v] = static_cast<int32_t>(xa[v]);
      bb[v] = TWO ? static_cast<int32_t>(xb[v]) : 0;
    }
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      const int u = u0 + v;
      // Predecessor bins: even steps shift right by one lane (lane 0 keeps the
      // previous step's value of lane 0), odd steps shift left (lane 63 keeps it).
      const int32_t pa = pred_bin(v, v == 0 ? prev_a : ba[v - 1], ba[v]);
      if (ba[v] != pa) {
        const uint32_t o = ga + 8u * static_cast<uint32_t>(ba[v]);
        if (form == kDiff) {
          const uint32_t op = ga + 8u * static_cast<uint32_t>(pa);
          lds_sub64(smem, o, cwr[u]);
          lds_add64(smem, op, cwr[u]);
          if (!PACKED) {
            lds_sub64(smem, o + ARR, csr[u]);
            lds_add64(smem, op + ARR, csr[u]);
          }
        } else {
          lds_add64(smem, o, cwr[u]);
          if (!PACKED) lds_add64(smem, o + ARR, csr[u]);
        }
      }
      if (TWO) {
        const int32_t pb = pred_bin(v, v == 0 ? prev_b : bb[v - 1], bb[v]);
        if (bb[v] != pb) {
          const uint32_t o = gb + 8u * static_cast<uint32_t>(bb[v]);
          if (form == kDiff) {
            const uint32_t op = gb + 8u * static_cast<uint32_t>(pb);
            lds_sub64(smem, o, cwr[u]);
            lds_add64(smem, op, cwr[u]);
            if (!PACKED) {
              lds_sub64(smem, o + ARR, csr[u]);
              lds_add64(smem, op + ARR, csr[u]);
            }
          } else {
            lds_add64(smem, o, cwr[u]);
            if (!PACKED) lds_add64(smem, o + ARR, csr[u]);
          }
        }
      }
    }
    prev_a = ba[kUGroup - 1];
    if (TWO) prev_b = bb[kUGroup - 1];
  }
}

// Work queue.  MI355X has 8 XCDs, each with its own L2, and consecutive workgroups
// of a launch go to consecutive XCDs.  The cost-ordered item list is cut into
// chunks of kQueueChunk items dealt round-robin to 8 queues; a workgroup drains
// the queue of its own XCD first (blockIdx mod 8), so the items of one star, which
// are adjacent in the list, run on one XCD and share its L2, then helps the other
// queues.  Each queue's item index only grows, so a queue found empty stays empty
// and every workgroup stops after at most 8 empty probes.
constexpr int kXcds = 8;
constexpr int kQueueChunk = 16;
constexpr int kCounterStride = 16;  // 64 bytes between counters

// After the counters: which kinds of star the prepared batch holds (precision 0),
// set by k_prepare and read by the exact telescoping launches.
constexpr int kFlagsIndex = kXcds * kCounterStride;

// Zero the work counters on the stream (a kernel, so the sequence can be captured).
__global__ void k_reset(unsigned int* next) {
  if (threadIdx.x < kXcds) next[threadIdx.x * kCounterStride] = 0u;
}

__global__ void k_clear_flags(unsigned int* next) {
  if (threadIdx.x == 0) next[kFlagsIndex] = 0u;
}

// Packed total -> (weight units, residual units).
__device__ __forceinline__ void unpack_units(unsigned long long h, unsigned long long& wsum, long long& ssum) {
  ssum = static_cast<long long>(h << (64 - kPackShift)) >> (64 - kPackShift);
  wsum = (h - static_cast<unsigned long long>(ssum)) >> kPackShift;
}

// Packed bin total -> (weight fraction, residual).  The weight is divided by the
// star's quantised total rather than taken in units of 2^-27: with equal weights
// every point rounds the same way, and only the ratio stays exact.
__device__ __forceinline__ void unpack(unsigned long long h, double s_scale, double w_unit, double& vw,
                                       double& vs) {
  unsigned long long wsum;
  long long ssum;
  unpack_units(h, wsum, ssum);
  vw = static_cast<double>(wsum) * w_unit;
  vs = static_cast<double>(ssum) * s_scale;
}

// Number of leading entries >= thr of steps[0, ng) (ordered largest first), by the
// 64 lanes of one wave: each round probes 64 evenly spaced entries and keeps the
// interval where the entries fall below thr (three rounds cover 262,144 entries).
__device__ int count_at_least(const double* __restrict__ steps, int ng, double thr) {
  const int lane = threadIdx.x & 63;
  int lo = 0, hi = ng;  // the count lies in [lo, hi]
  while (lo < hi) {
    const int step = (hi - lo + 63) / 64;
    const int pos = lo + lane * step;
    const unsigned long long m = __ballot(pos < hi && steps[pos] >= thr);
    const int c = __popcll(m);  // probes below the count (a prefix of the lanes)
    if (c == 0) break;          // steps[lo] < thr: the count is lo
    const int nlo = lo + (c - 1) * step + 1;
    hi = min(hi, lo + c * step);
    lo = nlo;
  }
  return lo;
}

// Next work item of this workgroup (the same for all its threads), or false when
// every queue is empty.  `queue` and `probes` are thread 0's state.  With
// `count_gaps`, a caller window also gets the number of gap points that can skip
// bins in its frequency range (plan items carry theirs).
__device__ bool next_item(const SearchArgs& a, GroupLds* g, int& queue, int& probes, WorkItem& it,
                          bool count_gaps = false) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    int32_t item = -1;
    while (probes < kXcds) {
      const unsigned t = atomicAdd(&a.next[queue * kCounterStride], 1u);
      const int64_t chunk = static_cast<int64_t>(t / kQueueChunk) * kXcds + queue;
      const int64_t cand = chunk * kQueueChunk + t % kQueueChunk;
      if (cand < a.n_items) {
        item = static_cast<int32_t>(cand);
        break;
      }
      queue = (queue + 1) % kXcds;
      ++probes;
    }
    g->item[0] = item;
  }
  __syncthreads();
  const int32_t item = g->item[0];
  __syncthreads();
  if (item < 0) return false;  // every wave of the group leaves together
  if (a.windows) {
    // Caller triples: a star outside the batch is skipped (empty range), the range
    // is clipped to the star's grid (in 64 bits, before narrowing).
    const int64_t* wv = a.windows + 3 * static_cast<int64_t>(item);
    const int64_t ws = wv[0];
    if (ws < 0 || ws >= a.n_stars) {
      it.star = 0;
      it.i0 = it.i1 = 0;
      it.n_gaps = -1;
      return true;
    }
    const StarDesc& d = a.stars[ws];
    const int64_t nfs = d.nf;
    it.star = static_cast<int32_t>(ws);
    it.i0 = static_cast<int32_t>(max<int64_t>(0, min<int64_t>(wv[1], nfs)));
    it.i1 = static_cast<int32_t>(max<int64_t>(0, min<int64_t>(wv[2], nfs)));
    it.n_gaps = -1;
    if (count_gaps && it.i1 > it.i0 && d.n_gaps > 0) {
      // the same bound as the plan's: steps below 0.99 / (f nb) at the range's top
      // frequency, f nb <= noverlap f^(1/3) / kq + f, move at most one bin
      if (tid < 64) {
        double f;
        int32_t nb;
        grid_point<false>(d, it.i1 - 1, a.c, f, nb);  // f only
        const double thr = 0.99 / (static_cast<double>(a.c.noverlap) * cbrt(f) / d.kq + f);
        const int c = count_at_least(a.gap_steps + d.g_off, d.n_gaps, thr);
        if (tid == 0) g->item[1] = c;
      }
      __syncthreads();
      it.n_gaps = g->item[1];
    }
  } else {
    it = a.items[item];
  }
  return true;
}

__device__ __forceinline__ double packed_w_unit(const StarRt& rt) {
  unsigned long long wt_units;
  long long st_units;
  unpack_units(static_cast<unsigned long long>(rt.cw_total), wt_units, st_units);
  return 1.0 / static_cast<double>(wt_units);
}

// ----------------------------------------------------------------------------
// Wide frequencies: more fine bins than one group's LDS holds (long periods of
// dense stars on long baselines).  One frequency is searched in passes over bin
// ranges: pass p keeps G of the nslot = span + m_max + 1 consecutive bins starting
// at b0 = p * span (slot i is bin (b0 + i) mod nb), so every window starting in
// [b0, b0 + span) lies inside the slots; the fold adds only boundaries whose bin
// falls in the range.  The best window over all passes is kept by thread 0.
// ----------------------------------------------------------------------------
template <bool PACKED>
__device__ __forceinline__ void fold_wide(unsigned char* smem, double f, double nbd, int32_t nb, int32_t b0,
                                          int32_t nslot, const double (&dtr)[kUMax], const long long (&cwr)[kUMax],
                                          const long long (&csr)[kUMax], double dt_before, int run) {
  int32_t prev = fold_bin_nc(dt_before, f, nbd);
#pragma unroll
  for (int u0 = 0; u0 < kUMax; u0 += kUGroup) {
    if (u0 >= run) break;
    double x[kUGroup];
    int32_t bb[kUGroup];
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) x[v] = dtr[u0 + v] * f;
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) asm volatile("" : "+v"(x[v]));
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) x[v] = __builtin_amdgcn_fract(x[v]);
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) asm volatile("" : "+v"(x[v]));
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) x[v] = x[v] * nbd;
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) asm volatile("" : "+v"(x[v]));
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) bb[v] = static_cast<int32_t>(x[v]);
#pragma unroll
    for (int v = 0; v < kUGroup; ++v) {
      const int u = u0 + v;
      const int32_t pa = pred_bin(v, v == 0 ? prev : bb[v - 1], bb[v]);
      int32_t slot = bb[v] - b0;
      if (slot < 0) slot += nb;
      if (bb[v] != pa && slot < nslot) {
        const uint32_t o = 8u * static_cast<uint32_t>(slot);
        lds_add64(smem, o, cwr[u]);
        if (!PACKED) lds_add64(smem, o + Win<true>::arr_bytes, csr[u]);
      }
    }
    prev = bb[kUGroup - 1];
  }
}

template <bool PACKED, bool EXQ>
__device__ void wide_frequency(unsigned char* smem, GroupLds* g, const SearchArgs& a, const StarDesc& d,
                               const StarRt& rt, int fi, double w_unit, const double* __restrict__ dt,
                               const int64_t* __restrict__ cw, const int64_t* __restrict__ cs, int nchunks, int run,
                               int64_t chunk_pts, double dt_last) {
  long long* GW = reinterpret_cast<long long*>(smem);
  long long* GS = reinterpret_cast<long long*>(smem + Win<true>::arr_bytes);
  double* HW = reinterpret_cast<double*>(smem);
  double* HS = reinterpret_cast<double*>(smem + Win<true>::arr_bytes);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, T = kSearchThreads;
  const int m_max = a.c.m_max;
  const uint32_t m_mask = a.c.m_mask;
  const bool dip = a.c.dip_only != 0;
  const int64_t n = d.n;
  double f;
  int32_t nb;
  grid_point<EXQ>(d, fi, a.c, f, nb);
  const double nbd = static_cast<double>(nb);
  const int32_t blast = fold_bin_nc(dt_last, f, nbd);
  const int mlim = min(m_max, nb - 1);
  const int per_pass = Win<true>::elems - m_max - 1;
  // at least two passes, so that nslot < nb and no two slots alias one bin
  const int passes = max(2, (nb + per_pass - 1) / per_pass);
  const int span = (nb + passes - 1) / passes;
  const int nslot = span + m_max + 1;  // G slots; H is defined on the first nslot - 1
  const bool gaps = d.n_gaps > 0;
  unsigned long long rkey = 0ull;      // running best of the passes (thread 0)
  uint32_t rmj = ~0u;
  double rr = 0.0, rs = 0.0;
  for (int p = 0; p < passes; ++p) {
    const int32_t b0 = p * span;
    for (int i = tid; i < nslot; i += T) {
      GW[i] = 0;
      GS[i] = 0;
    }
    if (tid == 0) {
      g->key[0] = 0ull;
      g->mj[0] = ~0u;
    }
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const int64_t wbase = static_cast<int64_t>(c) * chunk_pts + static_cast<int64_t>(wave) * 64 * run;
      if (wbase >= n) continue;
      const int64_t wend = min<int64_t>(n, wbase + static_cast<int64_t>(64) * run);
      double dtr[kUMax];
      long long cwr[kUMax], csr[kUMax];
#pragma unroll
      for (int u = 0; u < kUMax; ++u) {
        const int64_t q = min<int64_t>(wbase + u * 64 + ((u & 1) ? 63 - lane : lane), wend - 1);
        dtr[u] = dt[q];
        cwr[u] = cw[q];
        csr[u] = PACKED ? 0 : cs[q];
      }
      const double dt_before = dt[wbase > 0 ? wbase - 1 : 0];
      fold_wide<PACKED>(smem, f, nbd, nb, b0, nslot, dtr, cwr, csr, dt_before, run);
    }
    __syncthreads();
    // H on slots [0, nslot - 1), by wave 0 in place (64 slots at a time; the next
    // chunk's first slot is read before that chunk is written).
    if (wave == 0) {
      for (int i0 = 0; i0 < nslot - 1; i0 += 64) {
        const int i = i0 + lane;
        if (i < nslot - 1) {
          int32_t bin = b0 + i;
          if (bin >= nb) bin -= nb;
          unsigned long long dw = static_cast<unsigned long long>(GW[i + 1]) - static_cast<unsigned long long>(GW[i]);
          unsigned long long ds =
              PACKED ? 0ull : static_cast<unsigned long long>(GS[i + 1]) - static_cast<unsigned long long>(GS[i]);
          if (bin == blast) {
            dw += static_cast<unsigned long long>(rt.cw_total);
            ds += static_cast<unsigned long long>(rt.cs_total);
          }
          if (gaps) {
            GW[i] = static_cast<long long>(dw);
            if (!PACKED) GS[i] = static_cast<long long>(ds);
          } else {
            double vw, vs;
            if (PACKED) {
              unpack(dw, rt.s_scale, w_unit, vw, vs);
            } else {
              vw = static_cast<double>(static_cast<long long>(dw)) * kW62;
              vs = static_cast<double>(static_cast<long long>(ds)) * rt.s_scale;
            }
            HW[i] = vw;
            HS[i] = vs;
          }
        }
      }
    }
    __syncthreads();
    if (gaps) {
      const int32_t* gl = a.gaps + d.g_off;
      for (int idx = tid; idx < d.n_gaps; idx += T) {
        const int32_t q = gl[idx];
        const int32_t bq = fold_bin_nc(dt[q - 1], f, nbd);
        const int32_t bu = fold_bin_nc(dt[q], f, nbd);
        int32_t steps = bu - bq;
        if (steps < 0) steps += nb;
        if (steps > 1) {
          const int32_t bm1 = bu == 0 ? nb - 1 : bu - 1;
          int32_t s0 = bq - b0, s1 = bm1 - b0;
          if (s0 < 0) s0 += nb;
          if (s1 < 0) s1 += nb;
          const long long ew = cw[q];
          const long long es = PACKED ? 0 : cs[q];
          if (s0 < nslot - 1) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&GW[s0]), static_cast<unsigned long long>(ew));
            if (!PACKED) atomicAdd(reinterpret_cast<unsigned long long*>(&GS[s0]), static_cast<unsigned long long>(es));
          }
          if (s1 < nslot - 1) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&GW[s1]), 0ull - static_cast<unsigned long long>(ew));
            if (!PACKED)
              atomicAdd(reinterpret_cast<unsigned long long*>(&GS[s1]), 0ull - static_cast<unsigned long long>(es));
          }
        }
      }
      __syncthreads();
      for (int i = tid; i < nslot - 1; i += T) {
        double vw, vs;
        if (PACKED) {
          unpack(static_cast<unsigned long long>(GW[i]), rt.s_scale, w_unit, vw, vs);
        } else {
          vw = static_cast<double>(GW[i]) * kW62;
          vs = static_cast<double>(GS[i]) * rt.s_scale;
        }
        HW[i] = vw;
        HS[i] = vs;
      }
      __syncthreads();
    }
    // scan of the windows starting in [b0, b0 + span)
    unsigned long long skey[kWideSlotIter];
    uint32_t smj[kWideSlotIter];
#pragma unroll
    for (int r = 0; r < kWideSlotIter; ++r) {
      const int j = tid + r * T;
      skey[r] = 0ull;
      smj[r] = ~0u;
      if (j < span && b0 + j < nb) {
        double bss = -1.0, bd = 1.0;
        uint32_t bmj = ~0u;
        double rv = 0.0, sv = 0.0;
        for (int m = 1; m <= mlim; ++m) {
          rv += HW[j + m - 1];
          sv += HS[j + m - 1];
          if (m_mask & (1u << (m - 1))) {
            const double dd = fma(-rv, rv, rv);
            const double ss = sv * sv;
            const uint32_t mj = (static_cast<uint32_t>(m) << 20) | static_cast<uint32_t>(b0 + j);
            if (dd > 0.0 && (!dip || sv < 0.0) && better(ss, dd, mj, bss, bd, bmj)) {
              bss = ss;
              bd = dd;
              bmj = mj;
            }
          }
        }
        if (bmj != ~0u) {
          skey[r] = static_cast<unsigned long long>(__double_as_longlong(bss / bd)) + 1ull;
          smj[r] = bmj;
          atomicMax(&g->key[0], skey[r]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kWideSlotIter; ++r)
      if (skey[r] != 0ull && skey[r] == g->key[0]) atomicMin(&g->mj[0], smj[r]);
    __syncthreads();
    if (tid == 0) {
      const unsigned long long kp = g->key[0];
      const uint32_t mp = g->mj[0];
      if (kp != 0ull && (kp > rkey || (kp == rkey && mp < rmj))) {
        rkey = kp;
        rmj = mp;
        const int m = static_cast<int>(mp >> 20);
        const int slot = static_cast<int>(mp & 0xFFFFFu) - b0;
        double r = 0.0, s = 0.0;
        for (int u = 0; u < m; ++u) {
          r += HW[slot + u];
          s += HS[slot + u];
        }
        rr = r;
        rs = s;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t out = d.f_off + fi;
    bls_best bb;
    bb.m = 0;
    bb.j = -1;
    bb.r = 0.0;
    bb.s = 0.0;
    double sr = 0.0;
    if (rkey != 0ull) {
      sr = sqrt((rs * rs) / (rr * (1.0 - rr)));
      bb.m = static_cast<int32_t>(rmj >> 20);
      bb.j = static_cast<int32_t>(rmj & 0xFFFFFu);
      bb.r = rr;
      bb.s = rs;
    }
    a.sr[out] = sr;
    if (a.best) a.best[out] = bb;
  }
}

// DFORM: this launch searches the stars with more than kGapLanes gap points (in
// difference form) and skips the others; without it, the reverse.  Two kernels
// keep the register allocation of the common case free of the second form.
// DIP: only windows with s < 0 (dips) count.  BIG: the large workgroup shape, for
// the frequencies whose fine-bin count lies in (kNbLimit, kNbLimitBig] and for every
// frequency up to kNbLimitBig bins of stars with more than big_points points.
template <bool PACKED, bool DFORM, bool DIP, bool BIG, bool EXQ, bool CNT>
__global__ void __launch_bounds__(Win<BIG>::threads, Win<BIG>::groups * Win<BIG>::threads / 256) k_search(SearchArgs a) {
  static_assert(!CNT || !PACKED, "counts replace the weight prefixes of the exact sums");
  using W = Win<BIG>;
  extern __shared__ __align__(16) unsigned char smem[];
  long long* GW = reinterpret_cast<long long*>(smem);
  long long* GS = reinterpret_cast<long long*>(smem + W::arr_bytes);
  double* HW = reinterpret_cast<double*>(smem);
  double* HS = reinterpret_cast<double*>(smem + W::arr_bytes);
  GroupLds* g = reinterpret_cast<GroupLds*>(smem + W::bytes);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int T = W::threads;
  const int m_max = a.c.m_max;
  const uint32_t m_mask = a.c.m_mask;

  // Exact sums: the stars of equal weights (counts) and the others run in separate
  // launches; k_prepare flags which kinds the batch holds, so a launch with nothing
  // to do ends here.
  if constexpr (!PACKED) {
    if ((a.next[kFlagsIndex] & (CNT ? kHasEqualWeights : kHasUnequalWeights)) == 0u) return;
  }
  int queue = static_cast<int>(blockIdx.x % kXcds);  // used by thread 0 only
  int probes = 0;
  WorkItem it;
  while (next_item(a, g, queue, probes, it, true)) {
    if (it.i1 <= it.i0) continue;
    const StarDesc d = a.stars[it.star];
    // Gap points that matter for this item: a prefix of the star's list.
    const int ng = it.n_gaps >= 0 ? it.n_gaps : d.n_gaps;
    if ((ng > kGapLanes) != DFORM) continue;  // the other launch's item
    // Long stars take the large shape for every frequency; the others only for
    // frequencies with more fine bins than the common shape holds.
    const bool long_star = d.n > a.c.big_points;
    if (!BIG && long_star) continue;
    const StarRt rt = a.rt[it.star];
    // Equal weights: CW[n] is the common weight times the number of weighted points
    // before n, so G_W accumulates those counts in 32 bits (telescoped differences
    // are exact modulo 2^32, every count is below 2^31) and H_W is rebuilt from them.
    if constexpr (!PACKED) {
      if ((rt.w_unit != 0) != CNT) continue;  // the other launch's star
    }
    constexpr bool cnt = CNT;
    const CountDiv inv_unit = cnt ? count_div(rt.w_unit) : CountDiv{0u, 0u};
    const double w_unit = PACKED ? packed_w_unit(rt) : 0.0;  // packed: 1 / quantised total weight
    const int64_t n = d.n;
    const double* __restrict__ dt = a.dt + d.p_off;
    const int64_t* __restrict__ cw = a.cw + d.p_off;
    const int64_t* __restrict__ cs = a.cs + d.p_off;

    {
      double f_first;
      int32_t nb_first;
      grid_point<EXQ>(d, it.i0, a.c, f_first, nb_first);
      if (nb_first > kNbWide || nb_first < 1) continue;  // rejected by the plan
    }

    // Points: wave w owns a contiguous block of 64 * run points per chunk; in step
    // u lane l holds point block + 64 u + l (u even) or block + 64 u + 63 - l (u
    // odd).  A point's predecessor is then the neighbouring lane of the same step,
    // except for the first point of a step, whose predecessor (the last point of
    // the previous step) sits in the same lane one step earlier: one DPP lane
    // shift per step, with that lane keeping the previous step's value.  Loads
    // stay coalesced and the boundaries of one step fall on consecutive bins.
    // The difference form keeps fewer points in registers (its fold holds more
    // values per boundary).
    constexpr int UM = DFORM ? 4 : W::um;
    static_assert(UM % kUGroup == 0, "the fold takes whole groups of steps");
    const int nchunks = static_cast<int>((n + static_cast<int64_t>(T) * UM - 1) / (static_cast<int64_t>(T) * UM));
    const int run = static_cast<int>((n + static_cast<int64_t>(T) * nchunks - 1) / (static_cast<int64_t>(T) * nchunks));
    const int64_t chunk_pts = static_cast<int64_t>(run) * T;
    const double dt_last = dt[n - 1];
    // Few gap points: keep their values in LDS for the whole item (read after the
    // first group's set-up barrier).
    if (!DFORM && tid < ng) {
      const int32_t q = a.gaps[d.g_off + tid];
      g->gdt0[tid] = dt[q - 1];
      g->gdt1[tid] = dt[q];
      g->gcw[tid] = cnt ? static_cast<long long>(count_of(cw[q], inv_unit)) : cw[q];
      g->gcs[tid] = PACKED ? 0 : cs[q];
    }

    for (int g0 = it.i0, F = 0; g0 < it.i1; g0 += F) {
      // Slot geometry of this group: the fine-bin count falls with frequency, so
      // the group's first frequency has the most bins (nb_cap); the stride holds
      // nb_cap bins plus room to replicate the first m_max bins after the last,
      // so windows that wrap past bin nb-1 read contiguously.  Recomputing it per
      // group lets long ranges take more frequencies per group as nb shrinks.
      double f_g;
      int32_t nb_cap;
      grid_point<EXQ>(d, g0, a.c, f_g, nb_cap);
      if (nb_cap > W::nb_hi) {  // searched by the large shape or k_search_wide
        F = 1;
        continue;
      }
      if (BIG && !long_star && nb_cap <= W::nb_lo) break;  // nb falls with frequency: the rest are the common shape's
      // with exact durations the count goes through the device asin, which need not
      // be monotone in its last place: one bin of room for a later frequency's count
      int stride = __builtin_amdgcn_readfirstlane(nb_cap + m_max + (EXQ ? 1 : 0));
      asm volatile("" : "+s"(stride));
      const float inv_stride = 1.0f / static_cast<float>(stride);
      F = min(min(kFMax, W::elems / stride), it.i1 - g0);
      if (tid < F) {
        double f;
        int32_t nb;
        grid_point<EXQ>(d, g0 + tid, a.c, f, nb);
        g->f[tid] = f;
        g->nb[tid] = nb;
        g->blast[tid] = fold_bin_nc(dt_last, f, static_cast<double>(nb));
        g->key[tid] = 0ull;
        g->mj[tid] = ~0u;
      }
      for (int idx = tid; idx < F * stride; idx += T) {
        GW[idx] = 0;
        GS[idx] = 0;
      }
      __syncthreads();
      // Gap points of the star: the telescoping H[b] = G[b+1] - G[b] assumes that
      // a visit to bin b ends where a visit to bin b + 1 begins.  A point whose
      // step from bin bp to bin b skips bins ends the visit to bp instead: its
      // prefix values E belong to the exit of bp, not of b - 1, so H[bp] += E and
      // H[b-1] -= E.  With at most one gap point per lane these corrections are
      // found per frequency while G is converted to H.  Stars with more (the
      // cadence is coarser than the finest bins, so most steps skip bins) fold in
      // difference form instead, which needs no corrections.
      const bool gaps_direct = !DFORM && ng > 0;
      constexpr int form = DFORM ? kDiff : kTelescope;

      // ---- fold: a point whose bin differs from its predecessor's is a boundary
      // and adds its prefix values into G of its bin.  Two frequencies per pass
      // give the scheduler two independent chains per point.
      for (int c = 0; c < nchunks; ++c) {
        const int64_t wbase = static_cast<int64_t>(c) * chunk_pts + static_cast<int64_t>(wave) * 64 * run;
        if (wbase >= n) continue;
        const int64_t wend = min<int64_t>(n, wbase + static_cast<int64_t>(64) * run);
        double dtr[UM];
        std::conditional_t<CNT, uint32_t, long long> cwr[UM];
        long long csr[UM];
        // Points past the block's end repeat its last point: same bin, no boundary.
#pragma unroll
        for (int u = 0; u < UM; ++u) {
          const int64_t q = min<int64_t>(wbase + u * 64 + ((u & 1) ? 63 - lane : lane), wend - 1);
          dtr[u] = dt[q];
          if constexpr (CNT)
            cwr[u] = count_of(cw[q], inv_unit);
          else
            cwr[u] = cw[q];
          csr[u] = PACKED ? 0 : cs[q];
        }
        const double dt_before = dt[wbase > 0 ? wbase - 1 : 0];
        for (int k0 = 0; k0 < F; k0 += 2) {
          if (k0 + 1 < F)
            fold_pass<true, PACKED, UM, W::arr_bytes>(smem, stride, k0, g, dtr, cwr, csr, dt_before, run, form);
          else
            fold_pass<false, PACKED, UM, W::arr_bytes>(smem, stride, k0, g, dtr, cwr, csr, dt_before, run, form);
        }
      }
      __syncthreads();

      // ---- G -> H: H[b] = G[b+1] - G[b] (+ the totals at the last point's bin;
      // G[nb] is G[0]; kDiff: H[b] = G[b] + those totals), one wave per
      // frequency, in place.  A wave converts 64 bins at a time: it reads G[b]
      // and G[b+1] of a chunk before writing the chunk, and the next chunk's first
      // bin is still unconverted then (a wave's LDS accesses run in program order);
      // G[0] is read before chunk 0 is written.  The result goes to FP64 with the
      // first bins replicated after the last (windows wrap past nb - 1).
      for (int k = __builtin_amdgcn_readfirstlane(wave); k < F; k += W::threads / 64) {
        const int32_t nb = __builtin_amdgcn_readfirstlane(g->nb[k]);
        const int32_t bl = g->blast[k];
        const int mrep = min(m_max, nb - 1);
        const uint32_t count_total = cnt ? count_of(rt.cw_total, inv_unit) : 0u;
        long long* gw = GW + k * stride;
        long long* gs = GS + k * stride;
        const long long g0w = gw[0], g0s = PACKED ? 0 : gs[0];
        // Lane l holds gap point l's two corrections at this frequency: +E at bin
        // c0 and -E at bin c1 (-1: the point's step crosses at most one bin).
        int32_t c0 = -1, c1 = -1;
        unsigned long long ew = 0, es = 0;
        if (gaps_direct && lane < ng) {
          const double f = g->f[k];
          const double nbd = static_cast<double>(nb);
          const int32_t bq = fold_bin_nc(g->gdt0[lane], f, nbd);
          const int32_t bu = fold_bin_nc(g->gdt1[lane], f, nbd);
          int32_t steps = bu - bq;
          if (steps < 0) steps += nb;
          if (steps > 1) {
            c0 = bq;
            c1 = bu == 0 ? nb - 1 : bu - 1;
            ew = static_cast<unsigned long long>(g->gcw[lane]);
            es = static_cast<unsigned long long>(g->gcs[lane]);
          }
        }
        for (int b0 = 0; b0 < nb; b0 += 64) {
          const int b = b0 + lane;
          // Corrections that fall in this chunk: found with one ballot per end,
          // broadcast from the lane that holds them (rare: two per gap point).
          unsigned long long aw = 0ull, as = 0ull;
          if (gaps_direct) {
            unsigned long long m0 = __ballot(static_cast<uint32_t>(c0 - b0) < 64u);
            unsigned long long m1 = __ballot(static_cast<uint32_t>(c1 - b0) < 64u);
            while (m0) {
              const int src = __builtin_ctzll(m0);
              m0 &= m0 - 1;
              if (b == __builtin_amdgcn_readlane(c0, src)) {
                aw += readlane_u64(ew, src);
                as += readlane_u64(es, src);
              }
            }
            while (m1) {
              const int src = __builtin_ctzll(m1);
              m1 &= m1 - 1;
              if (b == __builtin_amdgcn_readlane(c1, src)) {
                aw -= readlane_u64(ew, src);
                as -= readlane_u64(es, src);
              }
            }
          }
          if (b < nb) {
            unsigned long long dw, ds;
            if (DFORM) {
              dw = static_cast<unsigned long long>(gw[b]);
              ds = PACKED ? 0ull : static_cast<unsigned long long>(gs[b]);
            } else {
              const long long nw = b + 1 < nb ? gw[b + 1] : g0w;
              const long long ns = PACKED ? 0 : (b + 1 < nb ? gs[b + 1] : g0s);
              dw = static_cast<unsigned long long>(nw) - static_cast<unsigned long long>(gw[b]) + aw;
              ds = PACKED ? 0ull : static_cast<unsigned long long>(ns) - static_cast<unsigned long long>(gs[b]) + as;
            }
            if (b == bl) {
              dw += cnt ? static_cast<unsigned long long>(count_total) : static_cast<unsigned long long>(rt.cw_total);
              ds += static_cast<unsigned long long>(rt.cs_total);
            }
            // counts (low words; the slots' high words stay zero) -> weight prefixes
            if (cnt) dw = static_cast<unsigned long long>(static_cast<uint32_t>(dw)) * static_cast<unsigned long long>(rt.w_unit);
            double vw, vs;
            if (PACKED) {
              unpack(dw, rt.s_scale, w_unit, vw, vs);
            } else {
              vw = static_cast<double>(static_cast<long long>(dw)) * kW62;
              vs = static_cast<double>(static_cast<long long>(ds)) * rt.s_scale;
            }
            double* hw = reinterpret_cast<double*>(gw);
            double* hs = reinterpret_cast<double*>(gs);
            hw[b] = vw;
            hs[b] = vs;
            if (b < mrep) {
              hw[nb + b] = vw;
              hs[nb + b] = vs;
            }
          }
        }
      }
      __syncthreads();
      // ---- scan: slot (k, j) = every duration m of the ladder starting at bin j.
      // A slot keeps its best window with the power s^2 / (r (1 - r)) compared as
      // cross products (no division); the group's best per frequency is then the
      // largest power (an integer maximum on its IEEE bits) and, among slots that
      // reach it, the smallest (m, j).
      unsigned long long skey[W::slot_iter];
      uint32_t smj[W::slot_iter];
#pragma unroll
      for (int r = 0; r < W::slot_iter; ++r) {
        const int idx = tid + r * T;
        int k, j;
        slot_of(idx, stride, inv_stride, k, j);
        skey[r] = 0ull;
        smj[r] = ~0u;
        if (k < F && j < g->nb[k]) {
          const int32_t nb = g->nb[k];
          const int mlim = min(m_max, nb - 1);
          // H_S sits W::elems slots after H_W: one base address for both reads.
          const double* hwk = HW + idx;
          // Durations ascend, so a strict comparison keeps the smallest m of equal
          // powers within the slot.  Branch-free: every step is read (reads past
          // mlim stay inside the LDS allocation and are masked out).
          double bss = -1.0, bd = 1.0;
          int bm = 0;
          double rr = 0.0, ss0 = 0.0;
          // Durations of the ladder that fit this frequency (m <= mlim), as a
          // per-lane value: the compiler then selects instead of branching per
          // duration, and the LDS reads of a slot can be issued early.
          uint32_t live = m_mask & (mlim >= 32 ? 0xffffffffu : ((1u << mlim) - 1u));
          asm volatile("" : "+v"(live));
          auto window = [&](int m, double rv, double sv) {
            const double dd = fma(-rv, rv, rv);  // r (1 - r) > 0  <=>  0 < r < 1
            const double ss = sv * sv;
            const bool in_ladder = (live & (1u << (m - 1))) != 0u;
            const bool beats = ss * bd > bss * dd;
            const bool ok = in_ladder && dd > 0.0 && beats && (!DIP || sv < 0.0);
            bss = ok ? ss : bss;
            bd = ok ? dd : bd;
            bm = ok ? m : bm;
          };
#pragma unroll
          for (int m = 1; m <= 12; ++m) {
            rr += hwk[m - 1];
            ss0 += hwk[W::elems + m - 1];
            window(m, rr, ss0);
          }
          for (int m = 13; m <= mlim; ++m) {
            rr += hwk[m - 1];
            ss0 += hwk[W::elems + m - 1];
            window(m, rr, ss0);
          }
          if (bm != 0) {
            const double p = bss / bd;
            skey[r] = static_cast<unsigned long long>(__double_as_longlong(p)) + 1ull;
            smj[r] = (static_cast<uint32_t>(bm) << 20) | static_cast<uint32_t>(j);
            atomicMax(&g->key[k], skey[r]);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < W::slot_iter; ++r) {
        if (skey[r] != 0ull) {
          int k, j;
          slot_of(tid + r * T, stride, inv_stride, k, j);
          if (skey[r] == g->key[k]) atomicMin(&g->mj[k], smj[r]);
        }
      }
      __syncthreads();
      if (tid < F) {
        const int k = tid;
        const int64_t fi = d.f_off + g0 + k;
        bls_best bb;
        bb.m = 0;
        bb.j = -1;
        bb.r = 0.0;
        bb.s = 0.0;
        double sr = 0.0;
        const uint32_t mj = g->mj[k];
        if (g->key[k] != 0ull && mj != ~0u) {
          const int m = static_cast<int>(mj >> 20), j = static_cast<int>(mj & 0xFFFFFu);
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
}

// Frequencies with more fine bins than a large-shape group holds (kNbLimitBig);
// k_search skips them.  Same work list; nb falls with frequency, so the wide frequencies of
// an item are a prefix of its range.
template <bool PACKED, bool EXQ>
__global__ void __launch_bounds__(kSearchThreads, 4) k_search_wide(SearchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  GroupLds* g = reinterpret_cast<GroupLds*>(smem + Win<true>::bytes);
  const int T = kSearchThreads;
  int queue = static_cast<int>(blockIdx.x % kXcds);  // used by thread 0 only
  int probes = 0;
  WorkItem it;
  while (next_item(a, g, queue, probes, it)) {
    if (it.i1 <= it.i0) continue;
    const StarDesc d = a.stars[it.star];
    double f0;
    int32_t nb0;
    grid_point<EXQ>(d, it.i0, a.c, f0, nb0);
    if (nb0 <= kNbLimitBig || nb0 > kNbWide) continue;
    const StarRt rt = a.rt[it.star];
    const double w_unit = PACKED ? packed_w_unit(rt) : 0.0;
    const int64_t n = d.n;
    const double* __restrict__ dt = a.dt + d.p_off;
    const int64_t* __restrict__ cw = a.cw + d.p_off;
    const int64_t* __restrict__ cs = a.cs + d.p_off;
    const int nchunks = static_cast<int>((n + static_cast<int64_t>(T) * kUMax - 1) / (static_cast<int64_t>(T) * kUMax));
    const int run = static_cast<int>((n + static_cast<int64_t>(T) * nchunks - 1) / (static_cast<int64_t>(T) * nchunks));
    const int64_t chunk_pts = static_cast<int64_t>(run) * T;
    const double dt_last = dt[n - 1];
    for (int fi = it.i0; fi < it.i1; ++fi) {
      double f;
      int32_t nb;
      grid_point<EXQ>(d, fi, a.c, f, nb);
      if (nb <= kNbLimitBig) break;
      wide_frequency<PACKED, EXQ>(smem, g, a, d, rt, fi, w_unit, dt, cw, cs, nchunks, run, chunk_pts, dt_last);
    }
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
  BLS_HIP_TRY(hipMemcpyAsync(base + plan->layout.stars, plan->stars.data(),
                             sizeof(StarDesc) * plan->stars.size(), hipMemcpyHostToDevice, st));
  if (!plan->items.empty())
    BLS_HIP_TRY(hipMemcpyAsync(base + plan->layout.items, plan->items.data(),
                               sizeof(WorkItem) * plan->items.size(), hipMemcpyHostToDevice, st));
  if (!plan->gaps.empty()) {
    BLS_HIP_TRY(hipMemcpyAsync(base + plan->layout.gaps, plan->gaps.data(),
                               sizeof(int32_t) * plan->gaps.size(), hipMemcpyHostToDevice, st));
    BLS_HIP_TRY(hipMemcpyAsync(base + plan->layout.gap_steps, plan->gap_steps.data(),
                               sizeof(double) * plan->gap_steps.size(), hipMemcpyHostToDevice, st));
  }
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
  unsigned int* counters = reinterpret_cast<unsigned int*>(base + L.counter);
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, st, counters);
  BLS_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_prepare, dim3(plan->n_stars), dim3(kThreads), 0, st,
                     reinterpret_cast<const StarDesc*>(base + L.stars), reinterpret_cast<StarRt*>(base + L.rt),
                     d_t, d_y, d_w, reinterpret_cast<double*>(base + L.dt), reinterpret_cast<int64_t*>(base + L.cw),
                     reinterpret_cast<int64_t*>(base + L.cs), plan->consts.packed, counters + kFlagsIndex);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

template <bool PACKED, bool DFORM, bool BIG, bool EXQ, bool CNT>
static void launch_k(bool dip, const dim3& gd, const dim3& bd, size_t lds, hipStream_t st, const SearchArgs& a) {
  if (dip) hipLaunchKernelGGL((k_search<PACKED, DFORM, true, BIG, EXQ, CNT>), gd, bd, lds, st, a);
  else hipLaunchKernelGGL((k_search<PACKED, DFORM, false, BIG, EXQ, CNT>), gd, bd, lds, st, a);
}

// Accumulation forms of one launch: telescoping with weight prefixes, difference
// form, and both with counts of weighted points (precision 0, equal weights).
enum SearchForm { kFormPrefix = 0, kFormDiff = 1, kFormCount = 2, kFormDiffCount = 3 };

template <bool BIG, bool EXQ>
static void launch_search_x(bool packed, int form, bool dip, const dim3& gd, const dim3& bd, size_t lds,
                            hipStream_t st, const SearchArgs& a) {
  if (packed) {
    if (form == kFormDiff) launch_k<true, true, BIG, EXQ, false>(dip, gd, bd, lds, st, a);
    else launch_k<true, false, BIG, EXQ, false>(dip, gd, bd, lds, st, a);
  } else if (form == kFormDiff) {
    launch_k<false, true, BIG, EXQ, false>(dip, gd, bd, lds, st, a);
  } else if (form == kFormDiffCount) {
    launch_k<false, true, BIG, EXQ, true>(dip, gd, bd, lds, st, a);
  } else if (form == kFormCount) {
    launch_k<false, false, BIG, EXQ, true>(dip, gd, bd, lds, st, a);
  } else {
    launch_k<false, false, BIG, EXQ, false>(dip, gd, bd, lds, st, a);
  }
}

// The instantiations of k_search for one workgroup shape (packed sums, difference
// form, dips only, exact durations), as a persistent grid of `groups` workgroups
// per CU.
template <bool BIG>
static void launch_search(bool packed, int form, bool dip, bool exq, int64_t n_items, int cus, hipStream_t st,
                          const SearchArgs& a) {
  const int64_t grid = std::min<int64_t>(n_items, Win<BIG>::groups * static_cast<int64_t>(cus));
  const dim3 gd(static_cast<unsigned>(grid)), bd(Win<BIG>::threads);
  const size_t lds = search_lds<BIG>();
  if (exq)
    launch_search_x<BIG, true>(packed, form, dip, gd, bd, lds, st, a);
  else
    launch_search_x<BIG, false>(packed, form, dip, gd, bd, lds, st, a);
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
  a.gap_steps = reinterpret_cast<const double*>(base + L.gap_steps);
  a.windows = d_windows;
  a.sr = d_sr;
  a.best = d_best;
  a.next = reinterpret_cast<unsigned int*>(base + L.counter);
  a.c = plan->consts;
  const int64_t n_items = d_windows ? n_windows : static_cast<int64_t>(plan->items.size());
  if (n_items == 0) return BLS_OK;
  if (plan->consts.rebin) return rebin_search(plan, base, d_windows, n_items, d_sr, d_best, st);
  a.n_items = static_cast<int32_t>(n_items);
  a.n_stars = plan->n_stars;
  int dev = 0, cus = 0;
  BLS_HIP_TRY(hipGetDevice(&dev));
  BLS_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (cus < 1) return BLS_E_HIP;
  // Persistent launches, each preceded by a reset of the work counters: the common
  // shape, then the large shape for frequencies with more fine bins, and the
  // frequencies beyond one LDS pass.  Per shape: stars of equal weights with counts
  // (precision 0; a launch ends at once when the batch has none, and likewise the
  // next one when every star has equal weights), the other stars, and (when the
  // batch needs it) stars whose steps mostly skip fine bins in difference form, again
  // with counts and then with weight prefixes.
  // Each launch skips the others' work.
  const bool packed = plan->consts.packed != 0, dip = a.c.dip_only != 0, exq = a.c.exact_q != 0;
  const bool dform = d_windows ? plan->has_dform_star : plan->has_dform;
  int forms[4], n_forms = 0;
  if (!packed) forms[n_forms++] = kFormCount;
  forms[n_forms++] = kFormPrefix;
  if (dform && !packed) forms[n_forms++] = kFormDiffCount;
  if (dform) forms[n_forms++] = kFormDiff;
  for (int big = 0; big < (plan->has_big ? 2 : 1); ++big) {
    for (int fi = 0; fi < n_forms; ++fi) {
      hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, a.next);  // 8 counters
      BLS_HIP_TRY(hipGetLastError());
      if (big)
        launch_search<true>(packed, forms[fi], dip, exq, n_items, cus, st, a);
      else
        launch_search<false>(packed, forms[fi], dip, exq, n_items, cus, st, a);
      BLS_HIP_TRY(hipGetLastError());
    }
  }
  if (plan->has_wide) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, a.next);
    BLS_HIP_TRY(hipGetLastError());
    const int64_t grid = std::min<int64_t>(n_items, kSearchGroupsPerCuBig * static_cast<int64_t>(cus));
    const dim3 gd(static_cast<unsigned>(grid)), bd(kSearchThreads);
    if (packed) {
      if (exq) hipLaunchKernelGGL((k_search_wide<true, true>), gd, bd, search_lds<true>(), st, a);
      else hipLaunchKernelGGL((k_search_wide<true, false>), gd, bd, search_lds<true>(), st, a);
    } else {
      if (exq) hipLaunchKernelGGL((k_search_wide<false, true>), gd, bd, search_lds<true>(), st, a);
      else hipLaunchKernelGGL((k_search_wide<false, false>), gd, bd, search_lds<true>(), st, a);
    }
  }
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}
