// plan.hpp — host-side plan and device descriptor layouts of the MI355X BLS library.
//
// The plan turns the paper's problem statement (times, fluxes, weights, stellar
// density and period bounds; QLP Data Release Notes 003 Sec. 2.1) into per-star
// grid descriptors and a cost-ordered list of work items.  The frequency grid is
// never materialised: the device recomputes f_i = (umin + i A)^3 and the fine-bin
// count nb_i = ceil(noverlap / (kq (umin + i A)^2)) from four numbers per star,
// with the same IEEE operations as the host (no FMA contraction anywhere).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "mi355bls.h"

namespace mi355bls {

// Compiled limits.
constexpr int kThreads = 1024;        // threads per preparation / resampling workgroup
constexpr int kSnrThreads = 256;      // threads per S/N workgroup for short spectra
constexpr int64_t kSnrSmallMaxFreqs = 32768;  // longest spectrum of such a batch
constexpr int kSearchThreads = 512;   // threads per search workgroup
// Two shapes of the one-pass search workgroup.  The common one: 512 threads, 48 KB
// of per-frequency accumulators, 8 register-resident points per thread and at most
// 80 registers per lane, three workgroups per CU (6 waves per SIMD).  The large one,
// for frequencies with more fine bins: 768 threads, 72 KB, 8 points, 80 registers,
// two per CU (also 6 waves per SIMD).
constexpr int kGBytes = 48 * 1024;
constexpr int kUMaxSmall = 8;
constexpr int kSearchGroupsPerCu = 3;
constexpr int kGBytesBig = 72 * 1024;
constexpr int kUMax = 12;             // register-resident points per thread of k_search_wide
constexpr int kSearchGroupsPerCuBig = 2;
constexpr int kSearchThreadsBig = 768;   // large-shape workgroup (12 waves; 6 per SIMD at two per CU)
constexpr int kUMaxBig = 8;              // its register-resident points per thread
constexpr int kNbLimit = kGBytes / 16 - 32;        // largest fine-bin count of the common
                                                    // shape (16 B per bin, plus the
                                                    // replicated wrap bins): 3040
constexpr int kNbLimitBig = kGBytesBig / 16 - 32;  // of the large shape: 4576
constexpr int64_t kBigPoints = 100000;  // default: stars with more points take the large shape
                                       // for all their frequencies (fewer point
                                       // re-reads per frequency)
constexpr int kNbWide = (1 << 20) - 1;       // largest fine-bin count (window start bins
                                              // are 20-bit fields); beyond kNbLimitBig a
                                              // frequency is searched in passes over bin ranges
constexpr int kFMax = 64;             // most frequencies processed together
constexpr int kGapLanes = 64;         // stars with more gap points fold in difference form
constexpr int kMCap = 32;             // longest duration (in fine bins)
constexpr int64_t kMaxPoints = int64_t(1) << 30;
constexpr int kMaxSturges = 64;
constexpr int kRebinMax = 32;         // most durations of the per-duration rebinning ladder
constexpr int kWindowSlack = 16;      // extra tiles per star in a tiled window list (one
                                      // per disjoint window: a window adds at most one
                                      // partial tile)

// Per-star descriptor (device copy is read-only).
struct StarDesc {
  int64_t p_off;    // first point in the packed arrays
  int64_t n;        // points
  int64_t f_off;    // first frequency in the packed per-frequency outputs
  int64_t nf;       // frequencies
  double t0;        // first time with w > 0 (phase origin)
  double umin;      // grid start in u = f^(1/3)
  double A;         // grid step in u
  double kq;        // qmin_fac * krho: q_lo(f) = kq f^(2/3)
  int32_t nb0;      // fine bins at i = 0 (the largest of the star)
  int32_t sturges;  // Sturges bin count of the S/N trend
  int32_t n_gaps;   // points whose time step can cross more than one fine bin
  int32_t per_tile; // frequencies per work item of this star
  int64_t g_off;    // first entry of this star in the gap list
  double T, pmin, pmax, krho;  // descriptive (host queries)
  int64_t tile_off; // first slot of this star in a tiled window list (see pp_propose)
};
static_assert(sizeof(StarDesc) == 128, "StarDesc layout");

// Per-star values written by the preparation kernel.
struct StarRt {
  int64_t cw_total;  // sum of fixed-point weights (units of 2^-62); packed: the packed total
  int64_t cs_total;  // sum of fixed-point weighted residuals (units of s_scale); packed: 0
  double s_scale;    // 2^-e: value of one unit of the residual fixed point
  int64_t w_unit;    // precision 0: the common fixed-point weight when every point of
                     // nonzero weight has the same one (then CW[n] = w_unit times the
                     // number of such points before n), else 0; packed: 0
};

// Packed fixed point (precision 1): w~ in units of 2^-27 in the high 28 bits and
// w~ x in units of s_scale in the low 36 bits (two's complement) of one 64-bit
// integer, summed modulo 2^64.  A bin's total holds at most 2^27 + n/2 < 2^28
// weight units and |residual| < 2^35 units, so both fields decode exactly; bin
// weights are then divided by the star's quantised total.
constexpr int kPackShift = 36;
constexpr int kPackWBits = 27;

// A work item: frequencies [i0, i1) of one star.
struct WorkItem {
  int32_t star, i0, i1;
  int32_t n_gaps;  // leading entries of the star's gap list that matter in [i0, i1)
};

// Scalars shared by every kernel of a plan.
struct Consts {
  int32_t noverlap;
  int32_t dip_only;
  int32_t mad_of_raw;
  int32_t m_max;       // longest duration in bins
  uint32_t m_mask;     // bit (m-1) set for every duration m of the ladder
  int32_t packed;      // 1: weights and residuals share one int64 per point (precision 1)
  int64_t big_points;  // stars with more points take the large shape for every frequency
  int32_t exact_q;     // 1: exact circular duration (asin) for the shortest searched one
  int32_t rebin;       // 1: one bin set per duration of the continuous ladder
  int32_t n_rebin;     // durations of that ladder
  int32_t pad_;
  double qmin_fac;
  double rebin_g[kRebinMax];  // q_k / q_lo of the ladder (host libm exp, as the oracle's)
};

constexpr double kPi = 3.14159265358979323846;

// Shortest searched duty cycle at grid point uu = u^2 (Sec. 2.1): qmin_fac times
// the central circular-orbit duty cycle, small-angle (kq uu) or, with exact
// durations, qmin_fac asin(R*/a) / pi with R*/a = pi krho uu (clamped to 1), never
// taken below the small-angle value (so it never needs more bins).  The same IEEE
// operations on host and device; asin is the host's libm or the device's math
// library (the two can differ in the last place).
__host__ __device__ inline double qlo_at(const StarDesc& d, const Consts& c, double uu) {
  const double qs = d.kq * uu;
  if (!c.exact_q) return qs;
  double x = kPi * (d.krho * uu);
  if (x > 1.0) x = 1.0;
  const double qe = c.qmin_fac * (asin(x) / kPi);
  return qe > qs ? qe : qs;
}

// Fine bins at grid point uu: the fewest bins of width at most q_lo / noverlap.
__host__ __device__ inline int32_t fine_bins(const StarDesc& d, const Consts& c, double uu) {
  return static_cast<int32_t>(ceil(static_cast<double>(c.noverlap) / qlo_at(d, c, uu)));
}

// Bins of the k-th set of the per-duration rebinning: ceil(noverlap / (q_lo g_k)).
__host__ __device__ inline int32_t rebin_bins(double qlo, double g, int32_t noverlap) {
  return static_cast<int32_t>(ceil(static_cast<double>(noverlap) / (qlo * g)));
}

struct Layout {  // byte offsets inside the device workspace
  int64_t stars, rt, items, gaps, gap_steps, dt, cw, cs, rho, counter, total;
};

// Records the HIP error code of a failed HIP call (per thread) and returns
// BLS_E_HIP; bls_last_hip_error() reads it back.
bls_status hip_failed(int hip_error_code);

}  // namespace mi355bls

struct bls_plan;

namespace mi355bls {

// The per-duration rebinning search (rebin = 1) over the plan's work items or a
// caller's (star, i0, i1) list; `base` is the uploaded and prepared workspace.
bls_status rebin_search(const bls_plan* plan, const char* base, const int64_t* d_windows, int64_t n_items,
                        double* d_sr, bls_best* d_best, hipStream_t stream);

}  // namespace mi355bls

// Return from an entry point with BLS_E_HIP (recording the code) if a HIP call fails.
#define BLS_HIP_TRY(call)                                                          \
  do {                                                                             \
    const int bls_hip_e_ = static_cast<int>(call);                                 \
    if (bls_hip_e_ != 0) return mi355bls::hip_failed(bls_hip_e_);                 \
  } while (0)

struct bls_plan {
  bls_params params;
  int32_t n_stars = 0;
  int64_t n_points = 0;
  int64_t n_freq = 0;
  std::vector<mi355bls::StarDesc> stars;
  std::vector<mi355bls::WorkItem> items;
  std::vector<int32_t> gaps;  // per star (CSR by StarDesc::g_off): point indices n >= 1,
                              // largest time step first
  std::vector<double> gap_steps;  // the time step of each entry of gaps
  std::vector<int64_t> freq_offsets;
  int64_t tile_capacity = 0;  // slots of a tiled window list: per star, its tiles + 16
  bool has_big = false;        // some frequency needs the large workgroup shape
  bool has_wide = false;       // some frequency has more fine bins than one LDS pass holds
  bool has_dform = false;      // some work item has more than kGapLanes gap points
  bool has_dform_star = false; // some star has (caller windows use the star's count)
  std::vector<int32_t> durations;
  mi355bls::Consts consts{};
  mi355bls::Layout layout{};
  void* uploaded_to = nullptr;  // workspace the descriptors were copied into
};
