// plan.cpp — host plan of the MI355X BLS library: validation, period bounds, the
// Keplerian frequency grid, the duration ladder and the work schedule.
//
// References are to QLP Data Release Notes 003 (Kunimoto et al. 2023):
//   Sec. 2.1  stellar density (solar if missing), durations 0.5-2.0 x the central
//             circular-orbit duration, samples_per_peak / dlogq / noverlap
//             (footnote), minimum period at a = 2 R* (3 R*), maximum period from the
//             longest continuous stretch (half without gaps longer than a sector).
//   Sec. 2.2  S/N trend with Sturges' rule (footnote).
// The constants' evaluation order is fixed (documented with the kernels' grid
// formula) so the host and the device produce the same bits for f_i and nb_i.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>
#include <utility>

#include "plan.hpp"

using namespace mi355bls;

namespace {

constexpr double kGmSun = 1.3271244e20;  // m^3 s^-2 (IAU 2015 nominal)
constexpr double kRSun = 6.957e8;        // m (IAU 2015 nominal)
constexpr double kDay = 86400.0;         // s

// Circular-orbit duty cycle coefficient of the Sun: the central transit of a
// circular orbit lasts (P/pi)(R/a); with Kepler's third law, in days,
// q_circ(f) = K_sun rho^(-1/3) f^(2/3), K_sun = cbrt(4 pi^2 R^3/GM) / (pi cbrt(86400^2)).
// volatile: evaluated with the C library at run time, never folded at compile time.
double k_sun() {
  volatile double rs = kRSun, gm = kGmSun, day = kDay, pi = kPi;
  const double r3 = (rs * rs) * rs;
  const double num = std::cbrt((((4.0 * pi) * pi) * r3) / gm);
  return num / (pi * std::cbrt(day * day));
}

double density(double rho) { return (std::isnan(rho) || rho <= 0.0) ? 1.0 : rho; }

// Orbital period (days) at which a = a_min R* for density rho (solar units).
double period_at_a(double a_min, double rho) {
  volatile double rs = kRSun;
  const double r3 = (rs * rs) * rs;
  const double a3 = (a_min * a_min) * a_min;
  return ((2.0 * kPi) * std::sqrt((a3 * r3) / (kGmSun * density(rho)))) / kDay;
}

// Small-angle fine-bin count: an upper bound of every mode's count (the exact
// duration is never shorter), used for the launch decisions.
int32_t nbins_small(const StarDesc& d, int64_t i, int32_t noverlap) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  const double uu = u * u;
  return static_cast<int32_t>(std::ceil(static_cast<double>(noverlap) / (d.kq * uu)));
}

double freq_at(const StarDesc& d, int64_t i) {
  const double u = d.umin + static_cast<double>(i) * d.A;
  return (u * u) * u;
}

// Smallest time step that can advance the phase by 0.99 fine bins at frequencies
// up to f (f nb <= noverlap f^(1/3) / kq + f, increasing in f).
double gap_threshold(const StarDesc& d, double f, int32_t noverlap) {
  const double fnb = static_cast<double>(noverlap) * std::cbrt(f) / d.kq + f;
  return 0.99 / fnb;
}

bool valid_params(const bls_params& p) {
  return p.spp > 0.0 && p.qmin_fac > 0.0 && p.qmax_fac >= p.qmin_fac && p.dlogq > 0.0 &&
         p.noverlap >= 1 && p.a_min_rstar > 0.0 && p.sector_days > 0.0 &&
         (p.precision == 0 || p.precision == 1) && p.tile_cells >= 0 && p.big_points >= 0 &&
         p.item_freqs >= 0 && p.item_freqs <= (1 << 20) && (p.exact_duration == 0 || p.exact_duration == 1) &&
         (p.rebin == 0 || p.rebin == 1) && std::isfinite(p.spp) &&
         std::isfinite(p.qmin_fac) && std::isfinite(p.qmax_fac) && std::isfinite(p.dlogq);
}

// Duration ladder (dlogq, Sec. 2.1 footnote): m_k = round(noverlap e^(k dlogq)) for
// k = 0..ceil(ln(qmax/qmin)/dlogq), capped at round(noverlap qmax/qmin), sorted, unique.
std::vector<int32_t> duration_ladder(const bls_params& p) {
  const int32_t kmax = static_cast<int32_t>(std::ceil(std::log(p.qmax_fac / p.qmin_fac) / p.dlogq));
  const int32_t mcap =
      static_cast<int32_t>(std::floor(static_cast<double>(p.noverlap) * (p.qmax_fac / p.qmin_fac) + 0.5));
  std::vector<int32_t> m;
  for (int32_t k = 0; k <= kmax; ++k) {
    int32_t v = static_cast<int32_t>(
        std::floor(static_cast<double>(p.noverlap) * std::exp(static_cast<double>(k) * p.dlogq) + 0.5));
    v = std::max(1, std::min(v, mcap));
    m.push_back(v);
  }
  std::sort(m.begin(), m.end());
  m.erase(std::unique(m.begin(), m.end()), m.end());
  return m;
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

}  // namespace

extern "C" bls_status bls_default_params(bls_params* p) {
  if (!p) return BLS_E_ARG;
  std::memset(p, 0, sizeof(*p));
  p->spp = 2.0;
  p->qmin_fac = 0.5;
  p->qmax_fac = 2.0;
  p->dlogq = 0.1;
  p->noverlap = 3;
  p->dip_only = 0;
  p->mad_of_raw = 0;
  p->precision = 0;
  p->a_min_rstar = 2.0;
  p->sector_days = 27.4;
  return BLS_OK;
}

extern "C" bls_status bls_plan_create(const bls_params* p, int32_t n_stars, const bls_star* stars,
                                      const double* t, const double* y, const double* w,
                                      bls_plan** out, int32_t* bad_star) {
  if (out) *out = nullptr;
  if (bad_star) *bad_star = -1;
  if (!p || !stars || !t || !out || n_stars < 1) return BLS_E_ARG;
  if (!valid_params(*p)) return BLS_E_ARG;
  const std::vector<int32_t> ladder = duration_ladder(*p);
  if (ladder.empty() || ladder.back() > kMCap) return BLS_E_UNSUPPORTED;
  // per-duration rebinning: exact int64 sums only, at most kRebinMax durations
  const int32_t n_rebin = static_cast<int32_t>(std::ceil(std::log(p->qmax_fac / p->qmin_fac) / p->dlogq)) + 1;
  if (p->rebin && (p->precision != 0 || n_rebin > kRebinMax || n_rebin < 1 || p->noverlap > kMCap))
    return BLS_E_UNSUPPORTED;

  bls_plan* plan = new (std::nothrow) bls_plan();
  if (!plan) return BLS_E_NOMEM;
  plan->params = *p;
  plan->n_stars = n_stars;
  plan->durations = ladder;
  plan->consts.noverlap = p->noverlap;
  plan->consts.dip_only = p->dip_only ? 1 : 0;
  plan->consts.mad_of_raw = p->mad_of_raw ? 1 : 0;
  plan->consts.m_max = ladder.back();
  uint32_t mask = 0;
  for (int32_t m : ladder) mask |= 1u << (m - 1);
  plan->consts.m_mask = mask;
  plan->consts.packed = p->precision == 1 ? 1 : 0;
  plan->consts.big_points = p->big_points > 0 ? p->big_points : kBigPoints;
  plan->consts.exact_q = p->exact_duration ? 1 : 0;
  plan->consts.rebin = p->rebin ? 1 : 0;
  plan->consts.qmin_fac = p->qmin_fac;
  if (p->rebin) {
    // q_k / q_lo = min(e^(k dlogq), qmax/qmin), k = 0..n_rebin-1 (host libm exp)
    const double gcap = p->qmax_fac / p->qmin_fac;
    plan->consts.n_rebin = n_rebin;
    for (int32_t k = 0; k < n_rebin; ++k) {
      const double e = std::exp(static_cast<double>(k) * p->dlogq);
      plan->consts.rebin_g[k] = e < gcap ? e : gcap;
    }
  }
  try {
    plan->stars.resize(n_stars);
    plan->freq_offsets.assign(n_stars + 1, 0);
  } catch (...) {
    delete plan;
    return BLS_E_NOMEM;
  }

  const double ksun = k_sun();
  std::vector<double>& gap_steps = plan->gap_steps;
  // Offsets of the stars' points; the first star with an impossible point count
  // ends the plan there (stars after it are not read).
  int32_t n_valid = n_stars;
  std::vector<int64_t> poff;
  try {
    poff.assign(n_stars + 1, 0);
  } catch (...) {
    delete plan;
    return BLS_E_NOMEM;
  }
  for (int32_t s = 0; s < n_stars; ++s) {
    const int64_t n = stars[s].n_points;
    if (n < 2 || n > kMaxPoints) {
      n_valid = s;
      break;
    }
    poff[s + 1] = poff[s] + n;
  }
  // Per star (independent, on host threads): checks of its points, its period
  // range, grid, fine bins and gap list.  The results are then taken in star
  // order, so the plan and the first failing star reported do not depend on the
  // number of threads.
  struct StarOut {
    bls_status status = BLS_OK;
    bool big = false, wide = false, dform = false;
    std::vector<std::pair<double, int32_t>> gaps;
  };
  std::vector<StarOut> outs;
  try {
    outs.resize(n_valid);
  } catch (...) {
    delete plan;
    return BLS_E_NOMEM;
  }
  auto star_work = [&](int32_t s) -> bls_status {
    const bls_star& st = stars[s];
    StarOut& o = outs[s];
    const int64_t off = poff[s];
    auto fail = [](bls_status code) { return code; };
    const int64_t n = st.n_points;
    const double* ts = t + off;
    const double* ws = w ? w + off : nullptr;
    const double* ys = y ? y + off : nullptr;
    int64_t first = -1, last = -1;
    double wsum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      if (!std::isfinite(ts[i])) return fail(BLS_E_INPUT);
      if (i > 0 && ts[i] < ts[i - 1]) return fail(BLS_E_INPUT);
      const double wi = ws ? ws[i] : 1.0;
      if (!std::isfinite(wi) || wi < 0.0) return fail(BLS_E_INPUT);
      if (ys && !std::isfinite(ys[i])) return fail(BLS_E_INPUT);
      wsum += wi;
      if (wi > 0.0) {
        if (first < 0) first = i;
        last = i;
      }
    }
    if (first < 0 || first == last || !(wsum > 0.0) || !std::isfinite(wsum)) return fail(BLS_E_INPUT);
    StarDesc& d = plan->stars[s];
    d.p_off = off;
    d.n = n;
    d.t0 = ts[first];
    d.T = ts[last] - ts[first];
    if (!(d.T > 0.0)) return fail(BLS_E_INPUT);

    // Maximum period: longest continuous stretch; half of it without any gap
    // longer than one sector (Sec. 2.1).
    double L = 0.0, s_start = ts[first], prev = ts[first];
    bool long_gap = false;
    for (int64_t i = first + 1; i <= last; ++i) {
      const double wi = ws ? ws[i] : 1.0;
      if (!(wi > 0.0)) continue;
      if (ts[i] - prev > p->sector_days) {
        long_gap = true;
        if (prev - s_start > L) L = prev - s_start;
        s_start = ts[i];
      }
      prev = ts[i];
    }
    if (prev - s_start > L) L = prev - s_start;
    double pmax = long_gap ? L : 0.5 * L;
    double pmin = period_at_a(p->a_min_rstar, st.rho_solar);
    if (st.pmin_days > 0.0) pmin = st.pmin_days;
    if (st.pmax_days > 0.0) pmax = st.pmax_days;
    d.pmin = pmin;
    d.pmax = pmax;
    d.krho = ksun / std::cbrt(density(st.rho_solar));
    if (!(pmin < pmax) || !std::isfinite(pmin) || !std::isfinite(pmax)) return fail(BLS_E_EMPTY_GRID);

    // Keplerian grid, uniform in u = f^(1/3): a step shifts the phase at the end of
    // the baseline by 1/spp of the shortest searched duration q_lo = qmin_fac q_circ.
    const double umin = std::cbrt(1.0 / pmax);
    const double umax = std::cbrt(1.0 / pmin);
    d.umin = umin;
    d.A = (p->qmin_fac * d.krho) / ((3.0 * p->spp) * d.T);
    d.kq = p->qmin_fac * d.krho;
    const double steps = std::floor((umax - umin) / d.A);
    if (!(steps >= 0.0) || steps > 2.0e9) return fail(steps >= 0.0 ? BLS_E_UNSUPPORTED : BLS_E_EMPTY_GRID);
    d.nf = static_cast<int64_t>(steps) + 1;
    const int32_t nb_up = nbins_small(d, 0, p->noverlap);
    {
      const double u0 = d.umin;
      d.nb0 = fine_bins(d, plan->consts, u0 * u0);
    }
    if (nb_up > kNbWide || d.nb0 < 1) return fail(BLS_E_UNSUPPORTED);
    o.big = nb_up > kNbLimit || d.n > plan->consts.big_points;
    o.wide = nb_up > kNbLimitBig;
    const int32_t sturges =
        static_cast<int32_t>(std::floor(1.0 + 3.322 * std::log10(static_cast<double>(d.nf)) + 0.5));
    d.sturges = std::max(1, std::min(sturges, kMaxSturges));
    // Gap list: points whose time step may advance the phase by a whole fine bin or
    // more at some grid frequency.  The phase advance of a step dt is dt f nb, and
    // f nb <= noverlap f^(1/3) / kq + f, which grows with f; steps below 0.99 / that
    // bound at the top of the grid move at most one bin everywhere.  The list is
    // ordered by step, largest first, so that the points that can skip bins below
    // any lower frequency form a prefix of it.
    {
      const double fmax = freq_at(d, d.nf - 1);
      const double thr = gap_threshold(d, fmax, p->noverlap);
      std::vector<std::pair<double, int32_t>>& list = o.gaps;
      for (int64_t i = 1; i < n; ++i)
        if (ts[i] - ts[i - 1] >= thr) list.emplace_back(ts[i] - ts[i - 1], static_cast<int32_t>(i));
      std::stable_sort(list.begin(), list.end(),
                       [](const std::pair<double, int32_t>& a, const std::pair<double, int32_t>& b) {
                         return a.first > b.first;
                       });
      if (static_cast<int64_t>(list.size()) > 0x7fffffff) return fail(BLS_E_UNSUPPORTED);
      d.n_gaps = static_cast<int32_t>(list.size());
      o.dform = d.n_gaps > kGapLanes;
    }
    return BLS_OK;
  };
  {
    const int64_t total = poff[n_valid];
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int32_t n_threads = total < (int64_t(1) << 20) ? 1 : static_cast<int32_t>(std::min<unsigned>({hw, 16u,
                                                                    static_cast<unsigned>(std::max(1, n_valid))}));
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
      for (int32_t s; (s = next.fetch_add(1)) < n_valid;) {
        try {
          outs[s].status = star_work(s);
        } catch (...) {
          outs[s].status = BLS_E_NOMEM;
        }
      }
    };
    std::vector<std::thread> pool;
    try {
      for (int32_t k = 1; k < n_threads; ++k) pool.emplace_back(worker);
    } catch (...) {
      // fewer threads: the calling thread and those started share the stars
    }
    worker();
    for (auto& th : pool) th.join();
  }
  for (int32_t s = 0; s < n_stars; ++s) {
    auto fail = [&](bls_status code) {
      if (bad_star) *bad_star = s;
      delete plan;
      return code;
    };
    if (s == n_valid) return fail(stars[s].n_points < 2 ? BLS_E_INPUT : BLS_E_UNSUPPORTED);
    StarOut& o = outs[s];
    if (o.status != BLS_OK) return fail(o.status);
    StarDesc& d = plan->stars[s];
    d.g_off = static_cast<int64_t>(plan->gaps.size());
    try {
      for (const auto& e : o.gaps) {
        plan->gaps.push_back(e.second);
        gap_steps.push_back(e.first);
      }
    } catch (...) {
      return fail(BLS_E_NOMEM);
    }
    std::vector<std::pair<double, int32_t>>().swap(o.gaps);
    if (o.big) plan->has_big = true;
    if (o.wide) plan->has_wide = true;
    if (o.dform) plan->has_dform_star = true;
    d.f_off = plan->n_freq;
    plan->n_freq += d.nf;
    plan->freq_offsets[s + 1] = plan->n_freq;
  }
  plan->n_points = poff[n_stars];

  // Work items: frequency tiles of each star sized to a similar number of cells
  // (points x frequencies), ordered by cost, largest first, so that the tail of
  // the launch is made of small items.
  const int64_t target_cells = p->tile_cells > 0 ? p->tile_cells : int64_t(6) << 20;
  try {
    for (int32_t s = 0; s < n_stars; ++s) {
      const StarDesc& d = plan->stars[s];
      int64_t per = std::max<int64_t>(32, target_cells / std::max<int64_t>(1, d.n));
      // the default also caps an item at 128 frequencies: short stars then spread
      // over more items, and the groups working on one XCD share fewer stars' points
      per = std::min<int64_t>(per, p->item_freqs > 0 ? p->item_freqs : (p->tile_cells > 0 ? 4096 : 128));
      plan->stars[s].per_tile = static_cast<int32_t>(per);
      plan->stars[s].tile_off = plan->tile_capacity;
      plan->tile_capacity += (d.nf + per - 1) / per + kWindowSlack;
      for (int64_t i0 = 0; i0 < d.nf; i0 += per) {
        const int64_t i1 = std::min<int64_t>(d.nf, i0 + per);
        // gap points that can skip bins somewhere in [i0, i1): those whose step
        // reaches the threshold at the item's top frequency
        const double thr = gap_threshold(d, freq_at(d, i1 - 1), p->noverlap);
        const double* st0 = gap_steps.data() + d.g_off;
        const int32_t ng = static_cast<int32_t>(
            std::partition_point(st0, st0 + d.n_gaps, [thr](double v) { return v >= thr; }) - st0);
        if (ng > kGapLanes) plan->has_dform = true;
        plan->items.push_back(WorkItem{s, static_cast<int32_t>(i0), static_cast<int32_t>(i1), ng});
      }
    }
  } catch (...) {
    delete plan;
    return BLS_E_NOMEM;
  }
  std::stable_sort(plan->items.begin(), plan->items.end(), [&](const WorkItem& a, const WorkItem& b) {
    const int64_t ca = plan->stars[a.star].n * (a.i1 - a.i0);
    const int64_t cb = plan->stars[b.star].n * (b.i1 - b.i0);
    return ca > cb;
  });

  Layout& L = plan->layout;
  int64_t pos = 0;
  L.stars = pos;
  pos = align256(pos + int64_t(sizeof(StarDesc)) * n_stars);
  L.rt = pos;
  pos = align256(pos + int64_t(sizeof(StarRt)) * n_stars);
  L.items = pos;
  pos = align256(pos + int64_t(sizeof(WorkItem)) * int64_t(plan->items.size()));
  L.gaps = pos;
  pos = align256(pos + 4 * std::max<int64_t>(1, static_cast<int64_t>(plan->gaps.size())));
  L.gap_steps = pos;
  pos = align256(pos + 8 * std::max<int64_t>(1, static_cast<int64_t>(plan->gaps.size())));
  L.dt = pos;
  pos = align256(pos + 8 * plan->n_points);
  L.cw = pos;
  pos = align256(pos + 8 * plan->n_points);
  L.cs = pos;
  pos = align256(pos + 8 * plan->n_points);
  L.rho = pos;
  pos = align256(pos + 8 * plan->n_freq);
  L.counter = pos;  // 8 work-queue counters, 64 bytes apart, then the batch's flags word
  pos = align256(pos + 9 * 64);
  L.total = pos;
  *out = plan;
  return BLS_OK;
}

extern "C" bls_status bls_plan_query(const bls_plan* plan, int64_t* n_freq_total, int64_t* freq_offsets,
                                     int64_t* workspace_bytes) {
  if (!plan) return BLS_E_ARG;
  if (n_freq_total) *n_freq_total = plan->n_freq;
  if (freq_offsets)
    std::memcpy(freq_offsets, plan->freq_offsets.data(), sizeof(int64_t) * (plan->n_stars + 1));
  if (workspace_bytes) *workspace_bytes = plan->layout.total;
  return BLS_OK;
}

extern "C" bls_status bls_plan_star_info(const bls_plan* plan, int32_t star, double* o) {
  if (!plan || !o || star < 0 || star >= plan->n_stars) return BLS_E_ARG;
  const StarDesc& d = plan->stars[star];
  o[0] = d.t0;
  o[1] = d.T;
  o[2] = d.pmin;
  o[3] = d.pmax;
  o[4] = d.krho;
  o[5] = d.umin;
  o[6] = d.A;
  o[7] = static_cast<double>(d.nf);
  o[8] = static_cast<double>(d.nb0);
  o[9] = static_cast<double>(d.sturges);
  return BLS_OK;
}

extern "C" bls_status bls_plan_frequencies(const bls_plan* plan, int32_t star, double* f, int32_t* nb) {
  if (!plan || star < 0 || star >= plan->n_stars) return BLS_E_ARG;
  const StarDesc& d = plan->stars[star];
  for (int64_t i = 0; i < d.nf; ++i) {
    if (f) f[i] = freq_at(d, i);
    if (nb) {
      const double u = d.umin + static_cast<double>(i) * d.A;
      nb[i] = fine_bins(d, plan->consts, u * u);
    }
  }
  return BLS_OK;
}

extern "C" bls_status bls_plan_durations(const bls_plan* plan, int32_t* m, int32_t cap, int32_t* n) {
  if (!plan || !n) return BLS_E_ARG;
  *n = static_cast<int32_t>(plan->durations.size());
  if (m) {
    if (cap < *n) return BLS_E_ARG;
    std::copy(plan->durations.begin(), plan->durations.end(), m);
  }
  return BLS_OK;
}

extern "C" void bls_plan_destroy(bls_plan* plan) { delete plan; }

extern "C" const char* bls_status_string(bls_status s) {
  switch (s) {
    case BLS_OK: return "ok";
    case BLS_E_ARG: return "invalid argument";
    case BLS_E_INPUT: return "invalid light curve";
    case BLS_E_EMPTY_GRID: return "empty period range";
    case BLS_E_NOMEM: return "host allocation failed";
    case BLS_E_HIP: return "HIP call failed";
    case BLS_E_STATE: return "workspace missing, too small or not uploaded";
    case BLS_E_UNSUPPORTED: return "star exceeds a compiled limit";
    case BLS_E_SCRATCH: return "workspace larger than the static scratch of bls_run_noalloc";
    default: return "unknown status";
  }
}

extern "C" bls_status bls_limits(int64_t* o) {
  if (!o) return BLS_E_ARG;
  o[0] = kNbWide;
  o[1] = kMCap;
  o[2] = kMaxPoints;
  return BLS_OK;
}

namespace mi355bls {
namespace {
thread_local int g_last_hip_error = 0;
}
bls_status hip_failed(int hip_error_code) {
  g_last_hip_error = hip_error_code;
  return BLS_E_HIP;
}
}  // namespace mi355bls

extern "C" int32_t bls_last_hip_error(void) { return mi355bls::g_last_hip_error; }
