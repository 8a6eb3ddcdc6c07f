/*
 * bls_oracle.c — CPU FP64 reference ("oracle") for the Keplerian-grid Box Least
 * Squares search and the spectroscopic S/N step of QLP Data Release Notes 003
 * (Kunimoto et al. 2023, "GPU-based Transit Search").
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that tests, the smoke check and
 * the benchmark's CPU baseline can check the HIP library against a plain, slow,
 * obviously correct implementation.  Nothing in the product path may link, load
 * or call it.  It shares no code, header, constant or helper with the HIP path.
 *
 * Everything is FP64 and every sum runs sequentially in index order.  There is
 * no blocking, fusion or reordering beyond what the definitions below state.
 *
 * What is followed where (the paper is a research note; it fixes the parameters
 * and defers the BLS statistic to Kovacs, Zucker & Mazeh 2002, which it cites):
 *   - SR statistic and the weighted, mean-subtracted flux: Kovacs et al. 2002,
 *     cited in the Introduction; "signal residue" per Sec. 2.2 item 1.
 *   - Keplerian duration window 0.5-2.0 x the central circular-orbit duration,
 *     solar density when missing, samples_per_peak = 2, dlogq = 0.1,
 *     noverlap = 3: Sec. 2.1 and its footnote.
 *   - Minimum period at a = 2 R* (or 3 R*), maximum period from the longest
 *     continuous stretch (half of it without gaps longer than a sector): Sec. 2.1.
 *   - S/N: Sec. 2.2 item 1, Eq. 1 with its two changes (Sturges-rule median-
 *     binned trend, with its footnote; sigma = 1.4826 x MAD).
 * Points the paper leaves open are resolved by the readings listed with each
 * function below; the same readings are collected in the design notes.
 *
 * Parity pins: every function here is pinned by tests under tests/ against
 * closed forms, brute force, invariants and library special cases.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Physical constants: IAU 2015 nominal solar values, 1 d = 86400 s. */
static const double ORC_GM_SUN = 1.3271244e20; /* m^3 s^-2 */
static const double ORC_R_SUN = 6.957e8;       /* m */
static const double ORC_DAY = 86400.0;         /* s */
static const double ORC_PI = 3.14159265358979323846;

typedef struct {
  double spp;         /* samples per peak (2) */
  double qmin_fac;    /* shortest duration / circular duration (0.5) */
  double qmax_fac;    /* longest duration / circular duration (2.0) */
  double dlogq;       /* log spacing of the duration ladder (0.1) */
  int32_t noverlap;   /* shifted bin sets per shortest duration (3) */
  int32_t dip_only;   /* 1: only windows with s < 0 count */
  int32_t mad_of_raw; /* 1: sigma from the MAD of raw SR instead of the residual */
  int32_t exact_duration; /* 1: exact circular duration asin(R_star / a) P / pi, else small-angle */
  double a_min;       /* minimum a/R* (2) */
  double sector_days; /* gap length that splits continuous stretches (27.4) */
  int32_t rebin;      /* 1: one bin set per duration of a continuous ladder */
  int32_t pad_;
} orc_params;

/* Per-star bounds and grid description. */
typedef struct {
  double t0, tlast, T;   /* first/last time with w > 0, baseline */
  double pmin, pmax;     /* searched period range, days */
  double krho;           /* circular duration coefficient: q_circ(f) = krho * f^(2/3) */
  double umin, umax, A;  /* grid in u = f^(1/3): u_i = umin + i*A */
  int64_t nf;            /* number of frequencies */
} orc_bounds_t;

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_INPUT = -2, ORC_E_EMPTY = -3 };

/* ------------------------------------------------------------------------- */
/* Constants of the circular-orbit duration.                                  */
/* The central transit of a circular orbit lasts (P/pi)(R_star/a) (small-angle */
/* form).  With Kepler's third law and rho = rho_star/rho_sun (solar units),   */
/* a/R_star = (GM_sun P^2 rho / (4 pi^2 R_sun^3))^(1/3), so the duty cycle is */
/* q_circ(f) = K_sun rho^(-1/3) f^(2/3) with f in 1/day and                    */
/* K_sun = cbrt(4 pi^2 R_sun^3 / GM_sun) / (pi cbrt(86400^2)).                 */
/* The evaluation order below is a fixed reading so that any implementation   */
/* that follows it reproduces the same bits.                                   */
/* ------------------------------------------------------------------------- */
double orc_k_sun(void) {
  /* volatile: evaluate with the C library at run time (no compile-time folding) */
  volatile double rs = ORC_R_SUN, gm = ORC_GM_SUN, day = ORC_DAY, pi = ORC_PI;
  double r3 = (rs * rs) * rs;
  double num = cbrt((((4.0 * pi) * pi) * r3) / gm);
  return num / (pi * cbrt(day * day));
}

/* Density in solar units; missing (NaN or <= 0) means solar (Sec. 2.1). */
static double orc_rho(double rho) { return (isnan(rho) || rho <= 0.0) ? 1.0 : rho; }

double orc_krho(double rho) { return orc_k_sun() / cbrt(orc_rho(rho)); }

/* Period at which a = a_min R* for density rho (Kepler III), in days (Sec. 2.1). */
double orc_period_at_a(double a_min, double rho) {
  volatile double rs = ORC_R_SUN;
  double r3 = (rs * rs) * rs;
  double a3 = (a_min * a_min) * a_min;
  return ((2.0 * ORC_PI) * sqrt((a3 * r3) / (ORC_GM_SUN * orc_rho(rho)))) / ORC_DAY;
}

/* Circular duty cycle q = duration / period at frequency f (1/day). */
double orc_qcirc(double f, double rho) {
  double u = cbrt(f);
  return orc_krho(rho) * (u * u);
}

/* The same without the small-angle step: a central transit of a circular orbit
 * spans the orbital angle 2 theta with sin theta = R_star / a, so q =
 * asin(R_star / a) / pi, and R_star / a = pi q_small.  R_star / a above 1 (periods
 * below contact, only through an explicit minimum period) is clamped to 1. */
static double orc_exact_from_small(double qs) {
  double x = ORC_PI * qs;
  if (x > 1.0) x = 1.0;
  return asin(x) / ORC_PI;
}

double orc_qcirc_exact(double f, double rho) { return orc_exact_from_small(orc_qcirc(f, rho)); }

/* ------------------------------------------------------------------------- */
/* Period bounds (Sec. 2.1).                                                  */
/* Baseline: t0 = first time with w > 0, tlast = last such time, T = tlast-t0. */
/* Stretches: runs of valid points separated by gaps longer than one sector   */
/* (dt > sector_days).  L = longest (last - first) of a stretch.              */
/* Pmax = L if any such gap exists, else L / 2.  Pmin at a = a_min R*.         */
/* Explicit overrides (> 0) win.                                               */
/* ------------------------------------------------------------------------- */
int orc_bounds(const double* t, const double* w, int64_t n, double rho, const orc_params* p,
               double pmin_override, double pmax_override, orc_bounds_t* out) {
  if (!t || !p || !out || n < 2) return ORC_E_ARG;
  int64_t first = -1, last = -1;
  for (int64_t i = 0; i < n; ++i) {
    double wi = w ? w[i] : 1.0;
    if (wi > 0.0) {
      if (first < 0) first = i;
      last = i;
    }
  }
  if (first < 0 || first == last) return ORC_E_INPUT;
  out->t0 = t[first];
  out->tlast = t[last];
  out->T = out->tlast - out->t0;
  if (!(out->T > 0.0)) return ORC_E_INPUT;

  double L = 0.0, s_start = t[first], prev = t[first];
  int long_gap = 0;
  for (int64_t i = first + 1; i <= last; ++i) {
    double wi = w ? w[i] : 1.0;
    if (!(wi > 0.0)) continue;
    if (t[i] - prev > p->sector_days) {
      long_gap = 1;
      if (prev - s_start > L) L = prev - s_start;
      s_start = t[i];
    }
    prev = t[i];
  }
  if (prev - s_start > L) L = prev - s_start;
  double pmax = long_gap ? L : 0.5 * L;
  double pmin = orc_period_at_a(p->a_min, rho);
  if (pmin_override > 0.0) pmin = pmin_override;
  if (pmax_override > 0.0) pmax = pmax_override;
  out->pmin = pmin;
  out->pmax = pmax;
  out->krho = orc_krho(rho);
  if (!(pmin < pmax)) return ORC_E_EMPTY;

  /* Frequency grid, uniform in u = f^(1/3).  The spacing solves
   * df = q_lo(f) / (spp T) with q_lo = qmin_fac * q_circ: a frequency step
   * shifts the phase at the end of the baseline by 1/spp of the shortest
   * searched duration (samples_per_peak, Sec. 2.1 footnote).  With
   * q_circ = krho f^(2/3) this gives du = qmin_fac krho / (3 spp T). */
  out->umin = cbrt(1.0 / pmax);
  out->umax = cbrt(1.0 / pmin);
  out->A = (p->qmin_fac * out->krho) / ((3.0 * p->spp) * out->T);
  double steps = floor((out->umax - out->umin) / out->A);
  out->nf = (int64_t)steps + 1;
  if (out->nf < 1) return ORC_E_EMPTY;
  return ORC_OK;
}

/* Frequency i of the grid and its fine-bin count.  Fine bins are at most
 * q_lo / noverlap wide, so every searched duration is covered by at least
 * noverlap shifted bin sets (noverlap, Sec. 2.1 footnote). */
static double orc_freq(const orc_bounds_t* b, int64_t i, double* uu_out) {
  double u = b->umin + (double)i * b->A;
  double uu = u * u;
  if (uu_out) *uu_out = uu;
  return uu * u;
}

/* Shortest searched duty cycle at grid point uu = u^2: qmin_fac times the circular
 * one, small-angle (kq uu, kq = qmin_fac krho) or exact; the exact one is never
 * taken below the small-angle one (asin x >= x), so it never needs more bins. */
static double orc_qlo(const orc_bounds_t* b, const orc_params* p, double uu) {
  double kq = p->qmin_fac * b->krho;
  double qs = kq * uu;
  if (!p->exact_duration) return qs;
  double qe = p->qmin_fac * orc_exact_from_small(b->krho * uu);
  return qe > qs ? qe : qs;
}

static int32_t orc_nbins(const orc_bounds_t* b, const orc_params* p, double uu) {
  return (int32_t)ceil((double)p->noverlap / orc_qlo(b, p, uu));
}

int64_t orc_grid(const orc_bounds_t* b, const orc_params* p, double* f, int32_t* nb, int64_t cap) {
  if (b->nf > cap) return ORC_E_ARG;
  for (int64_t i = 0; i < b->nf; ++i) {
    double uu;
    f[i] = orc_freq(b, i, &uu);
    nb[i] = orc_nbins(b, p, uu);
  }
  return b->nf;
}

/* Duration ladder in fine bins: m_k = round(noverlap e^(k dlogq)) for
 * k = 0..ceil(ln(qmax/qmin)/dlogq), capped at round(noverlap qmax/qmin),
 * sorted and de-duplicated (dlogq, Sec. 2.1 footnote; natural log, rounding
 * half up).  At the paper's values this is {3, 4, ..., 12}. */
int32_t orc_durations(const orc_params* p, int32_t* m_out, int32_t cap) {
  int32_t kmax = (int32_t)ceil(log(p->qmax_fac / p->qmin_fac) / p->dlogq);
  int32_t mcap = (int32_t)floor((double)p->noverlap * (p->qmax_fac / p->qmin_fac) + 0.5);
  int32_t cnt = 0;
  for (int32_t k = 0; k <= kmax; ++k) {
    int32_t m = (int32_t)floor((double)p->noverlap * exp((double)k * p->dlogq) + 0.5);
    if (m > mcap) m = mcap;
    if (m < 1) m = 1;
    int32_t pos = 0;
    while (pos < cnt && m_out[pos] < m) ++pos;
    if (pos < cnt && m_out[pos] == m) continue;
    if (cnt >= cap) return ORC_E_ARG;
    for (int32_t q = cnt; q > pos; --q) m_out[q] = m_out[q - 1];
    m_out[pos] = m;
    ++cnt;
  }
  return cnt;
}

/* Continuous duration ladder of the per-duration rebinning (rebin = 1): factors
 * g_k = min(e^(k dlogq), qmax/qmin) for k = 0..ceil(ln(qmax/qmin)/dlogq), so that
 * q_k = g_k q_lo runs from the shortest to the longest searched duration in steps
 * of dlogq in ln q (Sec. 2.1 footnote). */
int32_t orc_rebin_ladder(const orc_params* p, double* g_out, int32_t cap) {
  int32_t kmax = (int32_t)ceil(log(p->qmax_fac / p->qmin_fac) / p->dlogq);
  double gcap = p->qmax_fac / p->qmin_fac;
  if (kmax + 1 > cap) return ORC_E_ARG;
  for (int32_t k = 0; k <= kmax; ++k) {
    double e = exp((double)k * p->dlogq);
    g_out[k] = e < gcap ? e : gcap;
  }
  return kmax + 1;
}

/* Bins of the k-th bin set: ceil(noverlap / q_k), q_k = q_lo g_k. */
static int32_t orc_rebin_nb(double qlo, double g, int32_t noverlap) {
  return (int32_t)ceil((double)noverlap / (qlo * g));
}

/* ------------------------------------------------------------------------- */
/* BLS for one star (Kovacs et al. 2002 statistic on the Keplerian grid).     */
/*   W = sum w;  wt = w / W;  ybar = sum wt y (compensated);  x = y - ybar.   */
/*   For each grid frequency f: phase = frac((t - t0) f), bin                 */
/*   b = min(nb-1, floor(phase nb)); H_W[b] += wt, H_S[b] += wt x.            */
/*   For each duration m (ascending) and start bin j: r = sum_{u<m} H_W[j+u], */
/*   s = sum_{u<m} H_S[j+u] (indices mod nb, summed in u order).  A window is */
/*   valid if m < nb and 0 < r < 1 (and s < 0 when dip_only); its power is    */
/*   s^2 / (r (1 - r)).  SR(f) = sqrt(max power); ties go to the smallest     */
/*   (m, j) in lexicographic order.  No valid window: SR = 0, m = 0, j = -1.  */
/* ------------------------------------------------------------------------- */
/* Neumaier compensated sum of a[i] (a == NULL: ones), times b[i] when b != NULL. */
static double orc_sum_comp(const double* a, const double* b, int64_t n) {
  double s = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v = a ? a[i] : 1.0;
    if (b) v = v * b[i];
    double t = s + v;
    if (fabs(s) >= fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  return s + c;
}

typedef struct {
  double* sr;   /* [nf] */
  int32_t* m;   /* [nf] best window length in bins */
  int32_t* j;   /* [nf] best window start bin */
  double* r;    /* [nf] in-window weight fraction of the best window */
  double* s;    /* [nf] in-window weighted residual sum of the best window */
  int32_t* nb;  /* [nf] fine bins at each frequency */
  double* f;    /* [nf] frequencies */
} orc_spectrum;

/* Normalised inputs of one star (Kovacs): wt = w / W, wx = wt (y - ybar), dt = t - t0. */
typedef struct {
  double* wt;
  double* wx;
  double* dt;
  int64_t n;
} orc_norm;

static int orc_normalise(const double* t, const double* y, const double* w, int64_t n, double t0,
                         orc_norm* o) {
  /* The weighted mean must be accurate in absolute terms: the flux level is far
   * above the signal, and s = sum_in wt (y - ybar) moves by r * (error of ybar).
   * Both sums therefore use Neumaier's compensated summation. */
  double W = orc_sum_comp(w, NULL, n);
  if (!(W > 0.0)) return ORC_E_INPUT;
  o->n = n;
  o->wt = (double*)malloc(sizeof(double) * (size_t)n);
  o->wx = (double*)malloc(sizeof(double) * (size_t)n);
  o->dt = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) o->wt[i] = (w ? w[i] : 1.0) / W;
  double ybar = orc_sum_comp(o->wt, y, n);
  for (int64_t i = 0; i < n; ++i) {
    o->wx[i] = o->wt[i] * (y[i] - ybar);
    o->dt[i] = t[i] - t0;
  }
  return ORC_OK;
}

static void orc_norm_free(orc_norm* o) {
  free(o->wt);
  free(o->wx);
  free(o->dt);
}

/* Fold, bin and scan at one frequency f with nb fine bins (hw, hs: nb scratch
 * values each).  Writes SR and the best window (m, j, r, s). */
static void orc_bls_freq(const orc_norm* d, double f, int32_t nb, const int32_t* mlist, int32_t nm,
                         int32_t dip_only, double* hw, double* hs, double* sr_out, int32_t* m_out,
                         int32_t* j_out, double* r_out, double* s_out) {
  for (int32_t k = 0; k < nb; ++k) hw[k] = hs[k] = 0.0;
  for (int64_t q = 0; q < d->n; ++q) {
    double ph = d->dt[q] * f;
    ph = ph - floor(ph);
    int32_t bin = (int32_t)floor(ph * (double)nb);
    if (bin >= nb) bin = nb - 1;
    hw[bin] += d->wt[q];
    hs[bin] += d->wx[q];
  }
  double best = -1.0, br = 0.0, bs = 0.0;
  int32_t bm = 0, bj = -1;
  for (int32_t mi = 0; mi < nm; ++mi) {
    int32_t m = mlist[mi];
    /* A window of nb or more bins covers every point (r = 1): never valid. */
    if (m >= nb) continue;
    for (int32_t j = 0; j < nb; ++j) {
      double r = 0.0, s = 0.0;
      for (int32_t u = 0; u < m; ++u) {
        int32_t k = (j + u) % nb;
        r += hw[k];
        s += hs[k];
      }
      if (!(r > 0.0 && r < 1.0)) continue;
      if (dip_only && !(s < 0.0)) continue;
      double pw = (s * s) / (r * (1.0 - r));
      if (pw > best) {
        best = pw;
        bm = m;
        bj = j;
        br = r;
        bs = s;
      }
    }
  }
  *sr_out = best >= 0.0 ? sqrt(best) : 0.0;
  *m_out = bm;
  *j_out = bj;
  *r_out = br;
  *s_out = bs;
}

/* Per-duration rebinning at one frequency (rebin = 1; the literal reading of the
 * cuvarbase parameters, Sec. 2.1 footnote): for each duration q_k of the continuous
 * ladder the phase circle gets its own nb_k = ceil(noverlap / q_k) bins, and the
 * windows are noverlap consecutive bins (cyclic) starting at every bin, i.e.
 * noverlap shifted bin sets of width about q_k.  Bin b = min(nb_k - 1,
 * floor(phase nb_k)); a window is valid when noverlap < nb_k and 0 < r < 1 (s < 0
 * with dip_only); ties go to the smallest (k, j).  Outputs: SR, k (in m), j, r, s
 * and the winning set's nb_k (nb_0 when no window is valid). */
static void orc_bls_freq_rebin(const orc_norm* d, double f, double qlo, const double* g, int32_t ng,
                               int32_t noverlap, int32_t dip_only, double* hw, double* hs, double* sr_out,
                               int32_t* k_out, int32_t* j_out, double* r_out, double* s_out,
                               int32_t* nb_out) {
  double best = -1.0, br = 0.0, bs = 0.0;
  int32_t bk = 0, bj = -1, bnb = orc_rebin_nb(qlo, g[0], noverlap);
  for (int32_t k = 0; k < ng; ++k) {
    int32_t nb = orc_rebin_nb(qlo, g[k], noverlap);
    if (noverlap >= nb) continue;
    for (int32_t b = 0; b < nb; ++b) hw[b] = hs[b] = 0.0;
    for (int64_t q = 0; q < d->n; ++q) {
      double ph = d->dt[q] * f;
      ph = ph - floor(ph);
      int32_t bin = (int32_t)floor(ph * (double)nb);
      if (bin >= nb) bin = nb - 1;
      hw[bin] += d->wt[q];
      hs[bin] += d->wx[q];
    }
    for (int32_t j = 0; j < nb; ++j) {
      double r = 0.0, s = 0.0;
      for (int32_t u = 0; u < noverlap; ++u) {
        int32_t c = (j + u) % nb;
        r += hw[c];
        s += hs[c];
      }
      if (!(r > 0.0 && r < 1.0)) continue;
      if (dip_only && !(s < 0.0)) continue;
      double pw = (s * s) / (r * (1.0 - r));
      if (pw > best) {
        best = pw;
        bk = k;
        bj = j;
        br = r;
        bs = s;
        bnb = nb;
      }
    }
  }
  *sr_out = best >= 0.0 ? sqrt(best) : 0.0;
  *k_out = bk;
  *j_out = bj;
  *r_out = br;
  *s_out = bs;
  *nb_out = bnb;
}

/* One grid frequency of a star in the configured mode; hw/hs hold nb_0 values. */
static void orc_search_at(const orc_norm* d, const orc_bounds_t* b, const orc_params* p, int64_t i,
                          const int32_t* mlist, int32_t nm, const double* g, int32_t ng, double* hw,
                          double* hs, orc_spectrum* out, int64_t o) {
  double uu;
  double f = orc_freq(b, i, &uu);
  out->f[o] = f;
  if (p->rebin) {
    orc_bls_freq_rebin(d, f, orc_qlo(b, p, uu), g, ng, p->noverlap, p->dip_only, hw, hs, out->sr + o,
                       out->m + o, out->j + o, out->r + o, out->s + o, out->nb + o);
  } else {
    int32_t nb = orc_nbins(b, p, uu);
    out->nb[o] = nb;
    orc_bls_freq(d, f, nb, mlist, nm, p->dip_only, hw, hs, out->sr + o, out->m + o, out->j + o,
                 out->r + o, out->s + o);
  }
}

/* Largest bin count the search uses at grid point i (the k = 0 set when rebinning). */
static int32_t orc_nb_needed(const orc_bounds_t* b, const orc_params* p, int64_t i, const double* g) {
  double uu;
  (void)orc_freq(b, i, &uu);
  if (p->rebin) return orc_rebin_nb(orc_qlo(b, p, uu), g[0], p->noverlap);
  return orc_nbins(b, p, uu);
}

int orc_bls_star(const double* t, const double* y, const double* w, int64_t n, double rho,
                 const orc_params* p, double pmin_override, double pmax_override,
                 orc_spectrum* out, int64_t cap, orc_bounds_t* bounds_out) {
  orc_bounds_t b;
  int st = orc_bounds(t, w, n, rho, p, pmin_override, pmax_override, &b);
  if (bounds_out) *bounds_out = b;
  if (st != ORC_OK) return st;
  if (b.nf > cap) return ORC_E_ARG;

  int32_t mlist[64];
  int32_t nm = orc_durations(p, mlist, 64);
  if (nm <= 0) return ORC_E_ARG;
  double g[64];
  int32_t ng = orc_rebin_ladder(p, g, 64);
  if (ng <= 0) return ORC_E_ARG;
  orc_norm d;
  st = orc_normalise(t, y, w, n, b.t0, &d);
  if (st != ORC_OK) return st;

  int32_t nb_max = 1;
  for (int64_t i = 0; i < b.nf; ++i) {
    int32_t nbi = orc_nb_needed(&b, p, i, g);
    if (nbi > nb_max) nb_max = nbi;
  }
  double* hw = (double*)malloc(sizeof(double) * (size_t)nb_max);
  double* hs = (double*)malloc(sizeof(double) * (size_t)nb_max);

  for (int64_t i = 0; i < b.nf; ++i) orc_search_at(&d, &b, p, i, mlist, nm, g, ng, hw, hs, out, i);
  free(hw);
  free(hs);
  orc_norm_free(&d);
  return ORC_OK;
}

/* The same search at a listed subset of the star's grid indices idx[0..k)
 * (each in [0, nf)); outputs are indexed like idx.  Used to check long
 * spectra at sampled frequencies and to time the oracle on a bounded sample. */
int orc_bls_star_at(const double* t, const double* y, const double* w, int64_t n, double rho,
                    const orc_params* p, double pmin_override, double pmax_override,
                    const int64_t* idx, int64_t k, orc_spectrum* out, orc_bounds_t* bounds_out) {
  orc_bounds_t b;
  int st = orc_bounds(t, w, n, rho, p, pmin_override, pmax_override, &b);
  if (bounds_out) *bounds_out = b;
  if (st != ORC_OK) return st;
  for (int64_t q = 0; q < k; ++q)
    if (idx[q] < 0 || idx[q] >= b.nf) return ORC_E_ARG;
  int32_t mlist[64];
  int32_t nm = orc_durations(p, mlist, 64);
  if (nm <= 0) return ORC_E_ARG;
  double g[64];
  int32_t ng = orc_rebin_ladder(p, g, 64);
  if (ng <= 0) return ORC_E_ARG;
  orc_norm d;
  st = orc_normalise(t, y, w, n, b.t0, &d);
  if (st != ORC_OK) return st;
  int32_t nb_max = 1;
  for (int64_t q = 0; q < k; ++q) {
    int32_t nbi = orc_nb_needed(&b, p, idx[q], g);
    if (nbi > nb_max) nb_max = nbi;
  }
  double* hw = (double*)malloc(sizeof(double) * (size_t)nb_max);
  double* hs = (double*)malloc(sizeof(double) * (size_t)nb_max);
  for (int64_t q = 0; q < k; ++q) orc_search_at(&d, &b, p, idx[q], mlist, nm, g, ng, hw, hs, out, q);
  free(hw);
  free(hs);
  orc_norm_free(&d);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Spectroscopic S/N (Sec. 2.2 item 1, Eq. 1 with its two changes).           */
/*   N_b = round(1 + 3.322 log10 n) Sturges bins (footnote; half rounds up),  */
/*   equal width in frequency between the first and last grid frequency.      */
/*   Knot of a non-empty bin k: centre x_k = f_0 + (k + 1/2) span / N_b,       */
/*   value = median SR of the bin (even count: mean of the middle two).       */
/*   Trend: linear interpolation between knots, constant beyond the ends.     */
/*   rho_i = SR_i - trend_i;  sigma = 1.4826 median|rho - median(rho)|.        */
/*   S/N_i = rho_i / sigma (sigma = 0: status 1 and S/N = 0).                  */
/*   The detection is argmax S/N; argmax SR is reported too (first on ties).   */
/* ------------------------------------------------------------------------- */
static int orc_cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* Median of v[0..n) (n >= 1) by sorting a copy. */
double orc_median(const double* v, int64_t n) {
  double* c = (double*)malloc(sizeof(double) * (size_t)n);
  memcpy(c, v, sizeof(double) * (size_t)n);
  qsort(c, (size_t)n, sizeof(double), orc_cmp_double);
  double med = (n & 1) ? c[n / 2] : (c[n / 2 - 1] + c[n / 2]) * 0.5;
  free(c);
  return med;
}

int32_t orc_sturges(int64_t n) {
  int32_t nb = (int32_t)floor(1.0 + 3.322 * log10((double)n) + 0.5);
  return nb < 1 ? 1 : nb;
}

typedef struct {
  int64_t i_snr, i_sr;
  double snr_max, sr_max, trend_at, sigma, median_resid;
  int32_t status, nbins_sturges;
} orc_snr_result;

int orc_snr(const double* f, const double* sr, int64_t n, const orc_params* p, double* snr,
            double* trend, orc_snr_result* res) {
  if (n < 1) return ORC_E_ARG;
  int32_t nbins = orc_sturges(n);
  double f0 = f[0], span = f[n - 1] - f[0];
  int32_t* k = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    int32_t ki = 0;
    if (span > 0.0) ki = (int32_t)floor(((f[i] - f0) / span) * (double)nbins);
    if (ki >= nbins) ki = nbins - 1;
    if (ki < 0) ki = 0;
    k[i] = ki;
  }
  double* kx = (double*)malloc(sizeof(double) * (size_t)nbins);
  double* ky = (double*)malloc(sizeof(double) * (size_t)nbins);
  double* buf = (double*)malloc(sizeof(double) * (size_t)n);
  int32_t nk = 0;
  for (int32_t b = 0; b < nbins; ++b) {
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i)
      if (k[i] == b) buf[c++] = sr[i];
    if (c == 0) continue;
    kx[nk] = f0 + (((double)b + 0.5) * span) / (double)nbins;
    ky[nk] = orc_median(buf, c);
    ++nk;
  }
  double* rho = (double*)malloc(sizeof(double) * (size_t)n);
  double* trv = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    double tr;
    if (f[i] <= kx[0]) {
      tr = ky[0];
    } else if (f[i] >= kx[nk - 1]) {
      tr = ky[nk - 1];
    } else {
      int32_t a = 0;
      while (a + 1 < nk && kx[a + 1] <= f[i]) ++a;
      double slope = (ky[a + 1] - ky[a]) / (kx[a + 1] - kx[a]);
      tr = slope * (f[i] - kx[a]) + ky[a];
    }
    if (trend) trend[i] = tr;
    trv[i] = tr;
    rho[i] = sr[i] - tr;
  }
  const double* base = p->mad_of_raw ? sr : rho;
  double med = orc_median(base, n);
  for (int64_t i = 0; i < n; ++i) buf[i] = fabs(base[i] - med);
  double sigma = 1.4826 * orc_median(buf, n);
  int32_t status = 0;
  if (!(sigma > 0.0) || isinf(sigma)) status = 1;
  int64_t i_snr = 0, i_sr = 0;
  double best = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v = status ? 0.0 : rho[i] / sigma;
    if (snr) snr[i] = v;
    if (i == 0 || v > best) {
      best = v;
      i_snr = i;
    }
    if (sr[i] > sr[i_sr]) i_sr = i;
  }
  double trend_i_snr = trv[i_snr];
  if (res) {
    res->i_snr = i_snr;
    res->i_sr = i_sr;
    res->snr_max = status ? 0.0 : rho[i_snr] / sigma;
    res->sr_max = sr[i_sr];
    res->trend_at = trend_i_snr;
    res->sigma = sigma;
    res->median_resid = p->mad_of_raw ? orc_median(rho, n) : med;
    res->status = status;
    res->nbins_sturges = nbins;
  }
  free(k);
  free(kx);
  free(ky);
  free(buf);
  free(rho);
  free(trv);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Batch driver: stars are independent; OpenMP spreads them over threads.     */
/* offsets[S+1] index the packed t/y/w arrays; fofs[S+1] index the per-       */
/* frequency outputs (sizes from orc_batch_sizes).  res[S*12] holds per star: */
/* i_snr, i_sr, period, t0, duration, depth, sr, snr, trend, sigma, status,   */
/* nf (as doubles).                                                           */
/* ------------------------------------------------------------------------- */
int orc_batch_sizes(int32_t S, const int64_t* offsets, const double* t, const double* w,
                    const double* rho, const double* pmin_o, const double* pmax_o,
                    const orc_params* p, int64_t* nf_out, int32_t* status_out) {
  int bad = 0;
  for (int32_t s = 0; s < S; ++s) {
    int64_t o = offsets[s], n = offsets[s + 1] - offsets[s];
    orc_bounds_t b;
    int st = orc_bounds(t + o, w ? w + o : NULL, n, rho ? rho[s] : 1.0, p, pmin_o ? pmin_o[s] : 0.0,
                        pmax_o ? pmax_o[s] : 0.0, &b);
    status_out[s] = st;
    nf_out[s] = (st == ORC_OK) ? b.nf : 0;
    if (st != ORC_OK) bad = 1;
  }
  return bad ? ORC_E_INPUT : ORC_OK;
}

int orc_batch_run(int32_t S, const int64_t* offsets, const double* t, const double* y,
                  const double* w, const double* rho, const double* pmin_o, const double* pmax_o,
                  const orc_params* p, const int64_t* fofs, double* f, int32_t* nb, double* sr,
                  int32_t* m, int32_t* j, double* r, double* s_out, double* snr, double* trend,
                  double* res, int32_t nthreads) {
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
#endif
  for (int32_t st = 0; st < S; ++st) {
    int64_t o = offsets[st], n = offsets[st + 1] - offsets[st];
    int64_t fo = fofs[st], nf = fofs[st + 1] - fofs[st];
    orc_spectrum sp = {sr + fo, m + fo, j + fo, r + fo, s_out + fo, nb + fo, f + fo};
    orc_bounds_t b;
    int code = orc_bls_star(t + o, y + o, w ? w + o : NULL, n, rho ? rho[st] : 1.0, p,
                            pmin_o ? pmin_o[st] : 0.0, pmax_o ? pmax_o[st] : 0.0, &sp, nf, &b);
    double* R = res + (int64_t)st * 12;
    if (code != ORC_OK || b.nf != nf) {
      err |= 1;
      for (int q = 0; q < 12; ++q) R[q] = NAN;
      continue;
    }
    orc_snr_result sres;
    orc_snr(f + fo, sr + fo, nf, p, snr ? snr + fo : NULL, trend ? trend + fo : NULL, &sres);
    int64_t i = sres.i_snr;
    double fi = f[fo + i];
    /* rebinning: m holds the duration index; the window is noverlap bins of nb */
    int32_t mi = p->rebin ? p->noverlap : m[fo + i], ji = j[fo + i], nbi = nb[fo + i];
    double ri = r[fo + i], si = s_out[fo + i];
    R[0] = (double)sres.i_snr;
    R[1] = (double)sres.i_sr;
    R[2] = 1.0 / fi;
    if (ji >= 0) {
      double c = ((double)ji + 0.5 * (double)mi) / (double)nbi;
      c = c - floor(c);
      R[3] = b.t0 + c / fi;
      R[4] = ((double)mi / (double)nbi) / fi;
      R[5] = -si / (ri * (1.0 - ri));
    } else {
      R[3] = R[4] = R[5] = NAN;
    }
    R[6] = sr[fo + i];
    R[7] = sres.snr_max;
    R[8] = sres.trend_at;
    R[9] = sres.sigma;
    R[10] = (double)sres.status;
    R[11] = (double)nf;
  }
  return err ? ORC_E_INPUT : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Other statistics of the detection (Sec. 2.2 item 5) and the detection     */
/* criteria (the paragraph after the list), at the best window of one       */
/* frequency f with nb fine bins: duration m bins starting at bin j.         */
/* Only points with w > 0 count as data.  With p = (t - t0) f, its integer   */
/* part ip and bin b = min(nb - 1, floor((p - ip) nb)) (the search's fold),  */
/* o = (b - j) mod nb places a point relative to the window:                 */
/*   in transit      o < m                (within half a duration of the    */
/*                                          mid-transit time, to a fine bin)*/
/*   after transit   m <= o < 2m          (one duration after egress)       */
/*   before transit  o >= max(2m, nb - m) (one duration before ingress)     */
/* Transit number of a point: k = floor((ip nb + b - j) / nb), the cycle in */
/* which its window starts; a transit counts when at least one in-transit   */
/* point has its number.  Out-of-transit level: sum w y / sum w over points  */
/* not in transit.  Candidate: at least two transits and S/N > 9.            */
/* out: n_in, n_before, n_after, n_transits, candidate (as doubles), level.  */
/* ------------------------------------------------------------------------- */
static int64_t orc_floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
  return q;
}

static int orc_cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x < y) ? -1 : (x > y) ? 1 : 0;
}

int orc_stats(const double* t, const double* y, const double* w, int64_t n, double t0, double f,
              int32_t nb, int32_t m, int32_t j, double snr, double* out) {
  if (!t || !y || !out || n < 1 || nb < 1 || m < 1 || m >= nb || j < 0 || j >= nb) return ORC_E_ARG;
  int64_t n_in = 0, n_before = 0, n_after = 0, nk = 0;
  int64_t* ks = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  double sw = 0.0, swy = 0.0;
  for (int64_t q = 0; q < n; ++q) {
    double wq = w ? w[q] : 1.0;
    if (!(wq > 0.0)) continue;
    double p = (t[q] - t0) * f;
    double ip = floor(p);
    int32_t b = (int32_t)floor((p - ip) * (double)nb);
    if (b >= nb) b = nb - 1;
    int32_t o = b - j;
    if (o < 0) o += nb;
    if (o < m) {
      ++n_in;
      ks[nk++] = orc_floor_div((int64_t)ip * nb + b - j, nb);
    } else {
      if (o < 2 * m) ++n_after;
      else if (o >= nb - m) ++n_before;
      sw += wq;
      swy += wq * y[q];
    }
  }
  qsort(ks, (size_t)nk, sizeof(int64_t), orc_cmp_i64);
  int64_t n_tr = 0;
  for (int64_t q = 0; q < nk; ++q)
    if (q == 0 || ks[q] != ks[q - 1]) ++n_tr;
  free(ks);
  out[0] = (double)n_in;
  out[1] = (double)n_before;
  out[2] = (double)n_after;
  out[3] = (double)n_tr;
  out[4] = (n_tr >= 2 && snr > 9.0) ? 1.0 : 0.0;
  out[5] = sw > 0.0 ? swy / sw : NAN;
  return ORC_OK;
}

/* Threads OpenMP would use (for reporting the CPU baseline's core count). */
int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
