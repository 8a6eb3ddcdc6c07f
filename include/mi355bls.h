/*
 * mi355bls.h — C ABI of the MI355X (gfx950) Box Least Squares transit search.
 *
 * The library computes, for many light curves at once, the Box Least Squares
 * periodogram of Kovacs, Zucker & Mazeh (2002) on a per-star Keplerian
 * frequency grid, followed by the spectroscopic S/N post-processing of QLP Data
 * Release Notes 003 (Kunimoto et al. 2023):
 *   - search grid and durations: Sec. 2.1 and its footnote (Keplerian duration
 *     window 0.5-2.0 x the circular-orbit duration at the star's density,
 *     samples_per_peak = 2, dlogq = 0.1, noverlap = 3);
 *   - period bounds: Sec. 2.1 (a = 2 R* or 3 R* for the minimum period; the
 *     longest continuous stretch, or half of it without gaps longer than a
 *     sector, for the maximum);
 *   - S/N: Sec. 2.2 item 1, Eq. 1 with its two changes (Sturges-rule
 *     median-binned trend; sigma = 1.4826 x MAD).
 *
 * Conventions
 *   - Every function returns a bls_status (0 = success, < 0 = error).  No C++
 *     exception crosses the ABI.  bls_status_string() names a code.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *     memory of the current device.  The caller owns every buffer it passes.
 *   - A plan owns host-side descriptors only.  Device state lives in a caller
 *     allocated workspace of bls_plan_query(...)->workspace_bytes bytes, filled by
 *     bls_plan_upload().  bls_search_batch() and bls_snr() allocate nothing, never
 *     synchronise the host and only enqueue work on the given stream, so they can
 *     be captured into a HIP graph.  A plan and its workspace serve one stream at
 *     a time.
 *   - Light curves are packed back to back ("ragged CSR"): star s owns points
 *     [off_s, off_s + n_points_s) of the t/y/w arrays, off_0 = 0.  Times are in
 *     days, ascending within a star; flux is unitless; weights are 1/sigma^2 (>= 0,
 *     points with w = 0 contribute nothing and are ignored for the baseline).
 *   - Per-frequency outputs of all stars are packed the same way, star s owning
 *     [freq_offsets[s], freq_offsets[s+1]) (bls_plan_query).
 */
#ifndef MI355BLS_H
#define MI355BLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* bls_stream_t; /* a hipStream_t; NULL = default stream */

typedef int32_t bls_status;
enum {
  BLS_OK = 0,
  BLS_E_ARG = -1,         /* invalid argument (NULL pointer, bad size or parameter) */
  BLS_E_INPUT = -2,       /* invalid light curve: non-finite value, w < 0, times not
                             ascending, fewer than 2 weighted points, zero total weight */
  BLS_E_EMPTY_GRID = -3,  /* Pmin >= Pmax for a star: nothing to search */
  BLS_E_NOMEM = -4,       /* host allocation failed */
  BLS_E_HIP = -5,         /* a HIP call failed (launch or copy) */
  BLS_E_STATE = -6,       /* workspace missing, too small or not uploaded */
  BLS_E_UNSUPPORTED = -7, /* a star exceeds a compiled limit (see bls_limits) */
  BLS_E_SCRATCH = -8      /* the plan's workspace exceeds the static scratch of
                             bls_run_noalloc (MI355BLS_NOALLOC_SCRATCH_BYTES) */
};

/* Search parameters.  bls_default_params() fills the paper's values (Sec. 2.1,
 * its footnote, and Sec. 2.2). */
typedef struct bls_params {
  double spp;          /* samples per peak of the frequency grid (2) */
  double qmin_fac;     /* shortest duration / circular duration (0.5) */
  double qmax_fac;     /* longest duration / circular duration (2.0) */
  double dlogq;        /* natural-log spacing of the duration ladder (0.1) */
  int32_t noverlap;    /* shifted bin sets per shortest duration (3) */
  int32_t dip_only;    /* 0: windows of either sign count (Kovacs s^2); 1: s < 0 only */
  int32_t mad_of_raw;  /* 0: sigma from the MAD of the detrended SR (default);
                          1: from the MAD of raw SR */
  int32_t precision;   /* 0: FP64 phase, exact int64 fixed-point bin sums (plain path);
                          1: FP64 phase, weights (2^-27) and weighted residuals packed
                          into one 64-bit fixed-point sum per bin: half the LDS atomics,
                          SR within ~1e-5 relative of the exact sums (reduced precision;
                          best-period indices can differ at near-ties) */
  double a_min_rstar;  /* minimum a/R*: 2 (Sectors 61+) or 3 (Sectors 59-60) */
  double sector_days;  /* gap length that splits continuous stretches (27.4) */
  int64_t tile_cells;  /* target points x frequencies per work item; 0 = library default
                          (6 Mi cells and at most 128 frequencies per item); an
                          autotuner may pick another (results do not change) */
  int64_t big_points;  /* stars with more points search every frequency in the large
                          workgroup shape (fewer point re-reads); 0 = 100,000 (results
                          do not change) */
  int32_t item_freqs;  /* most frequencies per work item; 0 = 128, or 4096 when
                          tile_cells is set (results do not change) */
  int32_t exact_duration; /* 0: circular duration (P / pi)(R* / a), the small-angle
                          form (default); 1: (P / pi) asin(R* / a), the exact central
                          transit of a circular orbit (Sec. 2.1): only the fine-bin
                          count nb changes (the frequency grid keeps the small-angle
                          spacing, which is the finer one) */
  int32_t rebin;       /* 0: one fine-bin set per frequency, windows of m bins from the
                          duration ladder (default); 1: one bin set per duration of a
                          continuous ladder q_k = min(e^(k dlogq), qmax/qmin) q_lo
                          (k = 0..ceil(ln(qmax/qmin)/dlogq)) with nb_k =
                          ceil(noverlap / q_k) bins and windows of noverlap bins
                          (the literal reading of the noverlap parameter, Sec. 2.1
                          footnote); bls_best.m then holds k.  Needs precision 0. */
  int32_t reserved;    /* 0 */
} bls_params;

/* Per-star inputs. */
typedef struct bls_star {
  int64_t n_points;    /* points of this star in the packed arrays (>= 2) */
  double rho_solar;    /* stellar density in solar units; NaN or <= 0 means solar */
  double pmin_days;    /* > 0 overrides the minimum period (else a = a_min_rstar) */
  double pmax_days;    /* > 0 overrides the maximum period (else from the stretches) */
} bls_star;

/* Best window at one frequency: m bins starting at fine bin j (start phase j/nb);
 * r = in-window weight fraction, s = in-window sum of w~ (y - ybar).
 * m = 0, j = -1 when no window is valid (then SR = 0).  With rebin = 1, m is the
 * duration index k and the window is noverlap bins of that duration's bin set
 * (nb_k bins), starting at its bin j. */
typedef struct bls_best {
  int32_t m, j;
  double r, s;
} bls_best;

/* Per-star summary written by bls_snr(). */
typedef struct bls_result {
  int64_t i_snr;       /* frequency index (within the star) of the maximum S/N */
  int64_t i_sr;        /* frequency index of the maximum SR */
  double period;       /* 1 / f at i_snr, days */
  double t0;           /* mid-time of the best window at i_snr (first after the
                          star's first weighted time), days; NaN without d_best */
  double duration;     /* (m / nb) / f, days; NaN without d_best */
  double depth;        /* -s / (r (1 - r)), positive for a dip; NaN without d_best */
  double sr;           /* SR at i_snr */
  double snr;          /* S/N at i_snr */
  double trend;        /* median-binned trend at i_snr */
  double sigma;        /* 1.4826 x MAD */
  int32_t status;      /* 0 ok; 1 sigma = 0 (S/N set to 0) */
  int32_t nbins;       /* Sturges bin count used for the trend */
} bls_result;

/* Other statistics of a star's detection (Sec. 2.2 item 5) and its detection
 * criteria (the paragraph after the list), written by bls_stats(). */
typedef struct bls_star_stats {
  int64_t n_in;        /* points (w > 0) in transit: in the best window's m fine bins */
  int64_t n_before;    /* points within one duration before ingress */
  int64_t n_after;     /* points within one duration after egress */
  int64_t n_transits;  /* transits with data within half a duration of mid-transit */
  double oot_level;    /* sum w y / sum w over the points out of transit (NaN if none) */
  int32_t candidate;   /* 1: n_transits >= 2 and S/N > the threshold (9 in the note) */
  int32_t status;      /* 0 ok; 1 no valid window at the detection frequency (counts 0) */
} bls_star_stats;

/* Trapezoid fit, noise and S/N_pink of a star's detection (Sec. 2.2 items 2-4) and
 * the complete detection criteria, written by bls_fit(). */
typedef struct bls_fit_result {
  double t0;           /* fitted mid-transit time, days */
  double depth;        /* fitted depth delta (flux; positive for a dip) */
  double q;            /* fitted duration / period */
  double q_in;         /* fitted ingress duration / duration, in [0, 0.5] */
  double level;        /* fitted out-of-transit level z */
  double chi2;         /* sum w (y - model)^2 over the fit points */
  double sigma_w;      /* white noise: standard deviation of y - model (w > 0 points) */
  double sigma_r;      /* red noise on the duration time scale */
  double depth_eff;    /* depth integral over the duration / duration = depth (1 - q_in) */
  double snr_pink;     /* depth_eff / sqrt(sigma_w^2 / n_t + sigma_r^2 / N_t) (Eq. 2);
                          +inf without residual scatter */
  int64_t n_fit;       /* points within two starting durations of mid-transit */
  int64_t n_t;         /* points in transit (|t - mid-transit| < duration / 2) */
  int64_t n_transits;  /* transits holding at least one of them */
  int32_t iterations;  /* Levenberg-Marquardt iterations */
  int32_t candidate;   /* 1: n_transits >= 2, snr_pink > pink_min and S/N > snr_min */
  int32_t status;      /* 0 ok; 1 no detection to start from (needs d_best in bls_snr);
                          2 no point within two durations */
  int32_t pad;
} bls_fit_result;

typedef struct bls_plan bls_plan;

/* Fill *p with the paper's parameters. */
bls_status bls_default_params(bls_params* p);

/* Build a plan for n_stars light curves (host work only, synchronous).
 * t_host: packed times [sum n_points] (required).  y_host, w_host: packed
 * fluxes and weights (nullable: NULL skips the flux check / means unit weights);
 * they must equal the device arrays later given to bls_search_batch().
 * Validates every star (BLS_E_INPUT, BLS_E_EMPTY_GRID), then derives per star the
 * baseline, the period bounds (Sec. 2.1), the frequency grid (uniform in f^(1/3),
 * spacing 1/spp of the shortest searched duration over the baseline) and the
 * work schedule.  On error *out is NULL and *bad_star (nullable) names the star. */
bls_status bls_plan_create(const bls_params* p, int32_t n_stars, const bls_star* stars,
                           const double* t_host, const double* y_host, const double* w_host,
                           bls_plan** out, int32_t* bad_star);

/* Sizes of a plan.  n_freq_total: frequencies of all stars.  freq_offsets_host
 * (nullable) receives n_stars + 1 prefix offsets.  workspace_bytes: device bytes the
 * caller must allocate (256-byte aligned) and pass to upload/search/snr. */
bls_status bls_plan_query(const bls_plan* plan, int64_t* n_freq_total, int64_t* freq_offsets_host,
                          int64_t* workspace_bytes);

/* Per-star description: out[0..9] = t0, T, pmin, pmax, krho (circular duty cycle
 * coefficient, q = krho f^(2/3)), umin, A (grid: f_i = (umin + i A)^3), nf,
 * nb_max, sturges bins. */
bls_status bls_plan_star_info(const bls_plan* plan, int32_t star, double* out10);

/* Frequencies (1/day) and fine-bin counts of one star's grid, exactly as the
 * device computes them (f_host [nf], nb_host [nf], both host, nullable).  With
 * exact_duration the count goes through asin, the host's libm here and the device
 * math library there; the two can differ in the last place, which changes nb only
 * where noverlap / q_lo lies within that of an integer.  With rebin, nb is the
 * count of the k = 0 bin set (the largest). */
bls_status bls_plan_frequencies(const bls_plan* plan, int32_t star, double* f_host, int32_t* nb_host);

/* The fine-bin duration ladder: writes up to cap lengths, returns the count
 * through *n. */
bls_status bls_plan_durations(const bls_plan* plan, int32_t* m_host, int32_t cap, int32_t* n);

/* Copy the plan's descriptors into the device workspace (enqueued on stream;
 * the host copy stays owned by the plan, which must outlive the copy). */
bls_status bls_plan_upload(bls_plan* plan, void* d_workspace, int64_t workspace_bytes,
                           bls_stream_t stream);

/* Preparation of a batch (the normalisation of Kovacs et al. 2002 as used in
 * Sec. 2.2 item 1): per star W = sum w, wt = w / W, ybar = sum wt y (compensated
 * sums), x = y - ybar; then dt = t - t0 and the exclusive prefix sums of wt and of
 * wt x in int64 fixed point, stored in the workspace.  Device inputs: packed t, y
 * (required) and w (nullable: unit weights), identical to the host arrays given to
 * bls_plan_create().  It also notes, per star, whether every point of nonzero weight
 * carries the same fixed-point weight; bls_search_batch() then sums counts of such
 * points in place of weight prefixes (the same integers once multiplied back, so the
 * same results).  Must precede bls_search_batch() on the same stream. */
bls_status bls_prepare(bls_plan* plan, void* d_workspace, const double* d_t, const double* d_y,
                       const double* d_w, bls_stream_t stream);

/* BLS search (Kovacs statistic on the Sec. 2.1 grid) over prepared data.  For every
 * frequency: phase-fold, fine-bin sums, every window of m fine bins (m in the
 * duration ladder) starting at every fine bin; SR = sqrt(max s^2 / (r (1 - r))) over
 * windows with m < nb and 0 < r < 1 (and s < 0 if dip_only), ties to the smallest
 * (m, j).  Outputs (device, caller-owned):
 *   d_sr   [n_freq_total]  SR per frequency;
 *   d_best [n_freq_total]  best window per frequency (nullable).
 * d_windows (nullable) restricts the search to n_windows triples
 * (star, i_begin, i_end) of int64 (device, row-major [n_windows][3]); each range is
 * clipped to [0, nf) of its star, triples naming no star of the plan are skipped,
 * and frequencies outside the ranges are not written.  NULL searches every star's
 * full grid; a non-NULL list with n_windows = 0 does nothing.  The per-frequency
 * results do not depend on how the grid is split into ranges. */
bls_status bls_search_batch(bls_plan* plan, void* d_workspace, const int64_t* d_windows,
                            int64_t n_windows, double* d_sr, bls_best* d_best, bls_stream_t stream);

/* Spectroscopic S/N (Sec. 2.2 item 1, Eq. 1 with the median-binned trend and the
 * MAD-based sigma).  d_sr: SR of every frequency (device).  d_best (nullable) feeds
 * t0/duration/depth of the result.  d_snr (nullable, device [n_freq_total]) gets
 * S/N per frequency.  d_result (device [n_stars]) gets the summary. */
bls_status bls_snr(bls_plan* plan, void* d_workspace, const double* d_sr, const bls_best* d_best,
                   double* d_snr, bls_result* d_result, bls_stream_t stream);

/* Other statistics of each star's detection (Sec. 2.2 item 5) and the detection
 * criteria of the paragraph after that list, at the best window (m fine bins from
 * bin j, from d_best) of the detection frequency i_snr (from d_result), using the
 * search's own phase fold of f_i with nb_i fine bins.  A point (w > 0) is in transit
 * when its bin lies in the window (within half a duration of mid-transit, to one fine
 * bin), after transit in the m bins that follow, before transit in the m bins that
 * precede (never both); a transit counts when at least one in-transit point falls
 * in its cycle.  candidate = (n_transits >= 2 && S/N > snr_min); the note's
 * threshold is 9, and its third criterion (S/N_pink, from the trapezoid fit of items
 * 2-4) is not part of this flag.  Device inputs: the packed t, y, w (w nullable:
 * unit weights) given to bls_prepare, d_best [n_freq_total] and d_result [n_stars]
 * of the same plan; output d_stats [n_stars].  The workspace must hold the plan
 * (bls_plan_upload).  Enqueued on stream; allocates nothing. */
bls_status bls_stats(bls_plan* plan, void* d_workspace, const double* d_t, const double* d_y, const double* d_w,
                     const bls_best* d_best, const bls_result* d_result, double snr_min,
                     bls_star_stats* d_stats, bls_stream_t stream);

/* Trapezoid fit of each star's detection and the statistics built on it (Sec. 2.2
 * items 2-4; the note's detection criteria in the paragraph after that list).
 * Starts from d_result (bls_snr with d_best: period, mid-transit time, duration and
 * depth of the best-S/N window); the period stays fixed.  Fits T0, depth, q = duration
 * / period, q_in = ingress / duration and the out-of-transit level z to the points
 * (w > 0) within two starting durations of mid-transit, flux = z - depth s with s the
 * trapezoid (1 in the flat bottom, linear ingress and egress, 0 outside), by
 * weighted Levenberg-Marquardt (start q_in = 0.2, lambda 1e-3, x10 / /10, at most 60
 * iterations, stop when a kept step lowers chi^2 by at most 1e-10 of it); q in
 * [1e-6, 1], q_in in [0, 0.5].  Then, over every w > 0 point: sigma_w = standard
 * deviation of y - model; sigma_r^2 = max(0, sigma_D^2 - sigma_w^2 / n_bar) from the
 * scatter sigma_D of the mean residuals in bins of one fitted duration (n_bar points
 * per non-empty bin); S/N_pink (Eq. 2) with the depth replaced by the trapezoid's mean
 * depth over the duration.  candidate = (n_transits >= 2 && snr_pink > pink_min &&
 * S/N > snr_min); the note uses 9 and 9.  Device inputs: the packed t, y, w (w
 * nullable) given to bls_prepare and d_result [n_stars]; output d_fit [n_stars].
 * Enqueued on stream; allocates nothing; deterministic (fixed reduction order). */
bls_status bls_fit(bls_plan* plan, void* d_workspace, const double* d_t, const double* d_y, const double* d_w,
                   const bls_result* d_result, double snr_min, double pink_min, bls_fit_result* d_fit,
                   bls_stream_t stream);

/* Release a plan (host memory only). */
void bls_plan_destroy(bls_plan* plan);

/* Static text naming a status code. */
const char* bls_status_string(bls_status s);

/* HIP error code (hipError_t value) of the last HIP call that failed inside the
 * library on the calling thread, behind a BLS_E_HIP return; 0 if none. */
int32_t bls_last_hip_error(void);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the whole device path of a
 * plan -- bls_plan_upload, bls_prepare, bls_search_batch and bls_snr with the same
 * arguments and results -- on a workspace held in a static device array of
 * MI355BLS_NOALLOC_SCRATCH_BYTES bytes (one per GPU, kept until the process ends)
 * instead of a caller allocation.  The caller still owns the inputs d_t, d_y, d_w
 * (w nullable) and the outputs d_sr, d_best (nullable), d_snr (nullable) and
 * d_result; d_windows / n_windows as for bls_search_batch.  Returns BLS_E_SCRATCH,
 * enqueueing nothing, when the plan's workspace (bls_plan_query) is larger.  Calls no
 * allocating routine.  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams, other threads) race and must be serialised by
 * the caller; a plan used here is uploaded to that array, so a later bls_prepare /
 * bls_search_batch / bls_snr on it needs a bls_plan_upload to its own workspace. */
#define MI355BLS_NOALLOC_SCRATCH_BYTES (64LL << 20)
bls_status bls_run_noalloc(bls_plan* plan, const double* d_t, const double* d_y, const double* d_w,
                           const int64_t* d_windows, int64_t n_windows, double* d_sr, bls_best* d_best,
                           double* d_snr, bls_result* d_result, bls_stream_t stream);

/* Compiled limits: out[0] = maximum fine bins per frequency, out[1] = maximum
 * duration-ladder length, out[2] = maximum points per star. */
bls_status bls_limits(int64_t* out3);

#ifdef __cplusplus
}
#endif
#endif /* MI355BLS_H */
