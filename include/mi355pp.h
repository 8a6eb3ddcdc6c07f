/* mi355pp.h — learned period proposal for the MI355X BLS library (libmi355bls.so).
 *
 * QLP Data Release Notes 003 searches every period of the Keplerian grid
 * (Sec. 2.1) with BLS and ranks them by the spectroscopic S/N (Sec. 2.2 item 1).
 * This optional front end guesses where the period is before that search: a small
 * 1-D CNN reads a resampled light curve and returns a heatmap over 512 log-spaced
 * period bins between 0.5 and 100 d plus a "no signal" class.  The few windows it
 * proposes are searched with the same BLS kernels (bls_search_batch with a window
 * list), periods beyond 100 d are always searched, and a star whose proposal is
 * not confident falls back to its full grid, so every reported detection is a
 * plain-BLS measurement.
 *
 * Conventions are those of mi355bls.h: caller-owned device buffers, no allocation,
 * work enqueued on the given stream, bls_status return codes.
 *
 * Network parameters are one FP32 vector of PP_NPARAM values (the master
 * weights); the forward pass rounds the two convolution weight tensors and the
 * activations to BF16 and accumulates in FP32 on the matrix cores.  Layout of
 * the vector: W1[16][2][16], b1[16], W2[16][16][8], b2[16], w3[16], alpha,
 * beta[512], delta.
 */
#ifndef MI355PP_H
#define MI355PP_H

#include <stdint.h>

#include "mi355bls.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PP_NPARAM 3122              /* network parameters */
#define PP_NCLASS 513               /* 512 period bins + the null class */
#define PP_NBINS_IN 4096            /* resampled bins per light curve */
#define PP_MAX_WINDOWS 16           /* window triples per star written by pp_propose */
#define PP_ACT_BYTES_PER_STAR 106496 /* saved activations per star (training) */

/* Bytes of saved activations for a batch (pp_forward's d_act, pp_backward). */
bls_status pp_act_bytes(int32_t batch, int64_t* bytes);

/* Resample every star of a plan onto 4096 uniform bins over its weighted baseline
 * [t0, t_last] (the plan's baseline).  With z = (y - median y) / (1.4826 MAD y)
 * over points with w > 0: d_x[s][0][b] = sum w z / sum w over the bin's points,
 * d_x[s][1][b] = 1 if the bin holds weight, else both 0; values are BF16 bit
 * patterns (uint16), row-major [n_stars][2][4096].  d_lag[s] (FP64) = baseline /
 * 1024, the time step between the network's output positions.  d_t/d_y/d_w are the
 * packed arrays given to bls_prepare (d_w nullable).  Needs bls_plan_upload. */
bls_status pp_resample(const bls_plan* plan, void* d_workspace, const double* d_t, const double* d_y,
                       const double* d_w, uint16_t* d_x, double* d_lag, bls_stream_t stream);

/* Forward pass for a batch: d_theta [PP_NPARAM] FP32, d_x [batch][2][4096] BF16,
 * d_lag [batch] FP64 -> d_logits [batch][PP_NCLASS] FP32.  d_act (nullable,
 * pp_act_bytes(batch) bytes) receives the activations pp_backward needs. */
bls_status pp_forward(const float* d_theta, const uint16_t* d_x, const double* d_lag, int32_t batch,
                      float* d_logits, void* d_act, bls_stream_t stream);

/* Gradient of the mean softmax cross entropy against soft targets d_target
 * [batch][PP_NCLASS] (rows sum to 1), given the logits and activations of
 * pp_forward on the same inputs.  Scratch: d_gpart [batch][PP_NPARAM] and d_lpart
 * [batch] FP32.  Outputs: d_grad [PP_NPARAM], d_loss [1] (nullable).  The batch
 * mean is taken in batch order, so results are deterministic. */
bls_status pp_backward(const float* d_theta, const uint16_t* d_x, const double* d_lag, const float* d_target,
                       const float* d_logits, const void* d_act, int32_t batch, float* d_gpart, float* d_lpart,
                       float* d_grad, float* d_loss, bls_stream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step >= 1) on
 * the FP32 master weights d_theta with moments d_m, d_v (zero before step 1). */
bls_status pp_adam(float* d_theta, float* d_m, float* d_v, const float* d_grad, int32_t step, float lr,
                   bls_stream_t stream);

/* Proposal for every star of a plan from its logits [n_stars][PP_NCLASS]: the topk
 * most probable period bins (ties to the lower bin), each widened by one bin on
 * both sides; confidence c = P(null) + probability of the selected bins.  If c >=
 * conf: the maximal runs of selected bins and, when Pmax > 100 d, [100 d, Pmax],
 * clipped to [Pmin, Pmax] and mapped to frequency-index ranges of the plan's grid
 * (i from ceil((cbrt(1/P_hi) - u_min)/A) to floor((cbrt(1/P_lo) - u_min)/A)).
 * Else the full grid and d_fallback[s] = 1.
 * Outputs (device, caller-owned):
 *   d_windows [n_stars][PP_MAX_WINDOWS][3] int64 (star, i_begin, i_end) triples,
 *             unused rows star = -1 (input of pp_snr_windows);
 *   d_fallback [n_stars] uint8;  d_conf [n_stars] FP32 (nullable) gets c;
 *   d_tiles (nullable) [pp_tile_capacity][3] int64: the same windows cut into the
 *             plan's work-item size (star s owns a fixed slot range, unused slots
 *             star = -1), the work list to pass to bls_search_batch with
 *             n_windows = pp_tile_capacity, so long windows and fallback grids are
 *             shared by many workgroups.
 * 1 <= topk <= PP_MAX_WINDOWS - 2. */
bls_status pp_propose(const bls_plan* plan, void* d_workspace, const float* d_logits, int32_t topk, float conf,
                      int64_t* d_windows, uint8_t* d_fallback, float* d_conf, int64_t* d_tiles,
                      bls_stream_t stream);

/* pp_propose guided by a coarse search: for a star that does not fall back, the
 * windows also cover the n_peaks largest values of d_coarse_snr (the S/N spectrum of
 * plan `coarse`, from bls_snr: the same stars on the same u = f^(1/3) grid origin
 * with fewer samples per peak), each chosen more than halfwidth coarse steps from
 * every larger one (ties to the lower index) and widened by halfwidth coarse steps
 * on both sides: fine indices from ceil((u_c(i - h) - u_min) / A) to
 * floor((u_c(i + h) - u_min) / A).  All windows of a star are merged into sorted
 * disjoint ranges.  search_long = 0 drops pp_propose's [100 d, Pmax] window (periods
 * the network cannot see): the coarse peaks cover every period of the grid.  topk
 * may be 0 (then c = P(null) and only the coarse peaks, with the long-period window
 * if search_long, are searched).  topk + 1 + n_peaks <= PP_MAX_WINDOWS.
 * Outputs as pp_propose.  Both plans must be uploaded to their workspaces. */
bls_status pp_propose_guided(const bls_plan* plan, void* d_workspace, const float* d_logits, int32_t topk,
                             float conf, int32_t search_long, const bls_plan* coarse, void* coarse_workspace, const double* d_coarse_snr,
                             int32_t n_peaks, int32_t halfwidth, int64_t* d_windows, uint8_t* d_fallback,
                             float* d_conf, int64_t* d_tiles, bls_stream_t stream);

/* Rows of the tiled work list of pp_propose for a plan. */
bls_status pp_tile_capacity(const bls_plan* plan, int64_t* n);

/* S/N of a windowed search.  For a star with d_fallback[s] = 0: trend and sigma of
 * Sec. 2.2 item 1 come from the SR spectrum d_coarse_sr of plan `coarse` (the same
 * stars on a grid with fewer samples per peak, searched in full), and S/N =
 * (SR - trend(f)) / sigma is evaluated at the fine frequencies inside the star's
 * window triples (rows s*windows_per_star .. +windows_per_star of d_windows);
 * the result names the best of those (status 2 if the windows hold no
 * frequency).  For d_fallback[s] = 1 the result is the plain S/N of the star's full
 * fine spectrum (as bls_snr).  Both plans must be uploaded to their workspaces. */
bls_status pp_snr_windows(const bls_plan* fine, void* fine_workspace, const double* d_sr, const bls_best* d_best,
                          const bls_plan* coarse, void* coarse_workspace, const double* d_coarse_sr,
                          const int64_t* d_windows, int32_t windows_per_star, const uint8_t* d_fallback,
                          bls_result* d_result, bls_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* MI355PP_H */
