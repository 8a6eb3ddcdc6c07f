// fit.hip — the post-BLS statistics of QLP Data Release Notes 003, Sec. 2.2 items
// 2-4, and the complete detection criteria of the paragraph after that list:
//   * a trapezoid fitted to the detection (period fixed to the detection's;
//     mid-transit time T0, depth, q = duration / P, q_in = ingress / duration and
//     the out-of-transit level z fitted to the points within two durations of
//     mid-transit; q in [1e-6, 1], q_in in [0, 0.5]) by Levenberg-Marquardt;
//   * white noise sigma_w (standard deviation of the residuals about the model) and
//     red noise sigma_r on the time scale of the duration (bins of one duration:
//     sigma_r^2 = max(0, sigma_D^2 - sigma_w^2 / n_bar), sigma_D the scatter of the
//     bins' mean residuals, n_bar the points per bin);
//   * S/N_pink = delta' / sqrt(sigma_w^2 / n_t + sigma_r^2 / N_t) (Eq. 2) with delta'
//     the trapezoid's depth integral over the duration divided by the duration,
//     delta (1 - q_in);
//   * candidate: N_t >= 2, S/N_pink and S/N above their thresholds (9 and 9).
// Model: with dt the time from the nearest mid-transit, D = q P, tau = q_in D:
// flux = z - delta s, s = 1 for |dt| <= D/2 - tau, (D/2 - |dt|) / tau on the ramps,
// 0 beyond D/2.  Levenberg-Marquardt: A = J^T W J, g = J^T W r, (A + lambda diag A) d
// = g (a parameter whose column is zero is held), clamp to the bounds, keep the step
// if chi^2 falls (lambda / 10, floor 1e-12) else lambda x 10; stop on a kept step that
// lowers chi^2 by at most 1e-10 of it, lambda above 1e10, or 60 iterations.  Start:
// the BLS mid-time, depth and duration, q_in = 0.2, z = the weighted mean of the fit
// points outside the starting box.
//
// One workgroup per star (256 or 512 threads, see below).  The times are sorted, so the points within two
// starting durations of a mid-transit form one index range per transit epoch: the
// ranges (found by binary search with a small margin; the exact test is still made
// per point) are kept in LDS and the fit's passes walk only them, spread evenly over
// the threads (stars with more epochs than LDS holds, or durations of a quarter
// period or more, walk every point).  The fit's sums (15 of A, 5 of g, chi^2) are
// per-thread partial sums over that walk, combined in a fixed order, so results are
// deterministic; the noise and transit passes walk
// contiguous chunks of the time-ordered points, one per thread, and merge the bins
// and transits that straddle chunk ends in thread order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "plan.hpp"

namespace mi355bls {

namespace {

// Workgroup shapes: 256 threads and ranges of up to 1024 epochs when every star of
// the batch is short (several stars share a CU), else 512 threads and 4096 epochs
// (one long star per CU, more waves on its fit).
constexpr int64_t kFitSmallMaxPoints = 65536;
constexpr int kNPar = 5;
constexpr int kNSum = 21;  // 15 (A, upper triangle) + 5 (g) + chi^2
constexpr double kQMin = 1e-6, kQMax = 1.0, kQinMax = 0.5, kQin0 = 0.2;
constexpr double kLambda0 = 1e-3, kRelTol = 1e-10;
constexpr int kMaxIter = 60;

template <int NT, int NE>  // threads, transit epochs whose fit-point ranges LDS holds
struct FitLds {
  static constexpr int kThreads = NT, kWaves = NT / 64, kEpochs = NE, kEpochsPerThread = NE / NT;
  int32_t elo[NE];       // first point of each epoch's fit range
  int32_t ecum[NE + 1];  // fit-range points before each epoch (exclusive prefix)
  int32_t ewave[NT / 64];
  double part[NT / 64][kNSum];
  double sum[kNSum];
  double th[kNPar], th2[kNPar];
  int go, accept;
  // noise and transit passes: one record per thread
  int64_t hb[NT], tb[NT];        // head / tail bin ids (-1: empty chunk)
  double hs[NT], ts[NT];
  int64_t hc[NT], tc[NT];
  int single[NT];
  double wn[NT], wm[NT], wq[NT];  // interior bins: count, mean, M2
  double rn[NT], rm[NT], rq[NT];  // residuals: count, mean, M2
  int64_t ef[NT], el[NT], ec[NT], nt[NT];
};

__device__ __forceinline__ double time_from_mid(double t, double T0, double P) {
  const double x = (t - T0) / P;
  return (x - floor(x + 0.5)) * P;
}

// s and the model's derivatives d/d(T0, delta, q, q_in, z).
__device__ __forceinline__ double model_jac(double t, double P, const double* th, double* J) {
  const double T0 = th[0], delta = th[1], q = th[2], qin = th[3], z = th[4];
  const double D = q * P;
  const double tau = qin * D;
  const double dt = time_from_mid(t, T0, P);
  const double a = fabs(dt);
  const double half = 0.5 * D;
  double s = 0.0;
  J[0] = J[2] = J[3] = 0.0;
  if (a <= half - tau) {
    s = 1.0;
  } else if (a < half && tau > 0.0) {
    s = (half - a) / tau;
    const double sg = dt > 0.0 ? 1.0 : (dt < 0.0 ? -1.0 : 0.0);
    const double ds_da = -1.0 / tau;
    const double ds_dD = 0.5 / tau - (half - a) * qin / (tau * tau);
    const double ds_dqin = -(half - a) * D / (tau * tau);
    J[0] = -delta * ds_da * (-sg);
    J[2] = -delta * ds_dD * P;
    J[3] = -delta * ds_dqin;
  }
  J[1] = -s;
  J[4] = 1.0;
  return z - delta * s;
}

__device__ __forceinline__ double model_only(double t, double P, const double* th) {
  const double D = th[2] * P;
  const double tau = th[3] * D;
  const double a = fabs(time_from_mid(t, th[0], P));
  const double half = 0.5 * D;
  double s = 0.0;
  if (a <= half - tau)
    s = 1.0;
  else if (a < half && tau > 0.0)
    s = (half - a) / tau;
  return th[4] - th[1] * s;
}

// Sum of v[0..nv) over the workgroup into L.sum (fixed order: lanes by shuffles,
// then waves in order).
template <class LDS>
__device__ void block_sums(double* v, int nv, LDS& L) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = 0; i < nv; ++i) {
    double x = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) L.part[wave][i] = x;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double x = 0.0;
    for (int w = 0; w < LDS::kWaves; ++w) x += L.part[w][threadIdx.x];
    L.sum[threadIdx.x] = x;
  }
  __syncthreads();
}

__device__ bool cholesky_solve(const double (&A)[kNPar][kNPar], const double (&g)[kNPar], double (&x)[kNPar]) {
  double Lm[kNPar][kNPar] = {};
  for (int i = 0; i < kNPar; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = 0; k < j; ++k) s += Lm[i][k] * Lm[j][k];
      const double v = A[i][j] - s;
      if (i == j) {
        if (!(v > 0.0)) return false;
        Lm[i][i] = sqrt(v);
      } else {
        Lm[i][j] = v / Lm[j][j];
      }
    }
  double yv[kNPar];
  for (int i = 0; i < kNPar; ++i) {
    double s = 0.0;
    for (int k = 0; k < i; ++k) s += Lm[i][k] * yv[k];
    yv[i] = (g[i] - s) / Lm[i][i];
  }
  for (int i = kNPar - 1; i >= 0; --i) {
    double s = 0.0;
    for (int k = i + 1; k < kNPar; ++k) s += Lm[k][i] * x[k];
    x[i] = (yv[i] - s) / Lm[i][i];
  }
  return true;
}

__device__ __forceinline__ void clamp_th(double* th) {
  th[2] = fmin(fmax(th[2], kQMin), kQMax);
  th[3] = fmin(fmax(th[3], 0.0), kQinMax);
}

// Chan et al. merge of (count, mean, M2) summaries.
__device__ __forceinline__ void chan_merge(double& n, double& m, double& q, double n2, double m2, double q2) {
  if (n2 == 0.0) return;
  if (n == 0.0) {
    n = n2;
    m = m2;
    q = q2;
    return;
  }
  const double nn = n + n2;
  const double d = m2 - m;
  m += d * (n2 / nn);
  q += q2 + d * d * (n * n2 / nn);
  n = nn;
}

}  // namespace

template <int NT, int NE>
__global__ void __launch_bounds__(NT) k_fit(const StarDesc* __restrict__ stars, const double* __restrict__ t,
                                                     const double* __restrict__ y, const double* __restrict__ w,
                                                     const bls_result* __restrict__ res, double snr_min,
                                                     double pink_min, bls_fit_result* __restrict__ out) {
  using LDS = FitLds<NT, NE>;
  constexpr int kFitThreads = NT, kFitWaves = NT / 64, kFitEpochs = NE, kEpochsPerThread = LDS::kEpochsPerThread;
  __shared__ LDS L;
  const int tid = threadIdx.x;
  const StarDesc d = stars[blockIdx.x];
  const int64_t n = d.n, off = d.p_off;
  const bls_result r = res[blockIdx.x];
  bls_fit_result o;
  o.t0 = o.depth = o.q = o.q_in = o.level = o.chi2 = NAN;
  o.sigma_w = o.sigma_r = o.depth_eff = o.snr_pink = NAN;
  o.n_fit = o.n_t = o.n_transits = 0;
  o.iterations = 0;
  o.candidate = 0;
  o.status = 1;
  o.pad = 0;
  const double P = r.period, T0b = r.t0, depthb = r.depth;
  const double qb = r.duration / P;
  if (!(P > 0.0) || !isfinite(T0b) || !isfinite(depthb) || !(qb > 0.0) || !isfinite(qb)) {
    if (tid == 0) out[blockIdx.x] = o;
    return;
  }
  const double D0 = qb * P;
  // ---- fit-point ranges, one per transit epoch (windows of half-width 2 D0 < P/4
  // apart by more than their width, so no point is in two)
  const double half = 2.0 * D0;
  const double t_lo = t[off], t_hi = t[off + n - 1];
  const int64_t ep0 = static_cast<int64_t>(floor((t_lo - T0b) / P + 0.5)) - 1;
  const int64_t ep1 = static_cast<int64_t>(floor((t_hi - T0b) / P + 0.5)) + 1;
  const int64_t n_ep = ep1 - ep0 + 1;
  const bool ranged = half < 0.25 * P && n_ep >= 1 && n_ep <= kFitEpochs && n < (int64_t(1) << 31);
  if (ranged) {
    const double margin = 1e-6;  // days; the per-point test decides
    int32_t cnt[kEpochsPerThread];
    int32_t mine = 0;
    for (int k = 0; k < kEpochsPerThread; ++k) {
      const int64_t e = static_cast<int64_t>(tid) * kEpochsPerThread + k;
      cnt[k] = 0;
      if (e >= n_ep) continue;
      const double c = T0b + static_cast<double>(ep0 + e) * P;
      const double a = c - half - margin, b = c + half + margin;
      int64_t lo = 0, hi = n;  // first index with t >= a
      while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (t[off + m] < a) lo = m + 1; else hi = m;
      }
      int64_t lo2 = lo, hi2 = n;  // first index with t > b
      while (lo2 < hi2) {
        const int64_t m = (lo2 + hi2) >> 1;
        if (t[off + m] <= b) lo2 = m + 1; else hi2 = m;
      }
      L.elo[e] = static_cast<int32_t>(lo);
      cnt[k] = static_cast<int32_t>(lo2 - lo);
      mine += cnt[k];
    }
    // exclusive prefix of the per-thread totals (waves by shuffles, then the waves)
    const int lane = tid & 63, wave = tid >> 6;
    int32_t incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t yv = __shfl_up(incl, o, 64);
      if (lane >= o) incl += yv;
    }
    if (lane == 63) L.ewave[wave] = incl;
    __syncthreads();
    int32_t before = 0;
    for (int v = 0; v < wave; ++v) before += L.ewave[v];
    int32_t acc = before + incl - mine;
    for (int k = 0; k < kEpochsPerThread; ++k) {
      const int64_t e = static_cast<int64_t>(tid) * kEpochsPerThread + k;
      if (e < n_ep) L.ecum[e] = acc;
      acc += cnt[k];
    }
    if (tid == kFitThreads - 1) L.ecum[n_ep] = acc;
    __syncthreads();
  }
  // Calls body(i) for the star's candidate fit points, i in a fixed per-thread order.
  auto for_fit = [&](auto&& body) {
    if (!ranged) {
      for (int64_t i = tid; i < n; i += kFitThreads) body(i);
      return;
    }
    const int32_t total = L.ecum[n_ep];
    int64_t e = 0;
    for (int32_t j = tid; j < total; j += kFitThreads) {
      while (L.ecum[e + 1] <= j) ++e;
      body(static_cast<int64_t>(L.elo[e]) + (j - L.ecum[e]));
    }
  };
  // ---- starting level: weighted mean of the fit points outside the starting box
  {
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // sum w y, sum w (outside); sum w y, sum w (all); count
    for_fit([&](int64_t i) {
      const double wi = w ? w[off + i] : 1.0;
      if (!(wi > 0.0)) return;
      const double a = fabs(time_from_mid(t[off + i], T0b, P));
      if (!(a <= 2.0 * D0)) return;
      const double yi = y[off + i];
      v[2] += wi * yi;
      v[3] += wi;
      v[4] += 1.0;
      if (a >= 0.5 * D0) {
        v[0] += wi * yi;
        v[1] += wi;
      }
    });
    block_sums(v, 5, L);
  }
  const int64_t nfit = static_cast<int64_t>(L.sum[4]);
  o.n_fit = nfit;
  if (nfit == 0) {
    o.status = 2;
    if (tid == 0) out[blockIdx.x] = o;
    return;
  }
  if (tid == 0) {
    L.th[0] = T0b;
    L.th[1] = depthb;
    L.th[2] = qb;
    L.th[3] = kQin0;
    L.th[4] = L.sum[1] > 0.0 ? L.sum[0] / L.sum[1] : L.sum[2] / L.sum[3];
    clamp_th(L.th);
  }
  __syncthreads();
  // ---- Levenberg-Marquardt
  double chi2 = 0.0, lam = kLambda0;
  int it = 0;
  bool need_normal = true;
  double A[kNPar][kNPar], g[kNPar];  // meaningful on thread 0
  for (;;) {
    if (need_normal) {
      double v[kNSum];
      for (int k = 0; k < kNSum; ++k) v[k] = 0.0;
      double th[kNPar];
      for (int k = 0; k < kNPar; ++k) th[k] = L.th[k];
      for_fit([&](int64_t i) {
        const double wi = w ? w[off + i] : 1.0;
        if (!(wi > 0.0)) return;
        const double ti = t[off + i];
        if (!(fabs(time_from_mid(ti, T0b, P)) <= 2.0 * D0)) return;
        double J[kNPar];
        const double res_i = y[off + i] - model_jac(ti, P, th, J);
        int e = 0;
        for (int a = 0; a < kNPar; ++a)
          for (int b = a; b < kNPar; ++b) v[e++] += wi * J[a] * J[b];
        for (int a = 0; a < kNPar; ++a) v[15 + a] += wi * J[a] * res_i;
        v[20] += wi * res_i * res_i;
      });
      block_sums(v, kNSum, L);
      if (tid == 0) {
        int e = 0;
        for (int a = 0; a < kNPar; ++a)
          for (int b = a; b < kNPar; ++b) {
            A[a][b] = L.sum[e];
            A[b][a] = L.sum[e];
            ++e;
          }
        for (int a = 0; a < kNPar; ++a) g[a] = L.sum[15 + a];
      }
      if (it == 0) chi2 = L.sum[20];  // every thread: the step decisions are uniform
      __syncthreads();
      need_normal = false;
    }
    if (it >= kMaxIter) break;
    ++it;
    // ---- step (thread 0)
    if (tid == 0) {
      double Ad[kNPar][kNPar], gd[kNPar], dx[kNPar];
      for (int a = 0; a < kNPar; ++a) {
        gd[a] = g[a];
        for (int b = 0; b < kNPar; ++b) Ad[a][b] = A[a][b];
      }
      for (int a = 0; a < kNPar; ++a) {
        if (A[a][a] == 0.0) {
          for (int b = 0; b < kNPar; ++b) Ad[a][b] = Ad[b][a] = 0.0;
          Ad[a][a] = 1.0;
          gd[a] = 0.0;
        } else {
          Ad[a][a] = A[a][a] * (1.0 + lam);
        }
      }
      L.go = cholesky_solve(Ad, gd, dx) ? 1 : 0;
      if (L.go) {
        for (int a = 0; a < kNPar; ++a) L.th2[a] = L.th[a] + dx[a];
        clamp_th(L.th2);
      }
    }
    __syncthreads();
    if (!L.go) {
      lam *= 10.0;
      if (lam > 1e10) break;
      continue;
    }
    // ---- chi^2 at the trial point
    {
      double v[1] = {0.0};
      double th2[kNPar];
      for (int k = 0; k < kNPar; ++k) th2[k] = L.th2[k];
      for_fit([&](int64_t i) {
        const double wi = w ? w[off + i] : 1.0;
        if (!(wi > 0.0)) return;
        const double ti = t[off + i];
        if (!(fabs(time_from_mid(ti, T0b, P)) <= 2.0 * D0)) return;
        const double ri = y[off + i] - model_only(ti, P, th2);
        v[0] += wi * ri * ri;
      });
      block_sums(v, 1, L);
    }
    const double chi2b = L.sum[0];
    bool done = false;
    if (chi2b < chi2) {
      done = (chi2 - chi2b) <= kRelTol * chi2;
      chi2 = chi2b;
      lam = fmax(lam / 10.0, 1e-12);
      if (tid == 0)
        for (int a = 0; a < kNPar; ++a) L.th[a] = L.th2[a];
      need_normal = true;
      __syncthreads();
      if (done) break;
    } else {
      lam *= 10.0;
      if (lam > 1e10) break;
    }
  }
  __syncthreads();
  double th[kNPar];
  for (int k = 0; k < kNPar; ++k) th[k] = L.th[k];
  const double D = th[2] * P;
  // ---- noise, transit count: contiguous chunks of the time-ordered points
  {
    const int64_t C = (n + kFitThreads - 1) / kFitThreads;
    const int64_t i0 = static_cast<int64_t>(tid) * C, i1 = i0 + C < n ? i0 + C : n;
    double tfirst = 0.0;
    // first weighted time of the star (the bins' origin)
    {
      int64_t f = n;
      for (int64_t i = tid; i < n; i += kFitThreads) {
        const double wi = w ? w[off + i] : 1.0;
        if (wi > 0.0) {
          f = i;
          break;
        }
      }
      // minimum over threads through the shared sum slots
      const int lane = tid & 63, wave = tid >> 6;
      double x = static_cast<double>(f);
#pragma unroll
      for (int oo = 32; oo > 0; oo >>= 1) x = fmin(x, __shfl_xor(x, oo, 64));
      if (lane == 0) L.part[wave][0] = x;
      __syncthreads();
      if (tid == 0) {
        double mn = L.part[0][0];
        for (int ww = 1; ww < kFitWaves; ++ww) mn = fmin(mn, L.part[ww][0]);
        L.sum[0] = mn;
      }
      __syncthreads();
      tfirst = t[off + static_cast<int64_t>(L.sum[0])];
    }
    int64_t hb = -1, tb = -1, hc = 0, tc = 0, cur = -1, cc = 0;
    double hs = 0.0, tsum = 0.0, cs = 0.0;
    int nopen = 0;  // bins opened in this chunk
    double bn = 0.0, bm = 0.0, bq = 0.0;  // interior bins: Welford of the means
    double rn = 0.0, rm = 0.0, rq = 0.0;  // residuals: Welford
    int64_t ef = INT64_MIN, el = INT64_MIN, ec = 0, ntc = 0;
    for (int64_t i = i0; i < i1; ++i) {
      const double wi = w ? w[off + i] : 1.0;
      if (!(wi > 0.0)) continue;
      const double ti = t[off + i];
      const double ri = y[off + i] - model_only(ti, P, th);
      rn += 1.0;
      const double dr = ri - rm;
      rm += dr / rn;
      rq += dr * (ri - rm);
      const int64_t k = static_cast<int64_t>(floor((ti - tfirst) / D));
      if (nopen == 0) {
        cur = k;
        cs = ri;
        cc = 1;
        nopen = 1;
      } else if (k == cur) {
        cs += ri;
        ++cc;
      } else {
        if (nopen == 1) {  // the chunk's first bin may continue a neighbour's
          hb = cur;
          hs = cs;
          hc = cc;
        } else {
          const double mean = cs / static_cast<double>(cc);
          bn += 1.0;
          const double d1 = mean - bm;
          bm += d1 / bn;
          bq += d1 * (mean - bm);
        }
        cur = k;
        cs = ri;
        cc = 1;
        ++nopen;
      }
      if (fabs(time_from_mid(ti, th[0], P)) < 0.5 * D) {
        ++ntc;
        const int64_t ep = static_cast<int64_t>(floor((ti - th[0]) / P + 0.5));
        if (ef == INT64_MIN) {
          ef = ep;
          ec = 1;
        } else if (ep > el) {
          ++ec;
        }
        el = ep;
      }
    }
    if (nopen == 1) {
      hb = tb = cur;
      hs = tsum = cs;
      hc = tc = cc;
    } else if (nopen > 1) {
      tb = cur;
      tsum = cs;
      tc = cc;
    }
    L.hb[tid] = hb;
    L.tb[tid] = tb;
    L.hs[tid] = hs;
    L.ts[tid] = tsum;
    L.hc[tid] = hc;
    L.tc[tid] = tc;
    L.single[tid] = nopen == 1 ? 1 : 0;
    L.wn[tid] = bn;
    L.wm[tid] = bm;
    L.wq[tid] = bq;
    L.rn[tid] = rn;
    L.rm[tid] = rm;
    L.rq[tid] = rq;
    L.ef[tid] = ef;
    L.el[tid] = el;
    L.ec[tid] = ec;
    L.nt[tid] = ntc;
  }
  __syncthreads();
  if (tid == 0) {
    double bn = 0.0, bm = 0.0, bq = 0.0, rn = 0.0, rm = 0.0, rq = 0.0;
    int64_t cb = -1, ccnt = 0;
    double csum = 0.0;
    auto finish = [&]() {
      if (cb >= 0) {
        chan_merge(bn, bm, bq, 1.0, csum / static_cast<double>(ccnt), 0.0);
        cb = -1;
      }
    };
    int64_t n_t = 0, N_t = 0, last_ep = INT64_MIN;
    for (int q = 0; q < kFitThreads; ++q) {
      chan_merge(rn, rm, rq, L.rn[q], L.rm[q], L.rq[q]);
      n_t += L.nt[q];
      if (L.ec[q] > 0) {
        N_t += L.ec[q] - (L.ef[q] == last_ep ? 1 : 0);
        last_ep = L.el[q];
      }
      if (L.hb[q] < 0) continue;  // no weighted point in this chunk
      if (L.hb[q] == cb) {
        csum += L.hs[q];
        ccnt += L.hc[q];
      } else {
        finish();
        cb = L.hb[q];
        csum = L.hs[q];
        ccnt = L.hc[q];
      }
      if (!L.single[q]) {
        finish();
        chan_merge(bn, bm, bq, L.wn[q], L.wm[q], L.wq[q]);
        cb = L.tb[q];
        csum = L.ts[q];
        ccnt = L.tc[q];
      }
    }
    finish();
    const double sw = rn >= 2.0 ? sqrt(rq / (rn - 1.0)) : 0.0;
    double sr = 0.0;
    if (rn >= 2.0 && bn >= 2.0) {
      const double sD2 = bq / (bn - 1.0);
      const double nbar = rn / bn;
      sr = sqrt(fmax(0.0, sD2 - sw * sw / nbar));
    }
    o.t0 = th[0];
    o.depth = th[1];
    o.q = th[2];
    o.q_in = th[3];
    o.level = th[4];
    o.chi2 = chi2;
    o.sigma_w = sw;
    o.sigma_r = sr;
    o.n_t = n_t;
    o.n_transits = N_t;
    o.depth_eff = th[1] * (1.0 - th[3]);
    const double den = (n_t > 0 && N_t > 0)
                           ? sqrt(sw * sw / static_cast<double>(n_t) + sr * sr / static_cast<double>(N_t))
                           : 0.0;
    o.snr_pink = den > 0.0 ? o.depth_eff / den : ((n_t > 0 && o.depth_eff > 0.0) ? INFINITY : 0.0);
    o.iterations = it;
    o.candidate = (N_t >= 2 && o.snr_pink > pink_min && r.snr > snr_min) ? 1 : 0;
    o.status = 0;
    out[blockIdx.x] = o;
  }
}

}  // namespace mi355bls

using namespace mi355bls;

extern "C" bls_status bls_fit(bls_plan* plan, void* ws, const double* d_t, const double* d_y, const double* d_w,
                              const bls_result* d_result, double snr_min, double pink_min, bls_fit_result* d_fit,
                              bls_stream_t stream) {
  if (!plan || !d_t || !d_y || !d_result || !d_fit) return BLS_E_ARG;
  if (!(snr_min == snr_min) || !(pink_min == pink_min)) return BLS_E_ARG;
  if (!ws || plan->uploaded_to != ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return BLS_E_STATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const StarDesc* sd = reinterpret_cast<const StarDesc*>(static_cast<char*>(ws) + plan->layout.stars);
  int64_t n_max = 0;
  for (const StarDesc& d : plan->stars) n_max = d.n > n_max ? d.n : n_max;
  if (n_max <= kFitSmallMaxPoints)
    hipLaunchKernelGGL((k_fit<256, 1024>), dim3(plan->n_stars), dim3(256), 0, st, sd, d_t, d_y, d_w, d_result,
                       snr_min, pink_min, d_fit);
  else
    hipLaunchKernelGGL((k_fit<512, 4096>), dim3(plan->n_stars), dim3(512), 0, st, sd, d_t, d_y, d_w, d_result,
                       snr_min, pink_min, d_fit);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}
