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
//    cancel.  Integer sums are exact, so the result does not depend on order.
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
  const double ph = p - floor(p);
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
// One workgroup per work item (a frequency range of one star).  LDS holds, per
// frequency of the current group, nb_cap (W, S) slots: int64 G sums during the
// fold, then the FP64 bin totals H during the scan.
// ----------------------------------------------------------------------------
struct SearchArgs {
  const StarDesc* stars;
  const StarRt* rt;
  const WorkItem* items;
  const double* dt;
  const int64_t* cw;
  const int64_t* cs;
  const int64_t* windows;  // optional (star, i0, i1) triples replacing items
  double* sr;
  bls_best* best;
  Consts c;
};

struct ScanBest {
  double p2;
  int32_t m, j;
};

__device__ __forceinline__ bool better(double p2, int32_t m, int32_t j, double q2, int32_t qm, int32_t qj) {
  return p2 > q2 || (p2 == q2 && (m < qm || (m == qm && j < qj)));
}

constexpr double kW62 = 2.168404344971008868e-19;  // 2^-62

__global__ void __launch_bounds__(kThreads) k_search(SearchArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* G = reinterpret_cast<unsigned long long*>(smem);
  double* H = reinterpret_cast<double*>(smem);
  double* s_f = reinterpret_cast<double*>(smem + kGBytes);
  int32_t* s_nb = reinterpret_cast<int32_t*>(s_f + kFMax);
  int32_t* s_blast = s_nb + kFMax;
  long long* s_g0 = reinterpret_cast<long long*>(s_blast + kFMax);  // [kFMax][2]
  ScanBest* s_res = reinterpret_cast<ScanBest*>(s_g0 + 2 * kFMax);   // [kFMax][16]

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
  const int F_act = min(kFMax, (kGBytes / 16) / nb_cap);

  // Points: thread t owns a contiguous run of `run` points per chunk.
  const int T = blockDim.x;
  const int run = static_cast<int>(min<int64_t>(kUMax, (n + T - 1) / T));
  const int64_t chunk_pts = static_cast<int64_t>(run) * T;
  const int nchunks = static_cast<int>((n + chunk_pts - 1) / chunk_pts);
  double dtr[kUMax];
  long long cwr[kUMax], csr[kUMax];
  double dtp = 0.0;
  int len = 0;
  bool has_prev = false;
  auto load_chunk = [&](int c) {
    const int64_t s = static_cast<int64_t>(c) * chunk_pts + static_cast<int64_t>(tid) * run;
    const int64_t rem = n - s;
    len = rem <= 0 ? 0 : static_cast<int>(min<int64_t>(run, rem));
    has_prev = (s > 0) && (len > 0);
    dtp = has_prev ? dt[s - 1] : 0.0;
#pragma unroll
    for (int u = 0; u < kUMax; ++u) {
      if (u < len) {
        dtr[u] = dt[s + u];
        cwr[u] = cw[s + u];
        csr[u] = cs[s + u];
      }
    }
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
      s_blast[tid] = fold_bin(dt_last, f, static_cast<double>(nb), nb - 1);
    }
    for (int idx = tid; idx < F * nb_cap * 2; idx += T) G[idx] = 0ull;
    __syncthreads();

    // ---- fold: boundaries add the prefix values into G ----
    for (int c = 0; c < nchunks; ++c) {
      if (nchunks > 1) load_chunk(c);
      for (int k = 0; k < F; ++k) {
        const double f = s_f[k];
        const int32_t nb = s_nb[k];
        const double nbd = static_cast<double>(nb);
        const int32_t nbm1 = nb - 1;
        unsigned long long* Gk = G + static_cast<size_t>(k) * nb_cap * 2;
        int32_t bprev = has_prev ? fold_bin(dtp, f, nbd, nbm1) : -1;
#pragma unroll
        for (int u = 0; u < kUMax; ++u) {
          if (u < len) {
            const int32_t b = fold_bin(dtr[u], f, nbd, nbm1);
            if (b != bprev) {
              if (bprev >= 0) {
                const unsigned long long ew = static_cast<unsigned long long>(cwr[u]);
                const unsigned long long es = static_cast<unsigned long long>(csr[u]);
                atomicAdd(&Gk[2 * b], ew);
                atomicAdd(&Gk[2 * b + 1], es);
                int32_t steps = b - bprev;
                if (steps < 0) steps += nb;
                int32_t beta = b;
                for (int32_t q = 1; q < steps; ++q) {
                  beta = beta == 0 ? nbm1 : beta - 1;
                  atomicAdd(&Gk[2 * beta], ew);
                  atomicAdd(&Gk[2 * beta + 1], es);
                }
              }
              bprev = b;
            }
          }
        }
      }
    }
    __syncthreads();

    // ---- G -> H (in place, chunked), with the wrap slot saved first ----
    if (tid < F) {
      s_g0[2 * tid] = static_cast<long long>(G[static_cast<size_t>(tid) * nb_cap * 2]);
      s_g0[2 * tid + 1] = static_cast<long long>(G[static_cast<size_t>(tid) * nb_cap * 2 + 1]);
    }
    __syncthreads();
    const int total = F * nb_cap;
    for (int base = 0; base < total; base += T) {
      const int idx = base + tid;
      bool act = false;
      double hw = 0.0, hs = 0.0;
      int k = 0, b = 0;
      if (idx < total) {
        k = idx / nb_cap;
        b = idx - k * nb_cap;
        const int32_t nb = s_nb[k];
        if (b < nb) {
          act = true;
          const unsigned long long* Gk = G + static_cast<size_t>(k) * nb_cap * 2;
          const long long w0 = static_cast<long long>(Gk[2 * b]);
          const long long s0 = static_cast<long long>(Gk[2 * b + 1]);
          long long w1, s1;
          if (b + 1 < nb) {
            w1 = static_cast<long long>(Gk[2 * b + 2]);
            s1 = static_cast<long long>(Gk[2 * b + 3]);
          } else {
            w1 = s_g0[2 * k];
            s1 = s_g0[2 * k + 1];
          }
          long long dw = static_cast<long long>(static_cast<unsigned long long>(w1) - static_cast<unsigned long long>(w0));
          long long ds = static_cast<long long>(static_cast<unsigned long long>(s1) - static_cast<unsigned long long>(s0));
          if (b == s_blast[k]) {
            dw = static_cast<long long>(static_cast<unsigned long long>(dw) + static_cast<unsigned long long>(rt.cw_total));
            ds = static_cast<long long>(static_cast<unsigned long long>(ds) + static_cast<unsigned long long>(rt.cs_total));
          }
          hw = static_cast<double>(dw) * kW62;
          hs = static_cast<double>(ds) * rt.s_scale;
        }
      }
      __syncthreads();
      if (act) {
        double* Hk = H + static_cast<size_t>(k) * nb_cap * 2;
        Hk[2 * b] = hw;
        Hk[2 * b + 1] = hs;
      }
      __syncthreads();
    }

    // ---- scan: every start bin j, durations m of the ladder ----
    const int wpk = F <= waves ? waves / F : 1;   // waves per frequency
    const int kstep = waves / wpk;
    const int m_max = a.c.m_max;
    const uint32_t m_mask = a.c.m_mask;
    const bool dip = a.c.dip_only != 0;
    for (int k = wave / wpk; k < F; k += kstep) {
      const int sub = wave - (wave / wpk) * wpk;
      const int32_t nb = s_nb[k];
      const double* Hk = H + static_cast<size_t>(k) * nb_cap * 2;
      double bp = -1.0, tp = -1.0;
      int32_t bm = 0, bj = -1;
      const int mlim = min(m_max, nb - 1);
      for (int j = sub * 64 + lane; j < nb; j += wpk * 64) {
        double r = 0.0, s = 0.0;
        int idx = j;
        for (int m = 1; m <= mlim; ++m) {
          const double2 h = *reinterpret_cast<const double2*>(Hk + 2 * idx);
          r += h.x;
          s += h.y;
          idx = idx + 1 == nb ? 0 : idx + 1;
          if (m_mask & (1u << (m - 1))) {
            const double da = fma(-r, r, r);
            const double ss = s * s;
            if (fma(-tp, da, ss) > 0.0) {
              if (r > 0.0 && r < 1.0 && (!dip || s < 0.0)) {
                const double p2 = (s * s) / (r * (1.0 - r));
                if (better(p2, m, j, bp, bm, bj)) {
                  bp = p2;
                  bm = m;
                  bj = j;
                  tp = bp > 0.0 ? bp * (1.0 - 0x1.0p-40) : -1.0;
                }
              }
            }
          }
        }
      }
      // wave reduction of (p2, m, j)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double q2 = __shfl_xor(bp, o, 64);
        const int32_t qm = __shfl_xor(bm, o, 64);
        const int32_t qj = __shfl_xor(bj, o, 64);
        if (better(q2, qm, qj, bp, bm, bj)) {
          bp = q2;
          bm = qm;
          bj = qj;
        }
      }
      if (lane == 0) s_res[k * 16 + sub] = ScanBest{bp, bm, bj};
    }
    __syncthreads();
    if (tid < F) {
      const int k = tid;
      ScanBest bsel = s_res[k * 16];
      for (int q = 1; q < wpk; ++q) {
        const ScanBest o = s_res[k * 16 + q];
        if (better(o.p2, o.m, o.j, bsel.p2, bsel.m, bsel.j)) bsel = o;
      }
      const int64_t fi = d.f_off + g0 + k;
      bls_best bb;
      if (bsel.p2 >= 0.0 && bsel.j >= 0) {
        const int32_t nb = s_nb[k];
        const double* Hk = H + static_cast<size_t>(k) * nb_cap * 2;
        double r = 0.0, s = 0.0;
        int idx = bsel.j;
        for (int m = 1; m <= bsel.m; ++m) {
          r += Hk[2 * idx];
          s += Hk[2 * idx + 1];
          idx = idx + 1 == nb ? 0 : idx + 1;
        }
        a.sr[fi] = sqrt(bsel.p2);
        bb.m = bsel.m;
        bb.j = bsel.j;
        bb.r = r;
        bb.s = s;
      } else {
        a.sr[fi] = 0.0;
        bb.m = 0;
        bb.j = -1;
        bb.r = 0.0;
        bb.s = 0.0;
      }
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
  a.windows = d_windows;
  a.sr = d_sr;
  a.best = d_best;
  a.c = plan->consts;
  const int64_t n_items = d_windows ? n_windows : static_cast<int64_t>(plan->items.size());
  if (n_items == 0) return BLS_OK;
  const size_t lds = kGBytes + kFMax * (8 + 4 + 4 + 16) + kFMax * 16 * sizeof(ScanBest);
  hipLaunchKernelGGL(k_search, dim3(static_cast<unsigned>(n_items)), dim3(kThreads), lds, st, a);
  if (hipGetLastError() != hipSuccess) return BLS_E_HIP;
  return BLS_OK;
}
