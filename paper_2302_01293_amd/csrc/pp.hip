// pp.hip — learned period proposal on gfx950: resampling of light curves, a small
// 1-D CNN (BF16 MFMA forward, hand-written FP32 backward, Adam), and the proposal
// of period windows for a restricted BLS search with full-grid fallback.
//
// The paper searches the full Keplerian grid of Sec. 2.1; this network only
// decides where to search first.  Every window it proposes is searched by the
// plain BLS kernels, and a star whose proposal is not confident (null probability
// plus the probability mass inside the windows below a threshold) falls back to
// its full grid, so BLS decides every detection.
//
// Network (per star): input [2, 4096] BF16 (standardised flux, coverage)
//   conv1 2->16, kernel 16, stride 2, padding 7, ReLU           -> [16, 2048] BF16
//   conv2 16->16, kernel 8, stride 2, padding 3, ReLU           -> [16, 1024] BF16
//   1x1 conv to one channel (no bias), mean removed             -> s[1024] FP32
//   autocorrelation A[tau] = sum_t s[t] s[t+tau] / 1024, normalised by A[0] + 1e-6
//   phi_k = A at the lag of period-bin centre k (512 log-spaced bins over
//   [0.5, 100] d; lag = P / (baseline / 1024); 0 outside lags [2, 1023])
//   logits_k = alpha phi_k + beta_k, null logit delta.
// conv1 and conv2 run as implicit GEMMs on v_mfma_f32_16x16x16_bf16 (FP32
// accumulation); the rest is FP32 VALU (head in FP64).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mi355pp.h"
#include "plan.hpp"
#include "select.hpp"

namespace mi355pp {

using mi355bls::StarDesc;

constexpr int kL0 = 4096, kCin = 2;
constexpr int kC1 = 16, kK1 = 16, kP1 = 7, kL1 = 2048;
constexpr int kC2 = 16, kK2 = 8, kP2 = 3, kL2 = 1024;
constexpr int kNpb = 512;
constexpr double kPbLo = 0.5, kPbHi = 100.0;
constexpr double kEps = 1e-6;
// Parameter vector layout (FP32).
constexpr int oW1 = 0, oB1 = oW1 + kC1 * kCin * kK1, oW2 = oB1 + kC1, oB2 = oW2 + kC2 * kC1 * kK2,
              oW3 = oB2 + kC2, oAlpha = oW3 + kC2, oBeta = oAlpha + 1, oDelta = oBeta + kNpb,
              kNParam = oDelta + 1;
static_assert(kNParam == PP_NPARAM, "parameter count");
static_assert(kNpb + 1 == PP_NCLASS, "class count");

// Saved activations of one star (bytes): a1 BF16 [16][2048], a2 BF16 [16][1024],
// s FP32 [1024] (mean removed), A FP32 [1024].
constexpr size_t kActA1 = 0, kActA2 = kActA1 + 2ull * kC1 * kL1, kActS = kActA2 + 2ull * kC2 * kL2,
                 kActA = kActS + 4ull * kL2, kActBytes = kActA + 4ull * kL2;
static_assert(kActBytes == PP_ACT_BYTES_PER_STAR, "activation layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ double period_centre(int k) {
  return kPbLo * pow(kPbHi / kPbLo, (static_cast<double>(k) + 0.5) / kNpb);
}
__device__ __forceinline__ double period_edge(int i) {
  return kPbLo * pow(kPbHi / kPbLo, static_cast<double>(i) / kNpb);
}

template <typename T>
__device__ T block_sum(T v, T* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T r = 0;
  for (int q = 0; q < static_cast<int>(blockDim.x >> 6); ++q) r += scratch[q];
  __syncthreads();
  return r;
}

template <typename T>
__device__ T block_max(T v, T* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  T r = scratch[0];
  for (int q = 1; q < static_cast<int>(blockDim.x >> 6); ++q) r = fmax(r, scratch[q]);
  __syncthreads();
  return r;
}

// ----------------------------------------------------------------------------
// Resample: 4096 uniform bins over [t0, t0 + T] (the weighted baseline of the
// plan).  z = (y - median y) / (1.4826 MAD y) over points with w > 0; channel 0 =
// sum w z / sum w per bin, channel 1 = 1 where the bin holds weight.  Bins are
// contiguous runs of the time-ordered points; each bin is summed in point order.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_resample(const StarDesc* __restrict__ stars, const double* __restrict__ t,
                                                   const double* __restrict__ y, const double* __restrict__ w,
                                                   uint16_t* __restrict__ x_out, double* __restrict__ lag_out) {
  __shared__ mi355bls::SelShared sh;
  __shared__ int32_t start[kL0 + 1];
  __shared__ int64_t cnt_s[16];
  const StarDesc d = stars[blockIdx.x];
  const int tid = threadIdx.x, T = blockDim.x;
  const double* ts = t + d.p_off;
  const double* ys = y + d.p_off;
  const double* ws = w ? w + d.p_off : nullptr;
  const int64_t n = d.n;
  auto wt = [&](int64_t i) { return ws ? ws[i] : 1.0; };
  int64_t good = 0;
  for (int64_t i = tid; i < n; i += T) good += wt(i) > 0.0 ? 1 : 0;
  good = block_sum<int64_t>(good, cnt_s);
  // weightless points sort last (+inf) and are never reached by the ranks
  auto yv = [&](int64_t i) { return wt(i) > 0.0 ? ys[i] : INFINITY; };
  double med;
  if (good & 1) {
    med = mi355bls::block_select(yv, 0, n, good / 2, sh);
  } else {
    const double a = mi355bls::block_select(yv, 0, n, good / 2 - 1, sh);
    const double b = mi355bls::block_select(yv, 0, n, good / 2, sh);
    med = (a + b) * 0.5;
  }
  auto dv = [&](int64_t i) { return wt(i) > 0.0 ? fabs(ys[i] - med) : INFINITY; };
  double mad;
  if (good & 1) {
    mad = mi355bls::block_select(dv, 0, n, good / 2, sh);
  } else {
    const double a = mi355bls::block_select(dv, 0, n, good / 2 - 1, sh);
    const double b = mi355bls::block_select(dv, 0, n, good / 2, sh);
    mad = (a + b) * 0.5;
  }
  const double scale = 1.4826 * mad;
  const double t0 = d.t0, span = d.T;
  auto bin_of = [&](int64_t i) -> int {
    int b = 0;
    if (span > 0.0) {
      const double v = floor(((ts[i] - t0) / span) * static_cast<double>(kL0));
      b = v < 0.0 ? 0 : (v > kL0 - 1 ? kL0 - 1 : static_cast<int>(v));
    }
    return b;
  };
  for (int b = tid; b <= kL0; b += T) start[b] = static_cast<int32_t>(n);
  __syncthreads();
  for (int64_t i = tid; i < n; i += T) {
    const int k = bin_of(i);
    const int kp = i > 0 ? bin_of(i - 1) : -1;
    for (int b = kp + 1; b <= k; ++b) start[b] = static_cast<int32_t>(i);
  }
  __syncthreads();
  uint16_t* xo = x_out + static_cast<int64_t>(blockIdx.x) * 2 * kL0;
  for (int b = tid; b < kL0; b += T) {
    double sw = 0.0, swz = 0.0;
    for (int64_t i = start[b]; i < start[b + 1]; ++i) {
      const double z = scale > 0.0 ? (ys[i] - med) / scale : 0.0;
      sw += wt(i);
      swz += wt(i) * z;
    }
    const bool occ = sw > 0.0;
    xo[b] = occ ? bf16_bits(static_cast<float>(swz / sw)) : static_cast<uint16_t>(0);
    xo[kL0 + b] = occ ? static_cast<uint16_t>(0x3F80) : static_cast<uint16_t>(0);
  }
  if (tid == 0) lag_out[blockIdx.x] = span / kL2;
}

// ----------------------------------------------------------------------------
// Forward.  One workgroup (4 waves) per star.
// MFMA 16x16x16 BF16 lane layout: lane l supplies A[row l%16][k 4(l/16)..+3] and
// B[k 4(l/16)..+3][col l%16], and receives D[row 4(l/16)+r][col l%16], r = 0..3.
// Rows are output channels, columns 16 consecutive output positions, k runs over
// (input channel, tap).
// ----------------------------------------------------------------------------
constexpr int kXPad = 16, kXRow = kL0 + 32;   // x[c][p] at xs[c * kXRow + p + kXPad]
constexpr int kA1Pad = 8, kA1Row = kL1 + 16;  // a1[c][p] at a1s[c * kA1Row + p + kA1Pad]
constexpr size_t kFwdLds = 2ull * kCin * kXRow + 2ull * kC1 * kA1Row + 2ull * kC2 * kL2 + 4ull * kL2 * 2 + 64;

__device__ void head_phi(const float* ac, double lag, int k, double& phi, int& i0, double& fr) {
  const double den = static_cast<double>(ac[0]) + kEps;
  const double tau = period_centre(k) / lag;
  phi = 0.0;
  i0 = -1;
  fr = 0.0;
  if (!(tau >= 2.0) || tau > kL2 - 1) return;
  i0 = static_cast<int>(floor(tau));
  fr = tau - i0;
  if (i0 >= kL2 - 1) {
    i0 = kL2 - 1;
    fr = 0.0;
    phi = static_cast<double>(ac[kL2 - 1]) / den;
    return;
  }
  phi = (1.0 - fr) * (static_cast<double>(ac[i0]) / den) + fr * (static_cast<double>(ac[i0 + 1]) / den);
}

__global__ void __launch_bounds__(256) k_forward(const float* __restrict__ theta, const uint16_t* __restrict__ x,
                                                 const double* __restrict__ lag, float* __restrict__ logits,
                                                 unsigned char* __restrict__ act) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint16_t* xs = reinterpret_cast<uint16_t*>(lds);
  uint16_t* a1s = xs + kCin * kXRow;
  uint16_t* a2s = a1s + kC1 * kA1Row;
  float* ss = reinterpret_cast<float*>(a2s + kC2 * kL2);
  float* ac = ss + kL2;
  float* red = ac + kL2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = blockIdx.x;
  const uint16_t* xb = x + static_cast<int64_t>(b) * kCin * kL0;

  for (int i = tid; i < kCin * kXRow; i += 256) {
    const int c = i / kXRow, p = i - c * kXRow - kXPad;
    xs[i] = (p >= 0 && p < kL0) ? xb[c * kL0 + p] : static_cast<uint16_t>(0);
  }
  for (int i = tid; i < kC1 * kA1Row; i += 256) a1s[i] = 0;
  __syncthreads();

  const int n = lane & 15, kb = lane >> 4;
  // ---- conv1: K = 2 channels x 16 taps = 2 MFMA k-steps
  {
    bf16x4 wa[2];
    for (int ks = 0; ks < 2; ++ks)
      for (int i = 0; i < 4; ++i)
        wa[ks][i] = static_cast<short>(bf16_bits(theta[oW1 + (n * kCin + ks) * kK1 + 4 * kb + i]));
    float bias[4];
    for (int r = 0; r < 4; ++r) bias[r] = theta[oB1 + 4 * kb + r];
    for (int tile = wave; tile < kL1 / 16; tile += 4) {
      const int l0 = tile * 16;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < 2; ++ks) {
        bf16x4 bv;
        const int base = ks * kXRow + 2 * (l0 + n) + 4 * kb - kP1 + kXPad;
        for (int i = 0; i < 4; ++i) bv[i] = static_cast<short>(xs[base + i]);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[ks], bv, acc, 0, 0, 0);
      }
      for (int r = 0; r < 4; ++r) {
        const int o = 4 * kb + r;
        const float v = fmaxf(acc[r] + bias[r], 0.0f);
        a1s[o * kA1Row + l0 + n + kA1Pad] = bf16_bits(v);
      }
    }
  }
  __syncthreads();
  // ---- conv2: K = 16 channels x 8 taps = 8 MFMA k-steps
  {
    bf16x4 wa[8];
    for (int ks = 0; ks < 8; ++ks)
      for (int i = 0; i < 4; ++i) {
        const int kk = 16 * ks + 4 * kb + i, c = kk >> 3, k = kk & 7;
        wa[ks][i] = static_cast<short>(bf16_bits(theta[oW2 + (n * kC1 + c) * kK2 + k]));
      }
    float bias[4];
    for (int r = 0; r < 4; ++r) bias[r] = theta[oB2 + 4 * kb + r];
    for (int tile = wave; tile < kL2 / 16; tile += 4) {
      const int l0 = tile * 16;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < 8; ++ks) {
        bf16x4 bv;
        for (int i = 0; i < 4; ++i) {
          const int kk = 16 * ks + 4 * kb + i, c = kk >> 3, k = kk & 7;
          bv[i] = static_cast<short>(a1s[c * kA1Row + 2 * (l0 + n) + k - kP2 + kA1Pad]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[ks], bv, acc, 0, 0, 0);
      }
      for (int r = 0; r < 4; ++r) {
        const int o = 4 * kb + r;
        a2s[o * kL2 + l0 + n] = bf16_bits(fmaxf(acc[r] + bias[r], 0.0f));
      }
    }
  }
  __syncthreads();
  // ---- 1x1 conv, mean removal
  float part = 0.f;
  for (int l = tid; l < kL2; l += 256) {
    float v = 0.f;
    for (int c = 0; c < kC2; ++c) v += theta[oW3 + c] * bf16_val(a2s[c * kL2 + l]);
    ss[l] = v;
    part += v;
  }
  const float mean = block_sum<float>(part, red) / kL2;
  for (int l = tid; l < kL2; l += 256) ss[l] -= mean;
  __syncthreads();
  // ---- autocorrelation
  for (int tau = tid; tau < kL2; tau += 256) {
    float v = 0.f;
    for (int t0 = 0; t0 + tau < kL2; ++t0) v += ss[t0] * ss[t0 + tau];
    ac[tau] = v / kL2;
  }
  __syncthreads();
  // ---- head (FP64)
  const double lg = lag[b];
  const double alpha = theta[oAlpha];
  float* lo = logits + static_cast<int64_t>(b) * (kNpb + 1);
  for (int k = tid; k < kNpb; k += 256) {
    double phi, fr;
    int i0;
    head_phi(ac, lg, k, phi, i0, fr);
    lo[k] = static_cast<float>(alpha * phi + static_cast<double>(theta[oBeta + k]));
  }
  if (tid == 0) lo[kNpb] = theta[oDelta];
  if (act) {
    unsigned char* ab = act + static_cast<size_t>(b) * kActBytes;
    uint16_t* ga1 = reinterpret_cast<uint16_t*>(ab + kActA1);
    uint16_t* ga2 = reinterpret_cast<uint16_t*>(ab + kActA2);
    float* gs = reinterpret_cast<float*>(ab + kActS);
    float* ga = reinterpret_cast<float*>(ab + kActA);
    for (int i = tid; i < kC1 * kL1; i += 256) {
      const int c = i / kL1, p = i - c * kL1;
      ga1[i] = a1s[c * kA1Row + p + kA1Pad];
    }
    for (int i = tid; i < kC2 * kL2; i += 256) ga2[i] = a2s[i];
    for (int i = tid; i < kL2; i += 256) {
      gs[i] = ss[i];
      ga[i] = ac[i];
    }
  }
}

// ----------------------------------------------------------------------------
// Backward of the mean softmax cross entropy, one workgroup per star; writes the
// star's gradient (not yet divided by the batch size) and loss.
// ----------------------------------------------------------------------------
constexpr size_t kBwdLds = 2ull * kC1 * kL1 + 4ull * kC2 * kL2 + 4ull * kL2 * 4 + 4ull * kNpb * 3 + 256;

__global__ void __launch_bounds__(256) k_backward(const float* __restrict__ theta, const uint16_t* __restrict__ x,
                                                  const double* __restrict__ lag, const float* __restrict__ target,
                                                  const float* __restrict__ logits,
                                                  const unsigned char* __restrict__ act, float* __restrict__ gpart,
                                                  float* __restrict__ lpart) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint16_t* a1s = reinterpret_cast<uint16_t*>(lds);                   // [16][2048]
  float* dz2 = reinterpret_cast<float*>(a1s + kC1 * kL1);             // [16][1024]
  float* ss = dz2 + kC2 * kL2;                                          // s (mean removed)
  float* ac = ss + kL2;                                                 // A, later ds
  float* dA = ac + kL2;                                                 // dAhat, then dA
  float* dz1 = dA + kL2;                                                // dz1 chunk [16][64]
  float* dphi = dz1 + kL2;                                              // [512]
  int32_t* bi0 = reinterpret_cast<int32_t*>(dphi + kNpb);               // [512]
  float* bfr = reinterpret_cast<float*>(bi0 + kNpb);                    // [512]
  double* red = reinterpret_cast<double*>(bfr + kNpb);                  // [8]
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const unsigned char* ab = act + static_cast<size_t>(b) * kActBytes;
  const uint16_t* ga1 = reinterpret_cast<const uint16_t*>(ab + kActA1);
  const uint16_t* ga2 = reinterpret_cast<const uint16_t*>(ab + kActA2);
  const float* gs = reinterpret_cast<const float*>(ab + kActS);
  const float* gac = reinterpret_cast<const float*>(ab + kActA);
  const uint16_t* xb = x + static_cast<int64_t>(b) * kCin * kL0;
  float* gp = gpart + static_cast<int64_t>(b) * kNParam;
  for (int i = tid; i < kC1 * kL1; i += 256) a1s[i] = ga1[i];
  for (int i = tid; i < kL2; i += 256) {
    ss[i] = gs[i];
    ac[i] = gac[i];
  }
  __syncthreads();

  // ---- softmax cross entropy (FP64)
  const float* zl = logits + static_cast<int64_t>(b) * (kNpb + 1);
  const float* q = target + static_cast<int64_t>(b) * (kNpb + 1);
  double zmax = -INFINITY;
  for (int k = tid; k <= kNpb; k += 256) zmax = fmax(zmax, static_cast<double>(zl[k]));
  zmax = block_max<double>(zmax, red);
  double se = 0.0;
  for (int k = tid; k <= kNpb; k += 256) se += exp(static_cast<double>(zl[k]) - zmax);
  se = block_sum<double>(se, red);
  const double lse = zmax + log(se);
  const double lg = lag[b];
  const double alpha = theta[oAlpha];
  double lossp = 0.0, galpha = 0.0;
  for (int k = tid; k <= kNpb; k += 256) {
    const double pk = exp(static_cast<double>(zl[k]) - lse);
    const double dz = pk - static_cast<double>(q[k]);
    if (q[k] > 0.0f) lossp -= static_cast<double>(q[k]) * (static_cast<double>(zl[k]) - lse);
    if (k < kNpb) {
      double phi, fr;
      int i0;
      head_phi(ac, lg, k, phi, i0, fr);
      galpha += dz * phi;
      gp[oBeta + k] = static_cast<float>(dz);
      dphi[k] = static_cast<float>(alpha * dz);
      bi0[k] = i0;
      bfr[k] = static_cast<float>(fr);
    } else {
      gp[oDelta] = static_cast<float>(dz);
    }
  }
  lossp = block_sum<double>(lossp, red);
  galpha = block_sum<double>(galpha, red);
  if (tid == 0) {
    lpart[b] = static_cast<float>(lossp);
    gp[oAlpha] = static_cast<float>(galpha);
  }
  // ---- interpolation: gather into each lag from the bins that read it, in bin
  // order (bin lags are non-decreasing in k)
  for (int tau = tid; tau < kL2; tau += 256) {
    float v = 0.f;
    for (int k = 0; k < kNpb; ++k) {
      const int i0 = bi0[k];
      if (i0 < 0 || i0 + 1 < tau) continue;
      if (i0 > tau) break;
      if (i0 == tau) v += (1.0f - bfr[k]) * dphi[k];
      else v += bfr[k] * dphi[k];  // i0 + 1 == tau
    }
    dA[tau] = v;
  }
  __syncthreads();
  // ---- normalisation Ahat = A / (A0 + eps)
  const double den = static_cast<double>(ac[0]) + kEps;
  double dot = 0.0;
  for (int tau = tid; tau < kL2; tau += 256) dot += static_cast<double>(dA[tau]) * static_cast<double>(ac[tau]);
  dot = block_sum<double>(dot, red);
  for (int tau = tid; tau < kL2; tau += 256) {
    double v = static_cast<double>(dA[tau]) / den;
    if (tau == 0) v -= dot / (den * den);
    dA[tau] = static_cast<float>(v);
  }
  __syncthreads();
  // ---- autocorrelation -> ds (into ac's storage), then remove its mean
  float* ds = ac;
  float dsv[4];
  for (int j = 0; j < 4; ++j) {
    const int t0 = tid + 256 * j;
    float v = 0.f;
    for (int tau = 0; tau < kL2; ++tau) {
      float u = 0.f;
      if (t0 + tau < kL2) u += ss[t0 + tau];
      if (t0 - tau >= 0) u += ss[t0 - tau];
      v += dA[tau] * u;
    }
    dsv[j] = v / kL2;
  }
  __syncthreads();  // every read of ac (A) is done
  float dsum = 0.f;
  for (int j = 0; j < 4; ++j) dsum += dsv[j];
  const float dmean = block_sum<float>(dsum, reinterpret_cast<float*>(red)) / kL2;
  for (int j = 0; j < 4; ++j) ds[tid + 256 * j] = dsv[j] - dmean;
  __syncthreads();
  // ---- 1x1 conv and ReLU2: dz2 = w3 ds [a2 > 0]; dw3, db2 by (channel, part) sums
  for (int i = tid; i < kC2 * kL2; i += 256) {
    const int o = i / kL2, l = i - o * kL2;
    dz2[i] = bf16_val(ga2[i]) > 0.0f ? theta[oW3 + o] * ds[l] : 0.0f;
  }
  __syncthreads();
  {
    const int c = tid >> 4, part16 = tid & 15;
    float w3p = 0.f, b2p = 0.f;
    for (int l = part16 * 64; l < part16 * 64 + 64; ++l) {
      w3p += ds[l] * bf16_val(ga2[c * kL2 + l]);
      b2p += dz2[c * kL2 + l];
    }
    dphi[tid] = w3p;        // dphi no longer needed: reuse as [16][16] partials
    dphi[256 + tid] = b2p;
  }
  __syncthreads();
  if (tid < kC2) {
    float w3s = 0.f, b2s = 0.f;
    for (int p = 0; p < 16; ++p) {
      w3s += dphi[tid * 16 + p];
      b2s += dphi[256 + tid * 16 + p];
    }
    gp[oW3 + tid] = w3s;
    gp[oB2 + tid] = b2s;
  }
  // ---- conv2 weights: thread (o, c) owns the 8 taps
  {
    const int o = tid >> 4, c = tid & 15;
    float g[kK2];
    for (int k = 0; k < kK2; ++k) g[k] = 0.f;
    for (int l = 0; l < kL2; ++l) {
      const float dzv = dz2[o * kL2 + l];
      if (dzv == 0.0f) continue;
      for (int k = 0; k < kK2; ++k) {
        const int p = 2 * l + k - kP2;
        if (p >= 0 && p < kL1) g[k] += dzv * bf16_val(a1s[c * kL1 + p]);
      }
    }
    for (int k = 0; k < kK2; ++k) gp[oW2 + (o * kC1 + c) * kK2 + k] = g[k];
  }
  // ---- conv2 data gradient -> ReLU1 -> conv1 weights, in chunks of 64 positions
  {
    const int o1 = tid >> 4, c1 = (tid >> 3) & 1, kp = (tid & 7) * 2;
    float gw0 = 0.f, gw1 = 0.f, gb = 0.f;
    for (int p0 = 0; p0 < kL1; p0 += 64) {
      __syncthreads();
      for (int i = tid; i < kC1 * 64; i += 256) {
        const int c = i >> 6, p = p0 + (i & 63);
        float v = 0.f;
        if (bf16_val(a1s[c * kL1 + p]) > 0.0f) {
          for (int k = (p + kP2) & 1; k < kK2; k += 2) {
            const int l = (p + kP2 - k) >> 1;
            if (l < 0 || l >= kL2) continue;
            for (int o = 0; o < kC2; ++o)
              v += dz2[o * kL2 + l] * bf16_val(bf16_bits(theta[oW2 + (o * kC1 + c) * kK2 + k]));
          }
        }
        dz1[i] = v;
      }
      __syncthreads();
      for (int pp = 0; pp < 64; ++pp) {
        const int l = p0 + pp;
        const float dzv = dz1[o1 * 64 + pp];
        const int xp0 = 2 * l + kp - kP1, xp1 = xp0 + 1;
        if (xp0 >= 0 && xp0 < kL0) gw0 += dzv * bf16_val(xb[c1 * kL0 + xp0]);
        if (xp1 >= 0 && xp1 < kL0) gw1 += dzv * bf16_val(xb[c1 * kL0 + xp1]);
        if (c1 == 0 && kp == 0) gb += dzv;
      }
    }
    gp[oW1 + (o1 * kCin + c1) * kK1 + kp] = gw0;
    gp[oW1 + (o1 * kCin + c1) * kK1 + kp + 1] = gw1;
    if (c1 == 0 && kp == 0) gp[oB1 + o1] = gb;
  }
}

// Mean over the batch, in batch order (deterministic).
__global__ void k_reduce(const float* __restrict__ gpart, const float* __restrict__ lpart, int32_t B,
                         float* __restrict__ grad, float* __restrict__ loss) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < kNParam) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += gpart[static_cast<int64_t>(b) * kNParam + j];
    grad[j] = static_cast<float>(s / B);
  }
  if (j == 0 && loss) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += lpart[b];
    *loss = static_cast<float>(s / B);
  }
}

// Adam (Kingma & Ba 2015) on FP32 master weights.
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kNParam) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.0f - b1) * gj;
  const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  theta[j] -= lr * (mj * c1) / (sqrtf(vj * c2) + eps);
}

// ----------------------------------------------------------------------------
// Proposal: one wave per star.  Softmax, top-k bins (ties to the lower bin), each
// widened by one bin on both sides; confidence = null probability + the mass of
// the selected bins.  Confident stars get the maximal runs of selected bins as
// period windows, plus every period beyond the heatmap, clipped to [Pmin, Pmax]
// and mapped to frequency-index ranges of the closed-form grid; the others get
// their full grid and the fallback flag.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_propose(const StarDesc* __restrict__ stars, const float* __restrict__ logits,
                                                int32_t topk, float conf, int32_t search_long,
                                                const StarDesc* __restrict__ cstars, const double* __restrict__ csnr,
                                                int32_t n_peaks, int32_t halfwidth,
                                                int64_t* __restrict__ windows, uint8_t* __restrict__ fallback,
                                                float* __restrict__ conf_out, int64_t* __restrict__ tiles) {
  __shared__ uint8_t sel[kNpb];
  __shared__ double pr[kNpb + 1];
  __shared__ int64_t s_w0[PP_MAX_WINDOWS], s_w1[PP_MAX_WINDOWS], s_cum[PP_MAX_WINDOWS + 1];
  __shared__ int64_t s_pick[PP_MAX_WINDOWS];
  __shared__ int s_nw, s_fb, s_np;
  const int s = blockIdx.x, lane = threadIdx.x;
  const StarDesc d = stars[s];
  const float* z = logits + static_cast<int64_t>(s) * (kNpb + 1);
  double zm = -INFINITY;
  for (int k = lane; k <= kNpb; k += 64) zm = fmax(zm, static_cast<double>(z[k]));
  for (int o = 32; o > 0; o >>= 1) zm = fmax(zm, __shfl_xor(zm, o, 64));
  double se = 0.0;
  for (int k = lane; k <= kNpb; k += 64) se += exp(static_cast<double>(z[k]) - zm);
  for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o, 64);
  for (int k = lane; k <= kNpb; k += 64) pr[k] = exp(static_cast<double>(z[k]) - zm) / se;
  for (int k = lane; k < kNpb; k += 64) sel[k] = 0;
  __syncthreads();
  unsigned long long taken = 0ull;  // bit j: bin lane + 64 j already chosen
  for (int r = 0; r < topk; ++r) {
    double bv = -1.0;
    int bk = kNpb;
    for (int j = 0; j < kNpb / 64; ++j) {
      const int k = lane + 64 * j;
      if (!((taken >> j) & 1ull) && (pr[k] > bv || (pr[k] == bv && k < bk))) {
        bv = pr[k];
        bk = k;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int ok = __shfl_xor(bk, o, 64);
      if (ov > bv || (ov == bv && ok < bk)) {
        bv = ov;
        bk = ok;
      }
    }
    if (bk < kNpb) {
      if ((bk & 63) == lane) taken |= 1ull << (bk >> 6);
      if (lane == 0)
        for (int k = bk - 1; k <= bk + 1; ++k)
          if (k >= 0 && k < kNpb) sel[k] = 1;
    }
    __syncthreads();
  }
  double mass = 0.0;
  for (int k = lane; k < kNpb; k += 64) mass += sel[k] ? pr[k] : 0.0;
  for (int o = 32; o > 0; o >>= 1) mass += __shfl_xor(mass, o, 64);
  const double c = pr[kNpb] + mass;
  int64_t* wo = windows + static_cast<int64_t>(s) * PP_MAX_WINDOWS * 3;
  if (lane == 0) {
    if (conf_out) conf_out[s] = static_cast<float>(c);
    int nw = 0;
    auto emit = [&](int64_t i0, int64_t i1) {
      if (nw < PP_MAX_WINDOWS && i1 > i0) {
        s_w0[nw] = i0;
        s_w1[nw] = i1;
        ++nw;
      }
    };
    const bool fb = !(c >= static_cast<double>(conf));
    fallback[s] = fb ? 1 : 0;
    s_fb = fb ? 1 : 0;
    if (fb) {
      emit(0, d.nf);
    } else {
      auto range = [&](double plo, double phi) {
        plo = fmax(plo, d.pmin);
        phi = fmin(phi, d.pmax);
        if (!(phi > plo)) return;
        const double flo = 1.0 / phi, fhi = 1.0 / plo;
        const double a = ceil((cbrt(flo) - d.umin) / d.A);
        const double e = floor((cbrt(fhi) - d.umin) / d.A);
        const int64_t i0 = a < 0.0 ? 0 : static_cast<int64_t>(a);
        const int64_t i1 = e > static_cast<double>(d.nf - 1) ? d.nf - 1 : static_cast<int64_t>(e);
        if (e >= 0.0 && i1 >= i0) emit(i0, i1 + 1);
      };
      int k = 0;
      while (k < kNpb) {
        if (sel[k]) {
          int k1 = k;
          while (k1 + 1 < kNpb && sel[k1 + 1]) ++k1;
          range(period_edge(k), period_edge(k1 + 1));
          k = k1 + 1;
        } else {
          ++k;
        }
      }
      if (search_long && d.pmax > kPbHi) range(kPbHi, d.pmax);
    }
    s_nw = nw;
    s_np = 0;
  }
  __syncthreads();
  // Coarse-peak windows of a confident star: the n_peaks largest coarse S/N values,
  // each blocking +-halfwidth coarse steps around it (ties to the lower index).
  if (cstars && csnr && n_peaks > 0 && !s_fb) {
    const StarDesc cd = cstars[s];
    const double* v = csnr + cd.f_off;
    const int64_t ncf = cd.nf;
    for (int r = 0; r < n_peaks; ++r) {
      double bv = -INFINITY;
      int64_t bi = INT64_MAX;
      for (int64_t i = lane; i < ncf; i += 64) {
        bool blocked = false;
        for (int q = 0; q < r; ++q) blocked |= (i - s_pick[q] <= halfwidth && s_pick[q] - i <= halfwidth);
        if (blocked) continue;
        const double x = v[i];
        if (x > bv || (x == bv && i < bi) || bi == INT64_MAX) {
          bv = x;
          bi = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int64_t oi = __shfl_xor(bi, o, 64);
        if (oi != INT64_MAX && (bi == INT64_MAX || ov > bv || (ov == bv && oi < bi))) {
          bv = ov;
          bi = oi;
        }
      }
      if (bi == INT64_MAX) break;  // the coarse grid is exhausted
      if (lane == 0) {
        s_pick[r] = bi;
        s_np = r + 1;
      }
      __syncthreads();
    }
    if (lane == 0) {
      int nw = s_nw;
      for (int r = 0; r < s_np; ++r) {
        const int64_t lo = max<int64_t>(0, s_pick[r] - halfwidth), hi = min<int64_t>(ncf - 1, s_pick[r] + halfwidth);
        const double a = ceil(((cd.umin + static_cast<double>(lo) * cd.A) - d.umin) / d.A);
        const double e = floor(((cd.umin + static_cast<double>(hi) * cd.A) - d.umin) / d.A);
        const int64_t i0 = a < 0.0 ? 0 : static_cast<int64_t>(a);
        const int64_t i1 = e > static_cast<double>(d.nf - 1) ? d.nf - 1 : static_cast<int64_t>(e);
        if (e >= 0.0 && i1 >= i0 && nw < PP_MAX_WINDOWS) {
          s_w0[nw] = i0;
          s_w1[nw] = i1 + 1;
          ++nw;
        }
      }
      // sorted, merged (overlapping or touching ranges join)
      for (int q = 1; q < nw; ++q) {
        const int64_t a0 = s_w0[q], a1 = s_w1[q];
        int u = q - 1;
        while (u >= 0 && (s_w0[u] > a0 || (s_w0[u] == a0 && s_w1[u] > a1))) {
          s_w0[u + 1] = s_w0[u];
          s_w1[u + 1] = s_w1[u];
          --u;
        }
        s_w0[u + 1] = a0;
        s_w1[u + 1] = a1;
      }
      int m = 0;
      for (int q = 0; q < nw; ++q) {
        if (m > 0 && s_w0[q] <= s_w1[m - 1]) {
          s_w1[m - 1] = max(s_w1[m - 1], s_w1[q]);
        } else {
          s_w0[m] = s_w0[q];
          s_w1[m] = s_w1[q];
          ++m;
        }
      }
      s_nw = m;
    }
  }
  __syncthreads();
  if (lane == 0) {
    const int nw = s_nw;
    for (int q = 0; q < nw; ++q) {
      wo[3 * q] = s;
      wo[3 * q + 1] = s_w0[q];
      wo[3 * q + 2] = s_w1[q];
    }
    for (int q = nw; q < PP_MAX_WINDOWS; ++q) {
      wo[3 * q] = -1;
      wo[3 * q + 1] = 0;
      wo[3 * q + 2] = 0;
    }
    s_cum[0] = 0;
    for (int q = 0; q < nw; ++q) s_cum[q + 1] = s_cum[q] + (s_w1[q] - s_w0[q] + d.per_tile - 1) / d.per_tile;
  }
  __syncthreads();
  if (!tiles) return;
  // The same windows cut into the star's work-item size, in the star's slots of the
  // tiled list (the windows are disjoint, so they need at most ceil(nf / per) + one
  // partial tile per window slots); unused slots have star = -1.
  const int64_t per = d.per_tile;
  const int64_t cap = (d.nf + per - 1) / per + mi355bls::kWindowSlack;
  const int nw = s_nw;
  const int64_t total = s_cum[nw];
  int64_t* to = tiles + 3 * d.tile_off;
  for (int64_t j = lane; j < cap; j += 64) {
    if (j < total) {
      int q = 0;
      while (s_cum[q + 1] <= j) ++q;
      const int64_t i0 = s_w0[q] + (j - s_cum[q]) * per;
      to[3 * j] = s;
      to[3 * j + 1] = i0;
      to[3 * j + 2] = min(s_w1[q], i0 + per);
    } else {
      to[3 * j] = -1;
      to[3 * j + 1] = 0;
      to[3 * j + 2] = 0;
    }
  }
}

}  // namespace mi355pp

using namespace mi355pp;

namespace {
bool ws_ready(const bls_plan* plan, const void* ws) { return plan && ws && plan->uploaded_to == ws; }
}  // namespace

extern "C" bls_status pp_act_bytes(int32_t batch, int64_t* bytes) {
  if (batch < 0 || !bytes) return BLS_E_ARG;
  *bytes = static_cast<int64_t>(batch) * static_cast<int64_t>(kActBytes);
  return BLS_OK;
}

extern "C" bls_status pp_resample(const bls_plan* plan, void* ws, const double* d_t, const double* d_y,
                                  const double* d_w, uint16_t* d_x, double* d_lag, bls_stream_t stream) {
  if (!plan || !d_t || !d_y || !d_x || !d_lag) return BLS_E_ARG;
  if (!ws_ready(plan, ws)) return BLS_E_STATE;
  if (plan->n_stars == 0) return BLS_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const StarDesc* sd = reinterpret_cast<const StarDesc*>(static_cast<char*>(ws) + plan->layout.stars);
  hipLaunchKernelGGL(k_resample, dim3(plan->n_stars), dim3(1024), 0, st, sd, d_t, d_y, d_w, d_x, d_lag);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

extern "C" bls_status pp_forward(const float* d_theta, const uint16_t* d_x, const double* d_lag, int32_t batch,
                                 float* d_logits, void* d_act, bls_stream_t stream) {
  if (!d_theta || !d_x || !d_lag || !d_logits || batch < 0) return BLS_E_ARG;
  if (batch == 0) return BLS_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_forward, dim3(batch), dim3(256), kFwdLds, st, d_theta, d_x, d_lag, d_logits,
                     static_cast<unsigned char*>(d_act));
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

extern "C" bls_status pp_backward(const float* d_theta, const uint16_t* d_x, const double* d_lag,
                                  const float* d_target, const float* d_logits, const void* d_act, int32_t batch,
                                  float* d_gpart, float* d_lpart, float* d_grad, float* d_loss,
                                  bls_stream_t stream) {
  if (!d_theta || !d_x || !d_lag || !d_target || !d_logits || !d_act || !d_gpart || !d_lpart || !d_grad ||
      batch < 1)
    return BLS_E_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_backward, dim3(batch), dim3(256), kBwdLds, st, d_theta, d_x, d_lag, d_target, d_logits,
                     static_cast<const unsigned char*>(d_act), d_gpart, d_lpart);
  BLS_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_reduce, dim3((kNParam + 255) / 256), dim3(256), 0, st, d_gpart, d_lpart, batch, d_grad,
                     d_loss);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

extern "C" bls_status pp_adam(float* d_theta, float* d_m, float* d_v, const float* d_grad, int32_t step, float lr,
                              bls_stream_t stream) {
  if (!d_theta || !d_m || !d_v || !d_grad || step < 1 || !(lr > 0.0f)) return BLS_E_ARG;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = static_cast<float>(1.0 / (1.0 - std::pow(b1, step)));
  const float c2 = static_cast<float>(1.0 / (1.0 - std::pow(b2, step)));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, st, d_theta, d_m, d_v, d_grad, lr,
                     static_cast<float>(b1), static_cast<float>(b2), 1e-8f, c1, c2);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

extern "C" bls_status pp_tile_capacity(const bls_plan* plan, int64_t* n) {
  if (!plan || !n) return BLS_E_ARG;
  *n = plan->tile_capacity;
  return BLS_OK;
}

extern "C" bls_status pp_propose(const bls_plan* plan, void* ws, const float* d_logits, int32_t topk, float conf,
                                 int64_t* d_windows, uint8_t* d_fallback, float* d_conf, int64_t* d_tiles,
                                 bls_stream_t stream) {
  if (!plan || !d_logits || !d_windows || !d_fallback || topk < 1 || topk > PP_MAX_WINDOWS - 2) return BLS_E_ARG;
  if (!ws_ready(plan, ws)) return BLS_E_STATE;
  if (plan->n_stars == 0) return BLS_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const StarDesc* sd = reinterpret_cast<const StarDesc*>(static_cast<char*>(ws) + plan->layout.stars);
  hipLaunchKernelGGL(k_propose, dim3(plan->n_stars), dim3(64), 0, st, sd, d_logits, topk, conf, 1,
                     static_cast<const StarDesc*>(nullptr), static_cast<const double*>(nullptr), 0, 0, d_windows,
                     d_fallback, d_conf, d_tiles);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}

extern "C" bls_status pp_propose_guided(const bls_plan* plan, void* ws, const float* d_logits, int32_t topk,
                                        float conf, int32_t search_long, const bls_plan* coarse, void* coarse_ws,
                                        const double* d_coarse_snr, int32_t n_peaks, int32_t halfwidth,
                                        int64_t* d_windows, uint8_t* d_fallback, float* d_conf, int64_t* d_tiles,
                                        bls_stream_t stream) {
  if (!plan || !coarse || !d_logits || !d_coarse_snr || !d_windows || !d_fallback) return BLS_E_ARG;
  if (topk < 0 || n_peaks < 0 || halfwidth < 0 || topk + 1 + n_peaks > PP_MAX_WINDOWS) return BLS_E_ARG;
  if (coarse->n_stars != plan->n_stars) return BLS_E_ARG;
  if (!ws_ready(plan, ws) || !ws_ready(coarse, coarse_ws)) return BLS_E_STATE;
  if (plan->n_stars == 0) return BLS_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const StarDesc* sd = reinterpret_cast<const StarDesc*>(static_cast<char*>(ws) + plan->layout.stars);
  const StarDesc* cd = reinterpret_cast<const StarDesc*>(static_cast<char*>(coarse_ws) + coarse->layout.stars);
  hipLaunchKernelGGL(k_propose, dim3(plan->n_stars), dim3(64), 0, st, sd, d_logits, topk, conf, search_long, cd,
                     d_coarse_snr,
                     n_peaks, halfwidth, d_windows, d_fallback, d_conf, d_tiles);
  BLS_HIP_TRY(hipGetLastError());
  return BLS_OK;
}
