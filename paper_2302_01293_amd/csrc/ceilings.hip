// ceilings.hip — microbenchmarks of the MI355X (gfx950) units the BLS search is bound
// by, so that its roofline can be stated against measured rather than only vendor
// figures:
//   * FP64 multiply and fract (the fold's phase arithmetic), FP64 -> int32 convert;
//   * 32-bit integer add (a plain VALU reference);
//   * 64-bit LDS atomic add (the boundary accumulation), per wave instruction,
//     with one and with all 64 lanes active, and the 32-bit one (counts of
//     weighted points when a star's weights are equal);
//   * a device-to-device copy (HBM read + write).
// Each kernel runs many independent chains on a full grid (8 waves per SIMD); the
// rates are in wave instructions per SIMD cycle (VALU) or CU cycles per wave
// instruction (LDS), at the device's reported clock.  Built as its own library
// (libmi355ceil.so): nothing in the search path depends on it.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kIters = 4096;
constexpr int kChains = 8;
constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) c_dmul(double* out, double f) {
  double x[kChains];
  for (int c = 0; c < kChains; ++c) x[c] = 1.0 + 1e-9 * (threadIdx.x + c);
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = x[c] * f;
  }
  double s = 0.0;
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) c_fract(double* out, double) {
  double x[kChains];
  for (int c = 0; c < kChains; ++c) x[c] = 1.5 + 1e-9 * (threadIdx.x + c);
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      x[c] = __builtin_amdgcn_fract(x[c]);
      asm volatile("" : "+v"(x[c]));
    }
  }
  double s = 0.0;
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// convert + xor per step: the xor's share is measured by c_iadd
__global__ void __launch_bounds__(kThreads) c_cvt(double* out, double) {
  double x[kChains];
  int acc[kChains];
  for (int c = 0; c < kChains; ++c) {
    x[c] = 1.5 + (threadIdx.x + c);
    acc[c] = 0;
  }
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      asm volatile("" : "+v"(x[c]));
      int v = static_cast<int>(x[c]);
      asm volatile("" : "+v"(v));
      acc[c] ^= v;
    }
  }
  int s = 0;
  for (int c = 0; c < kChains; ++c) s += acc[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) c_iadd(double* out, double) {
  int x[kChains];
  for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x + c;
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      x[c] = x[c] + 3;
      asm volatile("" : "+v"(x[c]));
    }
  }
  int s = 0;
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Two LDS atomic adds of type U (64- or 32-bit) per iteration on `active` lanes of
// each wave; every address stays inside the 16 KB array.
template <typename U>
__global__ void __launch_bounds__(kThreads) c_lds(double* out, int active) {
  constexpr unsigned kN = 16384 / sizeof(U);
  __shared__ U g[kN];
  for (unsigned i = threadIdx.x; i < kN; i += blockDim.x) g[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const unsigned off = threadIdx.x & (kN - 1);
  for (int i = 0; i < kIters / 4; ++i) {
    if (lane < active) {
      atomicAdd(&g[(off + i) & (kN - 1)], U(1));
      atomicAdd(&g[(off + i + kN / 4) & (kN - 1)], U(1));
    }
  }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = static_cast<double>(g[threadIdx.x & (kN - 1)]);
}

__global__ void c_copy(const double4* __restrict__ src, double4* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// out[0..8]: SIMD cycles per wave instruction of DMUL, FRACT, CVT+XOR, IADD; CU cycles
// per 64-bit LDS atomic wave instruction with 64 and with 1 active lane; HBM copy
// GB/s (read + write) over `copy_bytes` (0 skips it); the clock in GHz; CU cycles per
// 32-bit LDS atomic wave instruction with 64 active lanes.  Returns 0, or the
// failing hipError_t.
extern "C" int mi355_ceilings(double* out, int64_t copy_bytes) {
  int dev = 0, cus = 0, clk_khz = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, dev)) != hipSuccess) return e;
  const int blocks = cus * 8;
  double* buf = nullptr;
  if ((e = hipMalloc(&buf, sizeof(double) * kThreads * blocks)) != hipSuccess) return e;
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  const double clk = clk_khz * 1e3;
  auto timed = [&](auto launch) -> float {
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {  // the second run is timed
      hipEventRecord(a, 0);
      launch();
      hipEventRecord(b, 0);
      hipEventSynchronize(b);
    }
    hipEventElapsedTime(&ms, a, b);
    return ms;
  };
  const double valu_instr = double(blocks) * (kThreads / 64) * kIters * kChains;
  const double simd_cycles_per_ms = 1e-3 * clk * cus * 4;
  float ms;
  ms = timed([&] { hipLaunchKernelGGL(c_dmul, dim3(blocks), dim3(kThreads), 0, 0, buf, 1.0000001); });
  out[0] = ms * simd_cycles_per_ms / valu_instr;
  ms = timed([&] { hipLaunchKernelGGL(c_fract, dim3(blocks), dim3(kThreads), 0, 0, buf, 1.0); });
  out[1] = ms * simd_cycles_per_ms / valu_instr;
  ms = timed([&] { hipLaunchKernelGGL(c_cvt, dim3(blocks), dim3(kThreads), 0, 0, buf, 1.0); });
  out[2] = ms * simd_cycles_per_ms / valu_instr;
  ms = timed([&] { hipLaunchKernelGGL(c_iadd, dim3(blocks), dim3(kThreads), 0, 0, buf, 1.0); });
  out[3] = ms * simd_cycles_per_ms / valu_instr;
  const double lds_instr = double(blocks) * (kThreads / 64) * (kIters / 4) * 2;
  ms = timed([&] { hipLaunchKernelGGL(c_lds<unsigned long long>, dim3(blocks), dim3(kThreads), 0, 0, buf, 64); });
  out[4] = ms * 1e-3 * clk * cus / lds_instr;
  ms = timed([&] { hipLaunchKernelGGL(c_lds<unsigned long long>, dim3(blocks), dim3(kThreads), 0, 0, buf, 1); });
  out[5] = ms * 1e-3 * clk * cus / lds_instr;
  ms = timed([&] { hipLaunchKernelGGL(c_lds<unsigned int>, dim3(blocks), dim3(kThreads), 0, 0, buf, 64); });
  out[8] = ms * 1e-3 * clk * cus / lds_instr;
  out[6] = 0.0;
  if (copy_bytes >= 32) {
    const int64_t n = copy_bytes / 32;
    double4 *s = nullptr, *d = nullptr;
    if ((e = hipMalloc(&s, n * 32)) == hipSuccess && (e = hipMalloc(&d, n * 32)) == hipSuccess) {
      hipMemset(s, 0, n * 32);
      ms = timed([&] { hipLaunchKernelGGL(c_copy, dim3(cus * 16), dim3(256), 0, 0, s, d, n); });
      out[6] = 2.0 * n * 32 / (ms * 1e-3) / 1e9;
    }
    if (s) hipFree(s);
    if (d) hipFree(d);
  }
  out[7] = clk / 1e9;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipEventDestroy(a);
  hipEventDestroy(b);
  hipFree(buf);
  return 0;
}
