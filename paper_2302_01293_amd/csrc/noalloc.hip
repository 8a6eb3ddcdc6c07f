// bls_run_noalloc: the whole device path of a plan (descriptor upload, preparation,
// search, S/N) on a workspace that lives in a static device array, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The kernels are those of bls_plan_upload,
// bls_prepare, bls_search_batch and bls_snr; only the workspace differs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mi355bls.h"
#include "plan.hpp"

namespace {

constexpr int64_t kScratchBytes = MI355BLS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per device, held until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: only the address from hipGetSymbolAddress
// (kept per device below) may be handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up on the first call made
// with that device current.
bls_status scratch_address(void** out) {
  int dev = 0;
  BLS_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return BLS_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BLS_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return BLS_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BLS_OK;
}

}  // namespace

extern "C" bls_status bls_run_noalloc(bls_plan* plan, const double* d_t, const double* d_y, const double* d_w,
                                      const int64_t* d_windows, int64_t n_windows, double* d_sr, bls_best* d_best,
                                      double* d_snr, bls_result* d_result, bls_stream_t stream) {
  if (!plan || !d_t || !d_y || !d_sr || !d_result) return BLS_E_ARG;
  if (plan->layout.total > kScratchBytes) return BLS_E_SCRATCH;
  void* ws = nullptr;
  bls_status s = scratch_address(&ws);
  if (s != BLS_OK) return s;
  if ((s = bls_plan_upload(plan, ws, kScratchBytes, stream)) != BLS_OK) return s;
  if ((s = bls_prepare(plan, ws, d_t, d_y, d_w, stream)) != BLS_OK) return s;
  if ((s = bls_search_batch(plan, ws, d_windows, n_windows, d_sr, d_best, stream)) != BLS_OK) return s;
  return bls_snr(plan, ws, d_sr, d_best, d_snr, d_result, stream);
}
