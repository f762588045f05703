// sincosm_eval_planned_noalloc: sincosm_eval_planned on a workspace that the
// library holds in a static device array, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).
//
// The array lives in device memory of every GPU the library runs on until the
// process ends. In host code its name is only a host-side handle; the device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is ever passed to kernels.
#include <mutex>

#include "schemes.hpp"

namespace {

constexpr size_t kScratchBytes = SINCOSM_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices];   // device address of `scratch` per device, null until set up

// Device address of the current device's scratch array (set up on first use).
sincosm_status scratch_for_current_device(void** out) {
  int dev = -1;
  SC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return SINCOSM_E_UNSUPPORTED;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    SC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255u)) return SINCOSM_E_HIP;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return SINCOSM_OK;
}

}  // namespace

extern "C" {

sincosm_status sincosm_eval_planned_noalloc(int64_t n, int dtype, const void* A, int64_t lda, void* C,
                                            int64_t ldc, void* S, int64_t lds, int acc, int prod,
                                            const sincosm_plan* plan_in, sincosm_plan* plan_dev, void* stream) {
  if (n < 0) return SINCOSM_E_ARG;
  if (n == 0) return sc::eval_planned(0, dtype, A, lda, C, ldc, S, lds, acc, prod, plan_in, nullptr, 0, plan_dev,
                                      (hipStream_t)stream, false);
  const size_t need = sincosm_workspace_size(n, dtype, acc, prod);
  if (need == 0) return SINCOSM_E_ARG;
  if (need > kScratchBytes) return SINCOSM_E_TOO_LARGE;
  void* ws = nullptr;
  SC_TRY(scratch_for_current_device(&ws));
  // Nothing in the workspace has to start at zero: every call writes the
  // padded copy, the norm's partial sums and its max slot before reading them.
  return sc::eval_planned(n, dtype, A, lda, C, ldc, S, lds, acc, prod, plan_in, ws, kScratchBytes, plan_dev,
                          (hipStream_t)stream, false);
}

}  // extern "C"
