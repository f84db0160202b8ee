// Allocation-free apply: the same two launches as dogip_apply (tile kernel, shared-dof
// finish), with the staging buffer of the shared dofs' partial sums taken from a static
// device array instead of the operator's own buffer.  For callers that cannot allocate
// device memory at the call (graph capture, serving loops).
//
// Every partial sum in the staging buffer is written by exactly one tile before the
// finish kernel reads it, so nothing has to start at zero and no memset is issued.  The
// array is one per device and process: calls on one device that overlap in time (other
// streams, other host threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace dogip {

// 32 MiB per device, held until the process ends.  It covers the 3D 64^3 P3 elliptic
// operator with 512-cell tiles (about 3.9M staged partials).
static __device__ __align__(256) double scratch[DOGIP_NOALLOC_MAX_STAGE];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of scratch, taken once per device with the
// device current (the host-side name of the array is not a device address).
double* scratch_for_current_device() {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  DOGIP_CHECK(dev >= 0 && dev < kMaxDevices, DOGIP_E_RANGE, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DOGIP_CHECK(p != nullptr, DOGIP_E_HIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

void op_apply_noalloc(Op& op, const double* u, double* y, int prec, hipStream_t st) {
  const int64_t need = op_stage_entries(op);
  DOGIP_CHECK(need <= int64_t(DOGIP_NOALLOC_MAX_STAGE), DOGIP_E_RANGE,
              "operator stages " + std::to_string(need) + " partial sums; the static scratch holds " +
                  std::to_string(int64_t(DOGIP_NOALLOC_MAX_STAGE)) + " (use dogip_apply)");
  op_apply_staged(op, u, y, prec, scratch_for_current_device(), st);
}

}  // namespace dogip
