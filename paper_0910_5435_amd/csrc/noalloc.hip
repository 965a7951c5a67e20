// Synthesis that allocates nothing: for callers that cannot call hipMalloc (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).  The workspace of
// sht_synth (butterfly vector rows and the order-by-ring rows before the longitude FFT) is
// taken from a fixed device array of this library instead of the caller.
//
// The array is a file-scope __device__ variable: every GPU the library runs on holds its own
// copy (SHT_NOALLOC_SCRATCH_BYTES) from the first call on that device until the process
// ends.  In host code the variable's name is only a host-side handle, never a device address:
// its address on a device comes from hipGetSymbolAddress, asked once per device with that
// device current, and only that address is passed to the kernels.  Calls on one GPU share its
// array, so calls that overlap on one GPU (other streams, other host threads) race.  The
// kernels write every workspace row they later read, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sht_internal.h"

namespace sht {
namespace {

constexpr size_t kScratchBytes = SHT_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (the device must be current); null if the runtime cannot
// resolve it.
void* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace sht

extern "C" int sht_synth_noalloc(sht_plan_t plan, const double* coeff, double* grid, int nfields,
                                 void* stream) {
  if (!plan || nfields < 1) return SHT_EINVAL;
  if (sht::synth_workspace_bytes(plan, nfields) > SHT_NOALLOC_SCRATCH_BYTES) return SHT_EUNSUPPORTED;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return SHT_EHIP;
  if (prev != plan->device && hipSetDevice(plan->device) != hipSuccess) return SHT_EHIP;
  void* ws = sht::scratch_on(plan->device);
  if (prev != plan->device) (void)hipSetDevice(prev);
  if (!ws) return SHT_EHIP;
  return sht::run_synth(plan, plan->precision, coeff, grid, nfields, ws, SHT_NOALLOC_SCRATCH_BYTES, stream,
                        false);
}
