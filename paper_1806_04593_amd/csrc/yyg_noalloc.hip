// Device scratch of the allocation-free solve (yyg_solve_noalloc): one
// file-scope array per GPU, reached from host code only through the address
// hipGetSymbolAddress returns for the device that is current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "yyg_internal.h"

// Each GPU the library runs on holds its own copy until the process ends.
// In host code this name is a host-side stand-in, not a device address: it
// is never passed to a kernel or a copy; scratch_region hands out the
// per-device address instead.
static __device__ __align__(256) double scratch[yyg::kScratchBytes / sizeof(double)];

namespace yyg {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// The device address of this device's scratch array, looked up once per
// device (with that device current, which the caller guarantees) and kept.
hipError_t scratch_region(int device, double **ptr, size_t *bytes) {
  if (!ptr || !bytes) return hipErrorInvalidValue;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double *>(p);
  }
  *ptr = g_scratch_ptr[device];
  *bytes = kScratchBytes;
  return hipSuccess;
}

}  // namespace yyg
