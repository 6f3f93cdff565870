// Input checks of the C ABI (engineering safeguards, not part of the method).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "yyg_internal.h"

namespace yyg {

// Opt-in input check: *flag = 1 if any of x[0..n) is NaN or infinite.
// The flag is cleared by its own launch first (a fill kernel rather than a
// memset, so that the pair can sit in a recorded graph).
__global__ void clear_flag_kernel(int *flag) {
  if (threadIdx.x == 0) *flag = 0;
}

__global__ __launch_bounds__(256) void check_finite_kernel(const double *__restrict__ x, long n, int *flag) {
  bool bad = false;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) bad |= !__builtin_isfinite(x[i]);
  if (bad) *flag = 1;  // every writer stores the same value
}

hipError_t launch_check_finite(const double *x, long n, int *flag, hipStream_t s) {
  if (!flag || (n > 0 && !x) || n < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(64), 0, s, flag);
  if (n > 0) {
    const long want = (n + 256L * 8 - 1) / (256L * 8);
    const unsigned blocks = (unsigned)std::min<long>(want, 4096);
    hipLaunchKernelGGL(check_finite_kernel, dim3(blocks), dim3(256), 0, s, x, n, flag);
  }
  return hipGetLastError();
}

}  // namespace yyg
