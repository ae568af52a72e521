// Zero-fill of device words on a stream: the control block of the XCD-group kernels (all of it for
// a new run; the registration and barrier counters for a continued run and for each further
// launch of a run) and the master state of the per-iteration path before its first iteration.
// A small kernel instead of hipMemsetAsync keeps a run free of memset nodes when a caller records
// it into a HIP graph, and clears two ranges with one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "nmfa_internal.h"

namespace nmfa {

namespace {

// Words [a0, a1) and [b0, b1) of p set to zero, grid-stride.
__global__ void zero_ranges_kernel(uint32_t* __restrict__ p, size_t a0, size_t a1, size_t b0, size_t b1) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t k = a0 + i; k < a1; k += stride) p[k] = 0u;
  for (size_t k = b0 + i; k < b1; k += stride) p[k] = 0u;
}

}  // namespace

hipError_t launch_zero_words(uint32_t* p, size_t a0, size_t a1, size_t b0, size_t b1, hipStream_t st) {
  if (a1 < a0 || b1 < b0) return hipErrorInvalidValue;
  const size_t n = std::max(a1 - a0, b1 - b0);
  if (a1 == a0 && b1 == b0) return hipSuccess;
  const int threads = 256;
  const size_t blocks = std::min<size_t>((n + threads - 1) / threads, 2048);
  hipLaunchKernelGGL(zero_ranges_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, p, a0, a1, b0, b1);
  return hipGetLastError();
}

}  // namespace nmfa
