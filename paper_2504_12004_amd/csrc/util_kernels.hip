// Small device utilities of the C-ABI layer.
#include <hip/hip_runtime.h>

#include "sbv_internal.h"

namespace sbv {

// y_ord[pos_of[i]] = y[i]: observations from original order to block-rank order.
__global__ void k_scatter_y(const double* __restrict__ y, const int32_t* __restrict__ pos_of,
                            double* __restrict__ y_ord, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y_ord[pos_of[i]] = y[i];
}

hipError_t launch_scatter_y(const double* y, const int32_t* pos_of, double* y_ord, int64_t n,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_y, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, pos_of, y_ord, n);
  return hipGetLastError();
}

// y[i] = y_ord[pos_of[i]]: block-rank order back to original order.
__global__ void k_gather_y(const double* __restrict__ y_ord, const int32_t* __restrict__ pos_of,
                           double* __restrict__ y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = y_ord[pos_of[i]];
}

hipError_t launch_gather_y(const double* y_ord, const int32_t* pos_of, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_y, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y_ord, pos_of, y, n);
  return hipGetLastError();
}

}  // namespace sbv
