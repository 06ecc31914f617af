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

// Conditional simulation of predictions (Sec. 5.5): draw n_draws values per
// point from N(mean_j, var_j) with the caller's standard-normal innovations,
// then their sample mean and variance (Welford's update) and the 95 %
// interval sample mean -/+ z_{0.025} sample sd.  One thread per point; the
// innovations of one draw are contiguous, so a wave reads 64 consecutive ones.
__global__ void k_pred_draws(const double* __restrict__ mean, const double* __restrict__ var, int64_t n,
                             const double* __restrict__ xi, int n_draws, double* __restrict__ stats) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double mu = mean[j], sd = sqrt(var[j] > 0.0 ? var[j] : 0.0);
  double m = 0.0, m2 = 0.0;
  for (int t = 0; t < n_draws; ++t) {
    const double x = mu + sd * xi[(int64_t)t * n + j];
    const double dlt = x - m;
    m += dlt / (double)(t + 1);
    m2 += dlt * (x - m);
  }
  const double v = n_draws > 1 ? m2 / (double)(n_draws - 1) : 0.0;
  const double z = 1.959963984540054;  // standard-normal 0.975 quantile
  stats[j] = m;
  stats[n + j] = v;
  stats[2 * n + j] = m - z * sqrt(v);
  stats[3 * n + j] = m + z * sqrt(v);
}

hipError_t launch_pred_draws(const double* mean, const double* var, int64_t n, const double* xi, int n_draws,
                             double* stats, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pred_draws, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mean, var, n, xi, n_draws,
                     stats);
  return hipGetLastError();
}

}  // namespace sbv
