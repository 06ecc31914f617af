// FP32 kernels of the warm-start network (forward, backward, MSE, Adam) and
// of the neighbour part of its summary statistics.
#include <hip/hip_runtime.h>

#include "sbv_internal.h"

namespace sbv {

// C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) with strided operands:
//   A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn].
// Epilogue: mode 0 plain store (beta = 0) or accumulate (beta = 1);
// mode 1 adds bias and stores the pre-activation to C and GELU(.) to D.
// 64x64 output tiles, k in steps of 16 through LDS, 4x4 outputs per thread.
constexpr int kGT = 64, kGK = 16;

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_df(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__global__ __launch_bounds__(256) void k_gemm(int M, int N, int Kd, const float* __restrict__ A, int64_t sam,
                                              int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                              float* __restrict__ C, int64_t ldc, const float* __restrict__ bias,
                                              float* __restrict__ D, int mode, float beta) {
  __shared__ float As[kGK][kGT + 1];
  __shared__ float Bs[kGK][kGT + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < Kd; k0 += kGK) {
    for (int e = threadIdx.x; e < kGK * kGT; e += 256) {
      int kk = e / kGT, r = e - kk * kGT;
      int m = m0 + r, n = n0 + r, k = k0 + kk;
      As[kk][r] = (m < M && k < Kd) ? A[m * sam + k * sak] : 0.f;
      Bs[kk][r] = (n < N && k < Kd) ? B[k * sbk + n * sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[kk][ty * 4 + i];
        b[i] = Bs[kk][tx * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
      if (m >= M || n >= N) continue;
      float v = acc[i][j];
      if (mode == 1) {
        v += bias ? bias[n] : 0.f;
        C[m * ldc + n] = v;
        D[m * ldc + n] = gelu_f(v);
      } else if (mode == 2) {
        C[m * ldc + n] = v + (bias ? bias[n] : 0.f);
      } else {
        C[m * ldc + n] = (beta != 0.f ? C[m * ldc + n] : 0.f) + v;
      }
    }
}

hipError_t launch_gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                       int64_t sbn, float* C, int64_t ldc, const float* bias, float* D, int mode, float beta,
                       hipStream_t s) {
  dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, D, mode,
                     beta);
  return hipGetLastError();
}

// dZ = dA * GELU'(Z)
__global__ void k_gelu_bwd(const float* __restrict__ Z, const float* __restrict__ dA, float* __restrict__ dZ,
                           int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dZ[i] = dA[i] * gelu_df(Z[i]);
}

hipError_t launch_gelu_bwd(const float* Z, const float* dA, float* dZ, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z, dA, dZ, n);
  return hipGetLastError();
}

// column sums: db[n] = sum_m dZ[m][n] (fixed order per column)
__global__ void k_colsum(const float* __restrict__ dZ, int M, int N, float* __restrict__ db) {
  int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(int64_t)m * N + n];
  db[n] = s;
}

hipError_t launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, dZ, M, N, db);
  return hipGetLastError();
}

// MSE: loss = 1/(M N) sum (yhat - y)^2, dY = 2 (yhat - y) / (M N).  One
// workgroup; the loss is summed in FP64 in a fixed order.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ yhat, const float* __restrict__ y, int64_t n,
                                             float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  const float sc = 2.0f / (float)n;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    float e = yhat[i] - y[i];
    s += (double)e * e;
    dy[i] = sc * e;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / (double)n);
}

hipError_t launch_mse(const float* yhat, const float* y, int64_t n, float* dy, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, yhat, y, n, dy, loss);
  return hipGetLastError();
}

// Adam (Kingma & Ba 2015), bias-corrected, step t >= 1.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float mi = b1 * m[i] + (1.f - b1) * g[i];
  float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

// y = (x - mu) / sd per column (standardisation of features / targets) and the
// inverse map for predictions.
__global__ void k_affine_cols(const float* __restrict__ x, int64_t rows, int cols, const float* __restrict__ mu,
                              const float* __restrict__ sd, float* __restrict__ y, int inverse) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  int c = (int)(i % cols);
  y[i] = inverse ? x[i] * sd[c] + mu[c] : (x[i] - mu[c]) / sd[c];
}

hipError_t launch_affine_cols(const float* x, int64_t rows, int cols, const float* mu, const float* sd, float* y,
                              int inverse, hipStream_t s) {
  int64_t n = rows * cols;
  hipLaunchKernelGGL(k_affine_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, rows, cols, mu, sd, y,
                     inverse);
  return hipGetLastError();
}

// Gather rows of a batch: out[r] = in[idx[r]] (cols values each).
__global__ void k_gather_rows(const float* __restrict__ in, const int32_t* __restrict__ idx, int rows, int cols,
                              float* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  int r = i / cols, c = i - r * cols;
  out[i] = in[(int64_t)idx[r] * cols + c];
}

hipError_t launch_gather_rows(const float* in, const int32_t* idx, int rows, int cols, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_rows, dim3((rows * cols + 255) / 256), dim3(256), 0, s, in, idx, rows, cols, out);
  return hipGetLastError();
}

// 16 nearest neighbours (Euclidean, unscaled, excluding self) of every point of
// a subsample, FP64, ties to the lower index: one thread per query, points
// streamed through LDS.
constexpr int kFeatK = 16;
__global__ __launch_bounds__(256) void k_knn16(const double* __restrict__ P, int ns, int d, int32_t* __restrict__ nn) {
  __shared__ double tile[256 * kMaxDim];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double q[kMaxDim];
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k) q[k] = (i < ns && k < d) ? P[(int64_t)i * d + k] : 0.0;
  double bd[kFeatK];
  int bi[kFeatK];
#pragma unroll
  for (int k = 0; k < kFeatK; ++k) {
    bd[k] = __builtin_inf();
    bi[k] = 0x7fffffff;
  }
  for (int j0 = 0; j0 < ns; j0 += 256) {
    const int jn = min(256, ns - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < jn * d; e += 256) tile[e] = P[(int64_t)j0 * d + e];
    __syncthreads();
    if (i >= ns) continue;
    for (int jj = 0; jj < jn; ++jj) {
      const int j = j0 + jj;
      if (j == i) continue;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxDim; ++k)
        if (k < d) {
          double t = q[k] - tile[jj * d + k];
          s += t * t;
        }
      if (s < bd[kFeatK - 1]) {
        // insertion into the sorted list (strict: earlier index wins ties)
        double cd = s;
        int ci = j;
#pragma unroll
        for (int k = 0; k < kFeatK; ++k) {
          if (cd < bd[k]) {
            double td = bd[k];
            int tix = bi[k];
            bd[k] = cd;
            bi[k] = ci;
            cd = td;
            ci = tix;
          }
        }
      }
    }
  }
  if (i < ns)
    for (int k = 0; k < kFeatK; ++k) nn[(int64_t)i * kFeatK + k] = bi[k];
}

hipError_t launch_knn16(const double* P, int ns, int d, int32_t* nn, hipStream_t s) {
  hipLaunchKernelGGL(k_knn16, dim3((ns + 255) / 256), dim3(256), 0, s, P, ns, d, nn);
  return hipGetLastError();
}

}  // namespace sbv
