// Device kernels of the block builder (Alg. 3 assignment, Alg. 4 neighbour
// search), FP64 throughout so that distances match a plain CPU evaluation of
// sum_k (z_k - c_k)^2 in dimension order.
#include <hip/hip_runtime.h>

#include "sbv_internal.h"

namespace sbv {

// ---- nearest centre (Alg. 3 line "assign to the nearest anchor") -----------
// One thread per point; centres streamed through LDS in tiles.  Ties go to the
// lower centre id (strict comparison while scanning ids upward).
constexpr int kAssignTile = 256;

__global__ __launch_bounds__(256) void k_assign(const double* __restrict__ Z, int64_t n, int d,
                                                const double* __restrict__ C, int K,
                                                int32_t* __restrict__ lab, double* __restrict__ best_d2) {
  __shared__ double cs[kAssignTile * kMaxDim];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double z[kMaxDim];
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k) z[k] = (i < n && k < d) ? Z[i * d + k] : 0.0;
  double best = __builtin_inf();
  int bj = 0;
  for (int c0 = 0; c0 < K; c0 += kAssignTile) {
    const int cn = min(kAssignTile, K - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < cn * d; e += blockDim.x) cs[e] = C[(int64_t)c0 * d + e];
    __syncthreads();
    for (int c = 0; c < cn; ++c) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxDim; ++k) {
        if (k < d) {
          double t = z[k] - cs[c * d + k];
          s += t * t;
        }
      }
      if (s < best) {
        best = s;
        bj = c0 + c;
      }
    }
  }
  if (i < n) {
    lab[i] = bj;
    if (best_d2) best_d2[i] = best;
  }
}

hipError_t launch_assign(const double* Z, int64_t n, int d, const double* C, int K, int32_t* lab,
                         double* best_d2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_assign, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z, n, d, C, K, lab, best_d2);
  return hipGetLastError();
}

// ---- exact m nearest earlier points of each block centre (Alg. 4) ---------
// One wave per query block, eight queries per workgroup sharing point tiles in
// LDS.  Each wave keeps a candidate buffer of (distance, position) pairs below
// its running threshold tau (the m-th smallest distance kept so far); when the
// buffer could overflow it is sorted and cut back to m entries.  Ties order by
// ordered position, so the result is the exact brute-force answer.
constexpr int kKnnWaves = 8;
constexpr int kKnnTile = 256;
constexpr int kKnnCap = 1024;

struct KnnSmem {
  double pts[kKnnTile * kMaxDim];
  double bd[kKnnWaves][kKnnCap];
  int32_t bp[kKnnWaves][kKnnCap];
};

__device__ __forceinline__ bool knn_less(double da, int pa, double db, int pb) {
  return da < db || (da == db && pa < pb);
}

// Sort the first `cnt` entries of one wave's buffer (padding to the next power
// of two with +inf), bitonic network executed by the 64 lanes of the wave.
__device__ void knn_sort(double* bd, int32_t* bp, int cnt, int lane) {
  int len = 64;
  while (len < cnt) len <<= 1;
  for (int e = cnt + lane; e < len; e += 64) {
    bd[e] = __builtin_inf();
    bp[e] = 0x7fffffff;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  for (int k = 2; k <= len; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int e = lane; e < len; e += 64) {
        int p = e ^ j;
        if (p > e) {
          double de = bd[e], dp = bd[p];
          int pe = bp[e], pp = bp[p];
          bool up = (e & k) == 0;
          bool sw = up ? knn_less(dp, pp, de, pe) : knn_less(de, pe, dp, pp);
          if (sw) {
            bd[e] = dp;
            bd[p] = de;
            bp[e] = pp;
            bp[p] = pe;
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

__global__ __launch_bounds__(kKnnWaves * 64) void k_knn(const double* __restrict__ Z, int d,
                                                        const double* __restrict__ cen,
                                                        const int32_t* __restrict__ bptr, int K, int m,
                                                        const int64_t* __restrict__ nn_ptr,
                                                        int32_t* __restrict__ nn_pos,
                                                        const int32_t* __restrict__ qlist, int nq) {
  __shared__ KnnSmem sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // queries: blocks 0..K-1, or the ranks listed in qlist (ascending)
  const int nqq = qlist ? nq : K;
  const int q0 = blockIdx.x * kKnnWaves;
  const bool active = q0 + wave < nqq;
  const int q = active ? (qlist ? qlist[q0 + wave] : q0 + wave) : 0;
  const int prefix = active ? bptr[q] : 0;  // points of strictly earlier blocks
  const int ilast = min(q0 + kKnnWaves, nqq) - 1;
  const int maxprefix = bptr[qlist ? qlist[ilast] : ilast];
  double c[kMaxDim];
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k) c[k] = (active && k < d) ? cen[(int64_t)q * d + k] : 0.0;
  double* bd = sm.bd[wave];
  int32_t* bpos = sm.bp[wave];
  int cnt = 0;
  double tau = __builtin_inf();
  for (int p0 = 0; p0 < maxprefix; p0 += kKnnTile) {
    const int pn = min(kKnnTile, maxprefix - p0);
    __syncthreads();
    for (int e = tid; e < pn * d; e += kKnnWaves * 64) sm.pts[e] = Z[(int64_t)p0 * d + e];
    __syncthreads();
    if (!active || p0 >= prefix) continue;
    if (cnt > kKnnCap - kKnnTile) {
      knn_sort(bd, bpos, cnt, lane);
      cnt = min(cnt, m);
      tau = (cnt >= m) ? bd[m - 1] : __builtin_inf();
    }
    const int lim = min(pn, prefix - p0);
    for (int t0 = 0; t0 < kKnnTile; t0 += 64) {
      const int t = t0 + lane;
      double s = __builtin_inf();
      if (t < lim) {
        s = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
          if (k < d) {
            double df = sm.pts[t * d + k] - c[k];
            s += df * df;
          }
        }
      }
      const bool keep = t < lim && s <= tau;
      const unsigned long long mask = __ballot(keep);
      if (keep) {
        const int off = __popcll(mask & ((1ull << lane) - 1ull));
        bd[cnt + off] = s;
        bpos[cnt + off] = p0 + t;
      }
      cnt += __popcll(mask);
    }
  }
  if (!active) return;
  const int mi = (int)(nn_ptr[q + 1] - nn_ptr[q]);
  if (mi == 0) return;
  knn_sort(bd, bpos, cnt, lane);
  for (int e = lane; e < mi; e += 64) nn_pos[nn_ptr[q] + e] = bpos[e];
}

hipError_t launch_knn(const double* Z, int d, const double* cen, const int32_t* bptr, int K, int m,
                      const int64_t* nn_ptr, int32_t* nn_pos, hipStream_t s, const int32_t* qlist, int nq) {
  const int nqq = qlist ? nq : K;
  if (nqq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_knn, dim3((nqq + kKnnWaves - 1) / kKnnWaves), dim3(kKnnWaves * 64), 0, s, Z, d, cen,
                     bptr, K, m, nn_ptr, nn_pos, qlist, nq);
  return hipGetLastError();
}

// ---- filtered neighbour search (Alg. 4 with Eq. (distancethreashold)) -----
// Coarse step: for each query block q (one thread each, the ranks of a
// workgroup ascending), every earlier block j whose centroid lies within
// lambda_q + radius_j of q's centroid is a candidate: any point of j within
// lambda_q of c_q forces ||c_q - c_j|| <= lambda_q + radius_j.  Centroid
// tiles are shared through LDS.  cand holds at most cap ids per query; the
// count keeps running past cap so that an overflow is visible.
constexpr int kCoarseTile = 256;

__global__ __launch_bounds__(256) void k_knn_coarse(const double* __restrict__ cen, const double* __restrict__ rad,
                                                    int d, const int32_t* __restrict__ qlist, int nq,
                                                    const double* __restrict__ lam, int cap,
                                                    int32_t* __restrict__ cand, int32_t* __restrict__ ccount) {
  __shared__ double cs[kCoarseTile * kMaxDim];
  __shared__ double rs[kCoarseTile];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = i < nq;
  const int q = active ? qlist[i] : 0;
  const int qmax = qlist[min((int)(blockIdx.x * blockDim.x + blockDim.x), nq) - 1];
  double c[kMaxDim];
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k) c[k] = (active && k < d) ? cen[(int64_t)q * d + k] : 0.0;
  const double lq = active ? lam[i] : 0.0;
  int cnt = 0;
  for (int j0 = 0; j0 < qmax; j0 += kCoarseTile) {
    const int jn = min(kCoarseTile, qmax - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < jn * d; e += blockDim.x) cs[e] = cen[(int64_t)j0 * d + e];
    for (int e = threadIdx.x; e < jn; e += blockDim.x) rs[e] = rad[j0 + e];
    __syncthreads();
    const int lim = active ? min(jn, q - j0) : 0;
    for (int t = 0; t < lim; ++t) {
      double s2 = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxDim; ++k)
        if (k < d) {
          const double df = c[k] - cs[t * d + k];
          s2 += df * df;
        }
      const double thr = (lq + rs[t]) * (1.0 + 1e-12);
      if (s2 <= thr * thr) {
        if (cnt < cap) cand[(int64_t)i * cap + cnt] = j0 + t;
        ++cnt;
      }
    }
  }
  if (active) ccount[i] = cnt;
}

// Fine step: one wave per query; the points of its candidate blocks within
// lambda_q of the centroid go through the same candidate buffer and sort as the
// brute-force search.  The result is exact when at least m_q points lie within
// lambda_q (every point that close was examined); otherwise status[i] = 1 and
// the query is retried with a larger threshold, or status[i] = 2 when its
// candidate list overflowed (it goes to the brute-force search).
__global__ __launch_bounds__(kKnnWaves * 64) void k_knn_fine(const double* __restrict__ Z, int d,
                                                             const double* __restrict__ cen,
                                                             const int32_t* __restrict__ bptr,
                                                             const int32_t* __restrict__ qlist, int nq,
                                                             const double* __restrict__ lam, int cap,
                                                             const int32_t* __restrict__ cand,
                                                             const int32_t* __restrict__ ccount,
                                                             const int64_t* __restrict__ nn_ptr,
                                                             int32_t* __restrict__ nn_pos, int32_t* __restrict__ status) {
  __shared__ KnnSmem sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = blockIdx.x * kKnnWaves + wave;
  if (i >= nq) return;  // whole wave; no workgroup barrier below
  const int q = qlist[i];
  const int mi = (int)(nn_ptr[q + 1] - nn_ptr[q]);
  const int nc = ccount[i];
  if (nc > cap) {  // too many candidate blocks: a larger threshold would not help
    if (lane == 0) status[i] = 2;
    return;
  }
  double c[kMaxDim];
#pragma unroll
  for (int k = 0; k < kMaxDim; ++k) c[k] = k < d ? cen[(int64_t)q * d + k] : 0.0;
  const double l2 = lam[i] * lam[i];
  double* bd = sm.bd[wave];
  int32_t* bpos = sm.bp[wave];
  int cnt = 0, inside = 0;
  double tau = l2;
  for (int u = 0; u < nc; ++u) {
    const int j = cand[(int64_t)i * cap + u];
    const int p0 = bptr[j], p1 = bptr[j + 1];
    for (int pb = p0; pb < p1; pb += 64) {
      if (cnt > kKnnCap - 64) {
        knn_sort(bd, bpos, cnt, lane);
        cnt = min(cnt, mi);
        tau = (cnt >= mi) ? bd[mi - 1] : l2;
      }
      const int p = pb + lane;
      double s2 = __builtin_inf();
      if (p < p1) {
        s2 = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k)
          if (k < d) {
            const double df = Z[(int64_t)p * d + k] - c[k];
            s2 += df * df;
          }
      }
      inside += __popcll(__ballot(p < p1 && s2 <= l2));
      const bool keep = p < p1 && s2 <= tau;
      const unsigned long long mask = __ballot(keep);
      if (keep) {
        const int off = __popcll(mask & ((1ull << lane) - 1ull));
        bd[cnt + off] = s2;
        bpos[cnt + off] = p;
      }
      cnt += __popcll(mask);
    }
  }
  if (inside < mi) {
    if (lane == 0) status[i] = 1;
    return;
  }
  knn_sort(bd, bpos, cnt, lane);
  for (int e = lane; e < mi; e += 64) nn_pos[nn_ptr[q] + e] = bpos[e];
  if (lane == 0) status[i] = 0;
}

hipError_t launch_knn_coarse(const double* cen, const double* rad, int d, const int32_t* qlist, int nq,
                             const double* lam, int cap, int32_t* cand, int32_t* ccount, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_knn_coarse, dim3((nq + 255) / 256), dim3(256), 0, s, cen, rad, d, qlist, nq, lam, cap, cand,
                     ccount);
  return hipGetLastError();
}

hipError_t launch_knn_fine(const double* Z, int d, const double* cen, const int32_t* bptr, const int32_t* qlist,
                           int nq, const double* lam, int cap, const int32_t* cand, const int32_t* ccount,
                           const int64_t* nn_ptr, int32_t* nn_pos, int32_t* status, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_knn_fine, dim3((nq + kKnnWaves - 1) / kKnnWaves), dim3(kKnnWaves * 64), 0, s, Z, d, cen,
                     bptr, qlist, nq, lam, cap, cand, ccount, nn_ptr, nn_pos, status);
  return hipGetLastError();
}

int knn_max_m() { return kKnnCap - kKnnTile; }

}  // namespace sbv
