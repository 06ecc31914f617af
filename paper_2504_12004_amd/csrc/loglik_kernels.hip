// Fused per-block SBV log-likelihood kernels for gfx950 (MI355X).
//
// One workgroup owns one block i of one dataset at a time and computes the
// block term of Alg. 5 in a single pass over the joint set A = J_i u B_i
// (conditioning points first):
//   - gather the coordinates of A, scaled by the ranges (Sec. 4.4 Eq. (scale)),
//     and the observations into LDS;
//   - build the joint covariance Sigma_A = sigma^2 rho(r) + tau^2 I
//     (Eq. (maternkernel), nugget on the diagonal) straight into registers as
//     16x16 tiles in the MFMA accumulator layout;
//   - factor Sigma_A = L L^T with a right-looking tiled Cholesky whose trailing
//     updates run on v_mfma_*_16x16x4 (FP64 or FP32).  The leading m_i x m_i
//     part of L is Alg. 5's POTRF(Sigma_con), the off-diagonal part is its
//     TRSM(Sigma_cross) transposed, and the trailing b_i x b_i part is
//     POTRF(Sigma_con - Sigma_cor) -- the same numbers as Alg. 5 without ever
//     forming Sigma_cor separately;
//   - solve L z = [y_J; y_B] alongside (Alg. 5's TRSVs and GEMV);
//   - accumulate in FP64 the trailing log-pivots and z_k^2 (Alg. 5 Step 2's
//     log-determinant and dot product) and write
//       l_i = -1/2 (sum z_k^2 + 2 sum log L_kk + b_i log 2 pi).
//
// Register tiles: the lower triangle of the nt x nt tile grid (nt = ceil(nA/16))
// is numbered column by column and tile t lives in slot t / NW of wave t % NW.
// A slot holds G = -(trailing block)^T in the accumulator layout so that
// updates are plain MFMA accumulations and the triangular solve takes its A
// operand straight from the registers.
#include <hip/hip_runtime.h>

#include "sbv_internal.h"

namespace sbv {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 operand conventions (checked on the device):
//   A (16x4): lane l holds A[l%16][l/16];  B (4x16): lane l holds B[l/16][l%16];
//   C/D:      lane l, register t holds C[row(l/16, t)][l%16] with
//             row = g + 4t for FP64 and 4g + t for FP32.
// The K index of chunk q seen by lane group g is kap(q, g) = row(g, q), so that
// register q of a tile is the A operand of chunk q of its transpose.
template <typename T>
struct MF;
template <>
struct MF<double> {
  typedef d4 acc;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int g, int t) { return g + 4 * t; }
  __device__ static constexpr int qof(int c) { return c >> 2; }
  __device__ static constexpr int gof(int c) { return c & 3; }
};
template <>
struct MF<float> {
  typedef f4 acc;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int g, int t) { return 4 * g + t; }
  __device__ static constexpr int qof(int c) { return c & 3; }
  __device__ static constexpr int gof(int c) { return c >> 2; }
};

// Offset inside a 256-entry operand tile of element (r, c), c being the K index.
template <typename T>
__device__ __forceinline__ int opoff(int r, int c) {
  return 64 * MF<T>::qof(c) + 16 * MF<T>::gof(c) + r;
}

__device__ __forceinline__ double rlane(double v, int l) {
  unsigned long long u = (unsigned long long)__double_as_longlong(v);
  unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffull), l);
  unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float rlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float t_sqrt(float x) { return sqrtf(x); }

// Matern correlation, closed forms of Eq. (maternkernel) for half-integer nu.
template <typename T>
__device__ __forceinline__ T matern(T r, int two_nu) {
  T e = t_exp(-r);
  if (two_nu == 5) return (T(1) + r + r * r * T(1.0 / 3.0)) * e;
  if (two_nu == 3) return (T(1) + r) * e;
  if (two_nu == 7) return (T(1) + r + r * r * T(0.4) + r * r * r * T(1.0 / 15.0)) * e;
  return e;
}

constexpr double kLog2Pi = 1.83787706640934548356065947281123527;

template <typename T, int NTM>
struct Smem {
  T z[NTM * kTile * kMaxDim];  // scaled coordinates of A (padded rows unused)
  T yv[NTM * kTile];           // observations, overwritten by the forward solve
  T panel[NTM * 256];          // column k of L, operand layout, per tile row
  T diag[256];                 // diagonal tile to factor (row-major)
  T negM[256];                 // -(L_kk^{-T}) in B-operand layout
  T zk[kTile];                 // solved z of the current tile row
  int flag;
};

// Factor the 16x16 SPD tile in sm.diag on one wave (rows in lanes 0..15,
// lanes 16..63 shadow them): L by right-looking pivots with readlane
// broadcasts, the forward solve z_k = L_kk^{-1} y_k folded into the same pivot
// loop, then X = L^{-1} column by column, published as -X^T.  Lane r < 16
// returns its pivot L_rr and z_r; `bad` is raised for a non-positive or
// non-finite pivot and `low` for a pivot at or below tau * original diagonal
// (the FP32 fallback test).
template <typename T, int NTM>
__device__ void factor_diag(Smem<T, NTM>& sm, int lane, int k, int nreal, T diag0, T tau, T& pivot_out,
                            T& z_out, int& bad, int& low) {
  const int r = lane & 15;
  T a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = sm.diag[r * 16 + c];
  T yr = sm.yv[kTile * k + r];
  T invd[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    T piv = rlane(a[j], j);
    if (!(piv > T(0)) || !(piv == piv) || piv > T(3.0e38)) bad = 1;
    if (piv <= tau * (j < nreal ? diag0 : T(1))) low = 1;
    T sq = t_sqrt(piv);
    T inv = T(1) / sq;
    invd[j] = inv;
    a[j] = (r == j) ? sq : a[j] * inv;
    T zj = rlane(yr, j) * inv;
    yr = (r == j) ? zj : (r > j ? yr - a[j] * zj : yr);
#pragma unroll
    for (int c = j + 1; c < 16; ++c) {
      T lcj = rlane(a[j], c);
      a[c] = a[c] - a[j] * lcj;
    }
  }
  pivot_out = a[r];
  z_out = yr;
  // L to LDS (row-major, reusing the diagonal buffer), then X = L^{-1} with
  // lane r owning column r and reading L by broadcast; x[k] = 0 above the
  // diagonal.  One wave writes and reads, so waiting for its own LDS writes
  // orders them.
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) sm.diag[r * 16 + c] = (c <= r) ? a[c] : T(0);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  T x[16];
#pragma unroll
  for (int rr = 0; rr < 16; ++rr) {
    T acc = (rr == r) ? T(1) : T(0);
#pragma unroll
    for (int kk = 0; kk < rr; ++kk) acc = acc - sm.diag[rr * 16 + kk] * x[kk];
    x[rr] = acc * invd[rr];
  }
  // M = X^T: row r of M is column r of X, held here.  Store -M.
  if (lane < 16) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) sm.negM[opoff<T>(cc, r)] = -x[cc];
  }
}


// Stage tile column j of G = -Sigma_A^T blocks into sm.panel in accumulator
// order: tile i (i >= j) entry (register t, lane l) holds
// -Sigma(point 16i + l%16, point 16j + row(l/16, t)), with tau^2 on the
// diagonal and identity rows/columns past the joint size.
template <typename T, int NTM, int NTHR>
__device__ void gen_column(Smem<T, NTM>& sm, int tid, int j, int nt, int nA, int d, int two_nu, T sigma2,
                           T tau2) {
  const int total = (nt - j) * 256;
  for (int e = tid; e < total; e += NTHR) {
    const int i = j + (e >> 8);
    const int r8 = e & 255;
    const int t = r8 >> 6, l = r8 & 63;
    const int pb = kTile * i + (l & 15);
    const int pa = kTile * j + MF<T>::row(l >> 4, t);
    T v;
    if (pa >= nA || pb >= nA) {
      v = (pa == pb) ? T(-1) : T(0);
    } else {
      T r2 = T(0);
      for (int k = 0; k < d; ++k) {
        T df = sm.z[pa * d + k] - sm.z[pb * d + k];
        r2 += df * df;
      }
      v = -(sigma2 * matern<T>(t_sqrt(r2), two_nu));
      if (pa == pb) v -= tau2;
    }
    sm.panel[256 * i + r8] = v;
  }
}

// Panel wave: for every tile step factors the diagonal tile, solves the 16
// entries of z, accumulates the trailing log-pivots and z^2 in FP64, and
// applies the forward-solve update to the observations below.
template <typename T, int NTM, int NTHR>
__device__ void panel_wave(Smem<T, NTM>& sm, int lane, int nt, int mi, int nA, int d, int two_nu, T sigma2,
                           T tau2, T tau, double& ld_acc, double& q_acc, int& bad, int& low) {
  const T diag0 = sigma2 + tau2;
  for (int j = 0; j < nt; ++j) {
    gen_column<T, NTM, NTHR>(sm, lane, j, nt, nA, d, two_nu, sigma2, tau2);
    __syncthreads();  // G1
    __syncthreads();  // G2
  }
  for (int k = 0; k < nt; ++k) {
    __syncthreads();  // S1: diagonal tile published
    T piv, zr;
    factor_diag<T, NTM>(sm, lane, k, nA - kTile * k, diag0, tau, piv, zr, bad, low);
    const int rowg = kTile * k + lane;
    if (lane < 16) {
      sm.zk[lane] = zr;
      if (rowg >= mi && rowg < nA) {
        ld_acc += log((double)piv);
        q_acc += (double)zr * (double)zr;
      }
    }
    __syncthreads();  // S2: -L_kk^{-T} and z_k published
    __syncthreads();  // S3: column k of L published
    for (int rho = kTile * (k + 1) + lane; rho < kTile * nt; rho += 64) {
      const T* P = sm.panel + 256 * (rho >> 4);
      const int rr = rho & 15;
      T v = sm.yv[rho];
#pragma unroll
      for (int c = 0; c < 16; ++c) v -= P[opoff<T>(rr, c)] * sm.zk[c];
      sm.yv[rho] = v;
    }
  }
}

// Worker waves: own the register tiles, build them from the covariance, and
// run the column TRSMs and trailing MFMA updates of every step.
template <typename T, int NTM, int NWK, int NTHR>
__device__ void worker_waves(Smem<T, NTM>& sm, int wk, int lane, int nt, int nA, int d, int two_nu,
                             T sigma2, T tau2) {
  typedef typename MF<T>::acc acc_t;
  constexpr int NTT = NTM * (NTM + 1) / 2;
  constexpr int SLOTS = (NTT + NWK - 1) / NWK;
  const int g = lane >> 4;
  const int cl = lane & 15;
  const int ntt = nt * (nt + 1) / 2;
  int ti[SLOTS], tj[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    int t = s * NWK + wk;
    int i = -1, j = -1;
    if (t < ntt) {
      j = 0;
      while (t >= nt - j) {
        t -= nt - j;
        ++j;
      }
      i = j + t;
    }
    ti[s] = i;
    tj[s] = j;
  }
  // covariance tiles, one tile column at a time: every thread of the
  // workgroup builds entries into LDS (gen_column), owners copy theirs in.
  acc_t acc[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[s][t] = T(0);
  }
  for (int j = 0; j < nt; ++j) {
    gen_column<T, NTM, NTHR>(sm, 64 * (wk + 1) + lane, j, nt, nA, d, two_nu, sigma2, tau2);
    __syncthreads();  // G1: column j staged
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] == j) {
        const T* src = sm.panel + 256 * ti[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[s][t] = src[64 * t + lane];
      }
    }
    __syncthreads();  // G2: staging area free
  }
  for (int k = 0; k < nt; ++k) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (ti[s] == k && tj[s] == k) {
#pragma unroll
        for (int t = 0; t < 4; ++t) sm.diag[cl * 16 + MF<T>::row(g, t)] = -acc[s][t];
      }
    }
    __syncthreads();  // S1
    __syncthreads();  // S2
    // column-k TRSM: L_ik = A_ik L_kk^{-T}, published in operand layout
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] == k && ti[s] > k) {
        acc_t o = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 4; ++q) o = MF<T>::mma(acc[s][q], sm.negM[64 * q + lane], o);
        acc[s] = o;
        T* P = sm.panel + 256 * ti[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) P[opoff<T>(MF<T>::row(g, t), cl)] = o[t];
      }
    }
    __syncthreads();  // S3
    // trailing update G_ij += L_jk L_ik^T
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] > k) {
        const T* Pj = sm.panel + 256 * tj[s];
        const T* Pi = sm.panel + 256 * ti[s];
        acc_t o = acc[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) o = MF<T>::mma(Pj[64 * q + lane], Pi[64 * q + lane], o);
        acc[s] = o;
      }
      }
  }
}

template <typename T, int NTM, int NW>
__global__ __launch_bounds__(NW * 64) void k_block_loglik(const SetDesc* __restrict__ sets,
                                                          const double* __restrict__ theta,
                                                          const WorkItem* __restrict__ items,
                                                          const int* __restrict__ count,
                                                          double piv_tau) {
  __shared__ Smem<T, NTM> sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int total = *count;

  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const WorkItem w = items[it];
    const SetDesc S = sets[w.set];
    const int d = S.d;
    const double* th = theta + S.theta_off;
    const int b0 = S.bptr[w.block], b1 = S.bptr[w.block + 1];
    const int64_t n0 = S.nptr[w.block], n1 = S.nptr[w.block + 1];
    const int mi = (int)(n1 - n0), bi = b1 - b0, nA = mi + bi;
    const int nt = (nA + kTile - 1) / kTile;
    const T sigma2 = T(exp(th[d]));
    const T tau2 = T(exp(th[d + 1]));

    // gather A = J u B (J first): scaled coordinates and observations
    for (int e = tid; e < nA * d; e += NW * 64) {
      int p = e / d, k = e - p * d;
      int pos = p < mi ? S.nidx[n0 + p] : b0 + (p - mi);
      sm.z[p * d + k] = T(S.X[(int64_t)pos * d + k] * exp(-th[k]));
    }
    for (int p = tid; p < nt * kTile; p += NW * 64) {
      T v = T(0);
      if (p < nA) v = T(S.y[p < mi ? S.nidx[n0 + p] : b0 + (p - mi)]);
      sm.yv[p] = v;
    }
    __syncthreads();

    if (wave == 0) {
      double ld_acc = 0.0, q_acc = 0.0;
      int bad = 0, low = 0;
      panel_wave<T, NTM, NW * 64>(sm, lane, nt, mi, nA, d, S.two_nu, sigma2, tau2, T(piv_tau), ld_acc, q_acc,
                                  bad, low);
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) {
        ld_acc += __shfl_xor(ld_acc, off, 16);
        q_acc += __shfl_xor(q_acc, off, 16);
      }
      if (lane == 0) {
        int fb = (bad ? 2 : 0) | (low ? 1 : 0);
        double l = -0.5 * (q_acc + 2.0 * ld_acc + (double)bi * kLog2Pi);
        if (bad) l = -__builtin_inf();
        S.llb[w.block] = l;
        S.flag[w.block] = fb;
      }
    } else {
      worker_waves<T, NTM, NW - 1, NW * 64>(sm, wave - 1, lane, nt, nA, d, S.two_nu, sigma2, tau2);
    }
    __syncthreads();
  }
}

// ---- variants -------------------------------------------------------------
static const Variant kVariants[] = {{4, 2}, {8, 4}, {12, 8}, {17, 8}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int n_variants() { return kNumVariants; }
Variant variant(int v) { return kVariants[v]; }
int variant_for(int nA) {
  for (int v = 0; v < kNumVariants; ++v)
    if (nA <= kVariants[v].ntm * kTile) return v;
  return -1;
}

template <typename T, int NTM, int NW>
static hipError_t launch_t(int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                           const int* count, double piv_tau, hipStream_t s) {
  hipLaunchKernelGGL((k_block_loglik<T, NTM, NW>), dim3(grid), dim3(NW * 64), 0, s, sets, theta,
                     items, count, piv_tau);
  return hipGetLastError();
}

hipError_t launch_loglik(int prec, int v, int grid, const SetDesc* sets, const double* theta,
                         const WorkItem* items, const int* count, double piv_tau, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (prec == 0) {
    switch (v) {
      case 0: return launch_t<double, 4, 2>(grid, sets, theta, items, count, piv_tau, s);
      case 1: return launch_t<double, 8, 4>(grid, sets, theta, items, count, piv_tau, s);
      case 2: return launch_t<double, 12, 8>(grid, sets, theta, items, count, piv_tau, s);
      case 3: return launch_t<double, 17, 8>(grid, sets, theta, items, count, piv_tau, s);
    }
  } else {
    switch (v) {
      case 0: return launch_t<float, 4, 2>(grid, sets, theta, items, count, piv_tau, s);
      case 1: return launch_t<float, 8, 4>(grid, sets, theta, items, count, piv_tau, s);
      case 2: return launch_t<float, 12, 8>(grid, sets, theta, items, count, piv_tau, s);
      case 3: return launch_t<float, 17, 8>(grid, sets, theta, items, count, piv_tau, s);
    }
  }
  return hipErrorInvalidValue;
}

int max_grid(int prec, int v) {
  (void)prec;
  // enough resident workgroups to fill 256 CUs several times over
  return 256 * 8 / (kVariants[v].nw > 4 ? 4 : 1);
}

// ---- deterministic per-set reduction of the block terms ------------------
// One workgroup per set; thread t sums blocks t, t+256, ... in order, then a
// fixed-shape tree.  The result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_reduce(const SetDesc* __restrict__ sets,
                                                double* __restrict__ out, int* __restrict__ bad) {
  __shared__ double red[256];
  __shared__ int redb[256];
  const SetDesc S = sets[blockIdx.x];
  double s = 0.0;
  int b = 0;
  for (int i = threadIdx.x; i < S.K; i += 256) {
    s += S.llb[i];
    b |= (S.flag[i] >> 1) & 1;
  }
  red[threadIdx.x] = s;
  redb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      redb[threadIdx.x] |= redb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[blockIdx.x] = redb[0] ? -__builtin_inf() : red[0];
    if (bad) bad[blockIdx.x] = redb[0];
  }
}

hipError_t launch_reduce(const SetDesc* sets, int n_sets, const int* set_k, double* out, int* bad,
                         hipStream_t s) {
  (void)set_k;
  hipLaunchKernelGGL(k_reduce, dim3(n_sets), dim3(256), 0, s, sets, out, bad);
  return hipGetLastError();
}

// ---- FP32 fallback list: items whose fp32 pivot test fired ----------------
__global__ void k_flag_compact(const SetDesc* __restrict__ sets, const WorkItem* __restrict__ items,
                               const int* __restrict__ count, WorkItem* __restrict__ out,
                               int* __restrict__ out_count) {
  const int n = *count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    WorkItem w = items[i];
    if (sets[w.set].flag[w.block] & 3) {
      int slot = atomicAdd(out_count, 1);
      out[slot] = w;
    }
  }
}

hipError_t launch_flag_compact(const SetDesc* sets, const WorkItem* items, const int* count,
                               WorkItem* out_items, int* out_count, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_compact, dim3(256), dim3(256), 0, s, sets, items, count, out_items,
                     out_count);
  return hipGetLastError();
}

__global__ void k_zero_int(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace sbv
