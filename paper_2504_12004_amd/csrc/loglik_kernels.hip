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
  return 68 * MF<T>::qof(c) + 17 * MF<T>::gof(c) + r;
}
// Offset of lane l's operand in chunk q of a tile: 68 q + oplane(l).
__device__ __forceinline__ int oplane(int lane) { return 17 * (lane >> 4) + (lane & 15); }

__device__ __forceinline__ double rlane(double v, int l) {
  unsigned long long u = (unsigned long long)__double_as_longlong(v);
  unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffull), l);
  unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float rlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// e^x for the covariance generation (x = -r <= 0): Cody and Waite's reduction
// x = k ln 2 + f, k = rint(x / ln 2), |f| <= ln(2) / 2, with ln 2 split into a
// 42-bit leading part (k ln2_hi is exact for |k| < 2^11) and the rest; then
// e^f = 1 + (f + f^2 P(f)), P the Taylor series of (e^f - 1 - f) / f^2 to
// degree 11 (truncation below 1e-17 relative), evaluated by Estrin's scheme:
// the dependent chain is 6 operations deep against Horner's 13 (the
// generation is latency-bound), and adding the 1 last keeps the error within
// one ulp; finally scaled by 2^k.  x is clamped at -1000, where e^x is 0.
__device__ __forceinline__ double t_exp(double x) {
  x = fmax(x, -1000.0);
  const double k = rint(x * 0x1.71547652b82fep+0);
  double f = fma(-k, 0x1.62e42fefa3800p-1, x);
  f = fma(-k, 0x1.ef35793c76730p-45, f);
  const double f2 = f * f, f4 = f2 * f2, f8 = f4 * f4;
  const double d0 = fma(f, 0x1.5555555555555p-3, 0x1.0000000000000p-1);
  const double d1 = fma(f, 0x1.1111111111111p-7, 0x1.5555555555555p-5);
  const double d2 = fma(f, 0x1.a01a01a01a01ap-13, 0x1.6c16c16c16c17p-10);
  const double d3 = fma(f, 0x1.71de3a556c734p-19, 0x1.a01a01a01a01ap-16);
  const double d4 = fma(f, 0x1.ae64567f544e4p-26, 0x1.27e4fb7789f5cp-22);
  const double d5 = fma(f, 0x1.6124613a86d09p-33, 0x1.1eed8eff8d898p-29);
  const double e0 = fma(d1, f2, d0), e1 = fma(d3, f2, d2), e2 = fma(d5, f2, d4);
  const double p = fma(e2, f8, fma(e1, f4, e0));
  return __builtin_amdgcn_ldexp(1.0 + fma(f2, p, f), (int)k);
}
__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float t_sqrt(float x) { return sqrtf(x); }
// Distance from its square in the covariance generation (r2 >= 0): the
// hardware reciprocal square root (about 23 good bits) refined by one coupled
// Newton-Raphson step for sqrt(r2) and 1/(2 sqrt(r2)) and one residual
// correction (Goldschmidt's square-root iteration as in Markstein's IA-64
// elementary functions), which lands within rounding of the library sqrt.
// Squared distances below 2^-1000 give 0: no covariance entry can tell them
// apart.  FP32 takes the one-instruction hardware sqrt (1 ulp).
__device__ __forceinline__ double g_sqrt(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  double g = r2 * y, h = 0.5 * y;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  g = fma(fma(-g, g, r2), h, g);
  return r2 < 0x1p-1000 ? 0.0 : g;
}
__device__ __forceinline__ float g_sqrt(float r2) { return __builtin_amdgcn_sqrtf(r2); }

// Scaled coordinates in LDS: one row of zld(d) elements per point (d rounded
// up to 16 bytes, zero padded), so that the covariance generation reads them
// as 16-byte vectors.
template <typename T>
struct ZV;
template <>
struct ZV<double> {
  typedef double v __attribute__((ext_vector_type(2)));
  static constexpr int w = 2;
};
template <>
struct ZV<float> {
  typedef float v __attribute__((ext_vector_type(4)));
  static constexpr int w = 4;
};
template <typename T>
__device__ __forceinline__ int zld(int d) {
  return (d + ZV<T>::w - 1) / ZV<T>::w * ZV<T>::w;
}

// Matern correlation, closed forms of Eq. (maternkernel) for half-integer nu:
// p(r) e^{-r} with p = 1, 1 + r, 1 + r + r^2/3, 1 + r + 2 r^2/5 + r^3/15 for
// nu = 1/2, 3/2, 5/2, 7/2, taken as 1 + r (c1 + r (c2 + r c3)) with the
// coefficients selected once from the (uniform) smoothness: no branch per
// entry, so that the covariance generation can interleave its entries.
template <typename T>
__device__ __forceinline__ T matern(T r, int two_nu) {
  const T c1 = two_nu >= 3 ? T(1) : T(0);
  const T c2 = two_nu == 5 ? T(1.0 / 3.0) : (two_nu == 7 ? T(0.4) : T(0));
  const T c3 = two_nu == 7 ? T(1.0 / 15.0) : T(0);
  return fma(r, fma(r, fma(r, c3, c2), c1), T(1)) * t_exp(-r);
}

constexpr double kLog2Pi = 1.83787706640934548356065947281123527;

// Phase profile (profiling builds only, -DSBV_PHASE_PROFILE): cycles spent by
// the panel wave (slots 0..7) and the first worker wave (slots 8..15) per
// phase, summed over blocks.
#ifdef SBV_PHASE_PROFILE
__device__ unsigned long long g_phase[16];
// per-workgroup accumulation in LDS (one writer per slot), flushed once per
// workgroup: keeps the counters' own cost out of the phases they time
#define SBV_PROF_DECL long long prof_t = clock64();
#define SBV_PROF(slot, cond)                                        \
  do {                                                              \
    long long now_ = clock64();                                     \
    if ((cond) && (threadIdx.x & 63) == 0) sm.prof[slot] += (unsigned long long)(now_ - prof_t); \
    prof_t = now_;                                                  \
  } while (0)
#else
#define SBV_PROF_DECL
#define SBV_PROF(slot, cond) \
  do {                       \
  } while (0)
#endif

// Row stride of the diagonal tile in LDS: 17 elements, so that the 16 rows
// (or columns) one instruction touches fall on different banks.
constexpr int kDiagLd = 17;

// Row stride of the right-hand-side chunk used by the adjoint solves (32
// columns plus one of padding so that rows fall on different LDS banks).
constexpr int kRS = 33;
constexpr int kChunk = 32;

// FP64 register kernels generate covariance columns late (interleaved with the
// factorisation, see worker_waves); FP32 ones generate them all first.
template <typename T>
constexpr bool kLateCov = sizeof(T) == 8;

template <typename T, int NTM, bool GRAD = false, bool LA = false, bool SMP = false>
struct Smem {
  static constexpr int kPanel = NTM * kOpT;
  static constexpr int kRhs = NTM * kTile * kRS;
  // lookahead: two column buffers (steps alternate) before the stage
  static constexpr int kPanelElems = LA ? 3 * kPanel : (GRAD && kRhs > 2 * kPanel) ? kRhs : 2 * kPanel;
  static constexpr int kStageTiles = kPanelElems / 256;  // staged covariance tiles that fit the panel
  alignas(16) T z[NTM * kTile * kMaxDim];  // scaled coordinates of A, rows of zld(d)
  T yv[NTM * kTile];           // observations, overwritten by the forward solve
  // column k of L in operand layout (factorisation; lookahead: columns k and
  // k-1, in buffers k&1); the part after it stages the next covariance
  // column; right-hand-side chunk of the adjoint solves (GRAD only)
  T panel[kPanelElems];
  T diag[16 * kDiagLd];        // diagonal tile to factor (row-major, padded rows)
  T negM[kOpT];                // -(L_kk^{-T}) in B-operand layout
  T zk[2 * kTile];             // solved z of the current tile row (lookahead: of rows k and k-1)
  T zfull[GRAD ? NTM * kTile : 1];  // all of z = L^{-1} y (GRAD only)
  T xi[NTM * kTile];                // innovations of the conditional simulator
  int la_flag;                      // lookahead: last diagonal step published
  int next_item;                    // work-queue mode: the item taken by this workgroup
  double isc[kMaxDim];              // exp(-theta_k) of the set being processed
#ifdef SBV_PHASE_PROFILE
  unsigned long long prof[16];
#endif
  T gv[GRAD ? NTM * kTile : 1];     // g = Q z_B accumulated over chunks (GRAD only)
  T vacc[SMP ? NTM * kTile : 1];    // conditional simulation: sum of L_rc^2 over the block's columns
};

// 1/sqrt(p): hardware reciprocal square root refined by Newton steps
// r <- r (3 - p r^2) / 2 (two for FP64, one for FP32).
__device__ __forceinline__ double rsqrt_nr(double p) {
  double r = __builtin_amdgcn_rsq(p);
  r = r * (1.5 - 0.5 * p * r * r);
  r = r * (1.5 - 0.5 * p * r * r);
  return r;
}
__device__ __forceinline__ float rsqrt_nr(float p) {
  float r = __builtin_amdgcn_rsqf(p);
  return r * (1.5f - 0.5f * p * r * r);
}

__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float shfl_d(float v, int src) { return __shfl(v, src, 64); }

// Lane j of every 16-lane row broadcast to its row (DPP row_newbcast, j a
// constant after unrolling), and row gj broadcast to all four rows
// (v_permlane16_swap then v_permlane32_swap).  Both checked on the device.
// Every lane of a row broadcast has a valid source, so the old value is never
// kept; bound_ctrl with old = 0 says so and lets the compiler write the
// broadcast into a fresh register instead of copying the source first.
template <int J>
__device__ __forceinline__ unsigned nb_u(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + J, 0xf, 0xf, true);
}
__device__ __forceinline__ unsigned row_lane_u(unsigned v, int j) {
  switch (j) {
    case 0: return nb_u<0>(v);
    case 1: return nb_u<1>(v);
    case 2: return nb_u<2>(v);
    case 3: return nb_u<3>(v);
    case 4: return nb_u<4>(v);
    case 5: return nb_u<5>(v);
    case 6: return nb_u<6>(v);
    case 7: return nb_u<7>(v);
    case 8: return nb_u<8>(v);
    case 9: return nb_u<9>(v);
    case 10: return nb_u<10>(v);
    case 11: return nb_u<11>(v);
    case 12: return nb_u<12>(v);
    case 13: return nb_u<13>(v);
    case 14: return nb_u<14>(v);
    default: return nb_u<15>(v);
  }
}
__device__ __forceinline__ unsigned row_all_u(unsigned x, int gj) {
  const auto a = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows (0 0 2 2) / (1 1 3 3)
  const unsigned e = (gj & 1) ? a[1] : a[0];
  const auto b = __builtin_amdgcn_permlane32_swap(e, e, false, false);   // lower / upper half doubled
  return (gj & 2) ? b[1] : b[0];
}
// FP64: one 64-bit DPP move (v_mov_b64 row_newbcast, checked on the device)
template <int J>
__device__ __forceinline__ double nb_d(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + J, 0xf, 0xf, true);
}
__device__ __forceinline__ double row_lane(double v, int j) {
  switch (j) {
    case 0: return nb_d<0>(v);
    case 1: return nb_d<1>(v);
    case 2: return nb_d<2>(v);
    case 3: return nb_d<3>(v);
    case 4: return nb_d<4>(v);
    case 5: return nb_d<5>(v);
    case 6: return nb_d<6>(v);
    case 7: return nb_d<7>(v);
    case 8: return nb_d<8>(v);
    case 9: return nb_d<9>(v);
    case 10: return nb_d<10>(v);
    case 11: return nb_d<11>(v);
    case 12: return nb_d<12>(v);
    case 13: return nb_d<13>(v);
    case 14: return nb_d<14>(v);
    default: return nb_d<15>(v);
  }
}
__device__ __forceinline__ float row_lane(float v, int j) { return __uint_as_float(row_lane_u(__float_as_uint(v), j)); }
__device__ __forceinline__ double row_all(double v, int gj) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = row_all_u((unsigned)u, gj), hi = row_all_u((unsigned)(u >> 32), gj);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float row_all(float v, int gj) { return __uint_as_float(row_all_u(__float_as_uint(v), gj)); }

// Sum of the four rows' values at the same position within the row, left in
// every row: rows (0 1 2 3) -> permlane16_swap pairs (0,1) and (2,3), then
// permlane32_swap pairs the two halves.
__device__ __forceinline__ double rows_sum(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
  const double s1 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
                    __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  const unsigned long long w = (unsigned long long)__double_as_longlong(s1);
  const auto lo2 = __builtin_amdgcn_permlane32_swap((unsigned)w, (unsigned)w, false, false);
  const auto hi2 = __builtin_amdgcn_permlane32_swap((unsigned)(w >> 32), (unsigned)(w >> 32), false, false);
  return __longlong_as_double((long long)(((unsigned long long)hi2[0] << 32) | lo2[0])) +
         __longlong_as_double((long long)(((unsigned long long)hi2[1] << 32) | lo2[1]));
}
__device__ __forceinline__ float rows_sum(float v) {
  const unsigned u = __float_as_uint(v);
  const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  const float s1 = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const unsigned w = __float_as_uint(s1);
  const auto b = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Factor the 16x16 SPD tile in sm.diag on one wave with all 64 lanes: lane
// (r, g) = (l % 16, l / 16) holds columns c = g + 4q (q = 0..3) of row r.
// Right-looking pivots; by symmetry of the trailing matrix the column-j
// entries L[c][j] a lane needs are row j's entries of its own columns, read
// from lane (j, g).  Every update of step j takes the one multiplier
// L[r][j] / L[j][j] per row.  The same loop eliminates the rows of W, the
// inverse X = L^{-1} with its rows not yet divided by their pivots (lane (r, g)
// holds W[r][g + 4q], starting from the identity): row j of X is W[j] / L[j][j],
// so its elimination from row r is W[r] -= (L[r][j] / L[j][j]) W[j], and the
// division of every row by its pivot is left to the end.  Then
// z_k = L_kk^{-1} y_k = X y_k and -X^T is published for the column solves.
// Lanes r < 16 return the pivot L_rr and z_r.  Each lane keeps its row's pivot
// before the square root; after the loop `bad` is raised for a non-positive or
// non-finite pivot and `low` for a pivot at or below tau * original diagonal
// (the FP32 fallback test).
template <typename T, bool SAMPLE = false, class SM>
__device__ __forceinline__ void factor_diag(SM& sm, T* negM_out, int lane, int k, int nreal, T diag0, T tau,
                                            T& pivot_out, T& z_out, int& bad, int& low, int mi = 0,
                                            T* ysim = nullptr, T* vacc = nullptr) {
  // The lane index passes through an empty asm statement, so that the
  // compiler cannot hoist the lane-against-constant comparisons of the
  // unrolled steps out of the callers' tile loops: kept live there, they
  // exhausted the scalar registers and spilled (to vector lanes and scratch).
  int ln = lane;
  __asm__ volatile("" : "+v"(ln));
  const int r = ln & 15, g = ln >> 4;
  T a[4], w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = g + 4 * q;
    a[q] = sm.diag[r * kDiagLd + c];
    w[q] = (c == r) ? T(1) : T(0);
  }
  T yr = sm.yv[kTile * k + r];
  T pv = T(1);  // this lane's row pivot, before the square root
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int gj = j & 3, qj = j >> 2;
    const T piv = rlane(a[qj], j + 16 * gj);
    pv = (r == j) ? piv : pv;
    const T rs = rsqrt_nr(piv);
    const T sq = piv * rs;
    // A[r][j] of my row and row j of my columns, before this step's update.
    // Register q holds columns 4q..4q+3 (q and j are constants after
    // unrolling): it is final once 4q + 3 < j, lies wholly right of the pivot
    // once 4q > j, and holds column j for q = qj.
    const T arj = row_all(a[qj], gj);
    T ajc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * q + 3 > j) ajc[q] = row_lane(a[q], j);
    const T lrj = (r == j) ? sq : arj * rs;   // L[r][j] (r >= j)
    const T lrs = (r > j) ? lrj * rs : T(0);  // L[r][j] / L[j][j] below the pivot, 0 elsewhere
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (4 * q + 3 < j) continue;
      if (4 * q > j) {
        a[q] -= lrs * ajc[q];
      } else {
        const int c = g + 4 * q;
        if (c > j) a[q] = (r > j) ? a[q] - lrs * ajc[q] : a[q];
        if (c == j) a[q] = (r >= j) ? lrj : a[q];
      }
    }
    // W[j][c] = 0 for c > j, so registers with 4q > j take no part
    T wjc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * q <= j) wjc[q] = row_lane(w[q], j);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * q <= j) w[q] -= lrs * wjc[q];
    if (SAMPLE) {
      T zj;
      // conditional simulation: rows of J are solved (w = z), rows of B take
      // w = xi and emit y = L_jj xi - v, v being the eliminated part so far
      const int R = kTile * k + j;
      const T vj = rlane(yr, j);
      if (R < mi) {
        zj = vj * rs;
      } else {
        const T xj = sm.xi[R];
        zj = xj;
        if (r == j) *ysim = sq * xj - vj;
      }
      yr = (r == j) ? zj : (r > j ? yr - lrj * zj : yr);
    }
  }
  if (__any(!(pv > T(0)) || !(pv == pv) || pv > T(3.0e38))) bad = 1;
  if (__any(pv <= tau * (r < nreal ? diag0 : T(1)))) low = 1;
  // rows of X: W[r] / L[r][r]
  const T rsr = rsqrt_nr(pv);
  T x[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) x[q] = w[q] * rsr;
  if (SAMPLE && vacc) {
    // conditional variance of the block's rows of this tile: the within-tile
    // part of sum over the block's columns c <= r of L[r][c]^2 (columns of
    // earlier tiles were added by var_update)
    T part = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = g + 4 * q;
      if (c <= r && kTile * k + c >= mi) part += a[q] * a[q];
    }
    const T vs = rows_sum(part);
    if (g == 0 && kTile * k + r >= mi) vacc[kTile * k + r] += vs;
  }
  if (!SAMPLE) {
    // z_k = L_kk^{-1} y_k = X y_k: lane (r, g) sums X[r][c] y[c] over its
    // columns c = g + 4q, then the four row groups are added
    T part = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) part += x[q] * sm.yv[kTile * k + g + 4 * q];
    yr = rows_sum(part);
  }
  // pivot L_rr lives in lane (r, r % 4), register r / 4
  T mine = a[0];
#pragma unroll
  for (int q = 1; q < 4; ++q) mine = ((r >> 2) == q) ? a[q] : mine;
  pivot_out = shfl_d(mine, r + 16 * (r & 3));
  z_out = yr;
  // -X^T in B-operand layout: element X[a][b] at opoff(a, b)
#pragma unroll
  for (int q = 0; q < 4; ++q) negM_out[opoff<T>(r, g + 4 * q)] = -x[q];
}

// N work items of gen_column computed together (independent chains for the
// exp/sqrt latency): item e = (tile i0 + e/64, lane e%64), 4 entries each.
template <typename T, int N, class SM>
__device__ __forceinline__ void gen_items(SM& sm, T* dst, const int (&e)[N], int j, int i0, int nA, int d,
                                          int two_nu, T sigma2, T tau2) {
  int i[N], l[N], pb[N], pbc[N], pa[N][4], pac[N][4];
  T r2[N][4];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    i[n] = i0 + (e[n] >> 6);
    l[n] = e[n] & 63;
    pb[n] = kTile * i[n] + (l[n] & 15);
    pbc[n] = pb[n] < nA ? pb[n] : 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      pa[n][t] = kTile * j + MF<T>::row(l[n] >> 4, t);
      pac[n][t] = pa[n][t] < nA ? pa[n][t] : 0;
      r2[n][t] = T(0);
    }
  }
  typedef typename ZV<T>::v zv;
  const int ld = zld<T>(d);
  for (int k = 0; k < ld; k += ZV<T>::w) {
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const zv zb = *reinterpret_cast<const zv*>(sm.z + pbc[n] * ld + k);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const zv df = *reinterpret_cast<const zv*>(sm.z + pac[n][t] * ld + k) - zb;
#pragma unroll
        for (int c = 0; c < ZV<T>::w; ++c) r2[n][t] += df[c] * df[c];
      }
    }
  }
#pragma unroll
  for (int n = 0; n < N; ++n)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // padding rows and columns (beyond nA) take the identity; the entry is
      // computed either way (from clamped points) and selected, so that no
      // branch splits the straight-line code of the items
      T v = -(sigma2 * matern<T>(g_sqrt(r2[n][t]), two_nu));
      if (pa[n][t] == pb[n]) v -= tau2;
      const T pad = (pa[n][t] == pb[n]) ? T(-1) : T(0);
      dst[256 * i[n] + 64 * t + l[n]] = (pa[n][t] >= nA || pb[n] >= nA) ? pad : v;
    }
}

template <typename T, int NTHR, class SM>
__device__ __forceinline__ void gen_column(SM& sm, T* dst, int tid, int j, int i0, int nt, int nA, int d,
                                           int two_nu, T sigma2, T tau2) {
  // tiles (i, j) for i = i0..nt-1.  One work item = (tile i, lane l): the 4
  // entries of accumulator registers t = 0..3, which share the point
  // 16i + l%16 (read once) and differ in the point 16j + row(l/16, t); a
  // thread takes its items two at a time
  const int total = (nt - i0) * 64;
  int e = tid;
  for (; e + NTHR < total; e += 2 * NTHR) {
    const int ee[2] = {e, e + NTHR};
    gen_items<T, 2>(sm, dst, ee, j, i0, nA, d, two_nu, sigma2, tau2);
  }
  if (e < total) {
    const int ee[1] = {e};
    gen_items<T, 1>(sm, dst, ee, j, i0, nA, d, two_nu, sigma2, tau2);
  }
}

// Covariance tiles (i, j) of the columns j0 <= j < j1 (i >= j), numbered
// column by column from 0 and staged at dst + 256 u in the same per-tile order
// as gen_column; two work items per thread in flight.
template <typename T, class SM>
__device__ __forceinline__ void group_tile(int u, int j0, int nt, int& i, int& j) {
  j = j0;
  while (u >= nt - j) {
    u -= nt - j;
    ++j;
  }
  i = j + u;
}
template <typename T, int NTHR, class SM>
__device__ __forceinline__ void gen_group(SM& sm, T* dst, int tid, int j0, int j1, int nt, int nA, int d, int two_nu,
                                         T sigma2, T tau2) {
  int tiles = 0;
  for (int j = j0; j < j1; ++j) tiles += nt - j;
  const int total = 64 * tiles;
  auto one = [&](int e, T (&v)[4], int& u, int& l) {
    int i, j;
    u = e >> 6;
    l = e & 63;
    group_tile<T, SM>(u, j0, nt, i, j);
    const int pb = kTile * i + (l & 15);
    const int pbc = pb < nA ? pb : 0;
    int pa[4], pac[4];
    T r2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      pa[t] = kTile * j + MF<T>::row(l >> 4, t);
      pac[t] = pa[t] < nA ? pa[t] : 0;
      r2[t] = T(0);
    }
    typedef typename ZV<T>::v zv;
    const int ld = zld<T>(d);
    for (int k = 0; k < ld; k += ZV<T>::w) {
      const zv zb = *reinterpret_cast<const zv*>(sm.z + pbc * ld + k);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const zv df = *reinterpret_cast<const zv*>(sm.z + pac[t] * ld + k) - zb;
#pragma unroll
        for (int c = 0; c < ZV<T>::w; ++c) r2[t] += df[c] * df[c];
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // as in gen_items: computed from clamped points, padding selected
      T c = -(sigma2 * matern<T>(g_sqrt(r2[t]), two_nu));
      if (pa[t] == pb) c -= tau2;
      const T pad = (pa[t] == pb) ? T(-1) : T(0);
      v[t] = (pa[t] >= nA || pb >= nA) ? pad : c;
    }
  };
  int e = tid;
  for (; e + NTHR < total; e += 2 * NTHR) {
    T v0[4], v1[4];
    int u0, l0, u1, l1;
    one(e, v0, u0, l0);
    one(e + NTHR, v1, u1, l1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      dst[256 * u0 + 64 * t + l0] = v0[t];
      dst[256 * u1 + 64 * t + l1] = v1[t];
    }
  }
  if (e < total) {
    T v0[4];
    int u0, l0;
    one(e, v0, u0, l0);
#pragma unroll
    for (int t = 0; t < 4; ++t) dst[256 * u0 + 64 * t + l0] = v0[t];
  }
}

// Next group of whole columns [j0, j1) whose tiles fit `cap` staged tiles.
__device__ __forceinline__ int group_end(int j0, int nt, int cap) {
  int j1 = j0, tiles = 0;
  while (j1 < nt && tiles + (nt - j1) <= cap) {
    tiles += nt - j1;
    ++j1;
  }
  return j1 > j0 ? j1 : j0 + 1;
}

// Forward-solve update of the observations in rows r0..r1-1 with the column
// tile of L staged in the panel: y_rho -= L[rho][16k..16k+15] z_k, four rows
// per lane as independent chains (y_update: rows r0..16nt-1 with z_k from LDS).
template <typename T, int IT, class SM>
__device__ __forceinline__ void y_update_rows_t(SM& sm, const T* P, int lane, int r0, int r1, const T (&zk)[16]) {
  for (int base = r0; base < r1; base += 64 * IT) {
    T v[IT];
    int rho[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      rho[it] = base + lane + 64 * it;
      v[it] = rho[it] < r1 ? sm.yv[rho[it]] : T(0);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int rr = rho[it] < r1 ? rho[it] : r0;
        v[it] -= P[kOpT * (rr >> 4) + opoff<T>(rr & 15, c)] * zk[c];
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it)
      if (rho[it] < r1) sm.yv[rho[it]] = v[it];
  }
}
// (as many rows per lane as the range needs, up to four)
template <typename T, class SM>
__device__ __forceinline__ void y_update_rows(SM& sm, const T* P, int lane, int r0, int r1, const T (&zk)[16]) {
  const int rows = r1 - r0;
  if (rows > 128)
    y_update_rows_t<T, 4>(sm, P, lane, r0, r1, zk);
  else if (rows > 64)
    y_update_rows_t<T, 2>(sm, P, lane, r0, r1, zk);
  else if (rows > 0)
    y_update_rows_t<T, 1>(sm, P, lane, r0, r1, zk);
}
template <typename T, class SM>
__device__ __forceinline__ void y_update(SM& sm, int lane, int r0, int nt) {
  T zk[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) zk[c] = sm.zk[c];
  y_update_rows<T>(sm, sm.panel, lane, r0, kTile * nt, zk);
}
// Rows r0..r1-1 with the column in panel buffer b and z from zk buffer b
// (lookahead schedule).
template <typename T, int KP, class SM>
__device__ __forceinline__ void y_update_buf(SM& sm, int b, int lane, int r0, int r1) {
  T zk[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) zk[c] = sm.zk[kTile * b + c];
  y_update_rows<T>(sm, sm.panel + KP * b, lane, r0, r1, zk);
}
// The 16 rows of tile kt only: lane (r, g) sums columns 4g..4g+3 of row r,
// rows_sum adds the four partial sums.
template <typename T, int KP, class SM>
__device__ __forceinline__ void y_update_tile(SM& sm, int b, int lane, int kt) {
  const int r = lane & 15, g = lane >> 4;
  const T* P = sm.panel + KP * b + kOpT * kt;
  T part = T(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) part += P[opoff<T>(r, 4 * g + q)] * sm.zk[kTile * b + 4 * g + q];
  const T sum = rows_sum(part);
  if (g == 0) sm.yv[kTile * kt + r] -= sum;
}

// Stage column tile k of a large block's prefix panel (nt tiles of L below
// the prefix, operand layout, written by the prefix kernel) and z_k.
template <typename T, int NTHR, class SM>
__device__ __forceinline__ void load_prefix(SM& sm, int tid, int k, int nt, const T* W, const T* zp) {
  const T* src = W + (int64_t)k * kLargeNTM * kOpT;
  for (int e = tid; e < nt * kOpT; e += NTHR) sm.panel[e] = src[e];
  if (tid < kTile) sm.zk[tid] = zp[kTile * k + tid];
}

// Conditional simulation with variances: rows below tile k add the squares of
// their entries of L in the block's columns of tile k (column tile k of L
// staged in the panel); rows below a column of the block are block rows.
template <typename T, class SM>
__device__ __forceinline__ void var_update(SM& sm, int lane, int k, int nt, int mi) {
  if (kTile * k + kTile <= mi) return;  // no column of the block in this tile
  const int c0 = mi > kTile * k ? mi - kTile * k : 0;
  for (int rho = kTile * (k + 1) + lane; rho < kTile * nt; rho += 64) {
    T s = T(0);
    for (int c = c0; c < kTile; ++c) {
      const T v = sm.panel[kOpT * (rho >> 4) + opoff<T>(rho & 15, c)];
      s += v * v;
    }
    sm.vacc[rho] += s;
  }
}

// Panel wave: for every tile step factors the diagonal tile, solves the 16
// entries of z, accumulates the trailing log-pivots and z^2 in FP64, and
// applies the forward-solve update to the observations below.  In GRAD mode it
// also keeps all of z and then takes part in the adjoint solves (barriers,
// right-hand-side set-up and write-back).
template <typename T, int NTM, int NTHR, bool GRAD, bool SAMPLE, bool PRE, class SM>
__device__ __forceinline__ void panel_wave(SM& sm, int lane, int nt, int mi, int nA, int d, int two_nu, T sigma2,
                                           T tau2, T tau, double& ld_acc, double& q_acc, int& bad, int& low,
                                           double* yout, int p, const T* Wp, const T* zp, double* vout = nullptr) {
  const T diag0 = sigma2 + tau2;
  SBV_PROF_DECL
  if (!kLateCov<T>) {
    for (int j0 = 0; j0 < nt;) {
      const int j1 = group_end(j0, nt, Smem<T, NTM, GRAD>::kStageTiles);
      gen_group<T, NTHR>(sm, sm.panel, lane, j0, j1, nt, nA, d, two_nu, sigma2, tau2);
      __syncthreads();  // G1
      __syncthreads();  // G2
      j0 = j1;
    }
  }
  if (PRE) {
    // large block: y -= L_RP z_P, one prefix column tile at a time
    for (int k = 0; k < p; ++k) {
      load_prefix<T, NTHR>(sm, lane, k, nt, Wp, zp);
      __syncthreads();  // P1: prefix column k staged
      y_update<T>(sm, lane, 0, nt);
      __syncthreads();  // P2: staging area free
    }
  }
  if (kLateCov<T>) __syncthreads();  // G0: covariance column 0 staged (by the workers)
  SBV_PROF(0, true);
  for (int k = 0; k < nt; ++k) {
    __syncthreads();  // S1: diagonal tile published
    SBV_PROF(1, true);
    T piv, zr, ysim = T(0);
    // the serial diagonal factorisations are the critical path: they win issue
    // arbitration against the worker that shares this SIMD
    __builtin_amdgcn_s_setprio(2);
    T* vacc = nullptr;
    if constexpr (SAMPLE) vacc = vout ? sm.vacc : nullptr;
    factor_diag<T, SAMPLE>(sm, sm.negM, lane, k, nA - kTile * k, diag0, tau, piv, zr, bad, low, mi, &ysim, vacc);
    __builtin_amdgcn_s_setprio(0);
    const int rowg = kTile * k + lane;
    if (SAMPLE && lane < 16 && rowg >= mi && rowg < nA) {
      yout[rowg - mi] = (double)ysim;
      if constexpr (SAMPLE)
        if (vout) vout[rowg - mi] = (double)sm.vacc[rowg];
    }
    if (lane < 16) {
      sm.zk[lane] = zr;
      if (GRAD) sm.zfull[rowg] = zr;
      if (rowg >= mi && rowg < nA) {
        ld_acc += log((double)piv);
        q_acc += (double)zr * (double)zr;
      }
    }
    SBV_PROF(2, true);
    __syncthreads();  // S2: -L_kk^{-T} and z_k published
    __syncthreads();  // S3: column k of L published
    SBV_PROF(3, true);
    y_update<T>(sm, lane, kTile * (k + 1), nt);
    if constexpr (SAMPLE)
      if (vout) var_update<T>(sm, lane, k, nt, mi);
    SBV_PROF(4, true);
  }
}


// Re-derive the (wave-uniform) slot coordinates at the top of a loop body so
// that the compiler recomputes per-slot LDS addresses inside the loop instead
// of hoisting all of them into registers for the whole loop.
template <int SLOTS>
__device__ __forceinline__ void refresh_slots(int* ti, int* tj) {
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    int a = ti[s], b = tj[s];
    asm volatile("" : "+v"(a), "+v"(b));
    ti[s] = __builtin_amdgcn_readfirstlane(a);
    tj[s] = __builtin_amdgcn_readfirstlane(b);
  }
}

// ---- lookahead schedule (forward log-likelihood only) ----------------------
// The owner of the next diagonal tile updates it first in the trailing update
// of step k and publishes it with an LDS flag; the panel wave factors it while
// the workers finish step k.  Two barriers per step instead of three.
template <typename T, int NTM, int NTHR, class SM>
__device__ __forceinline__ void panel_wave_la(SM& sm, int lane, int nt, int mi, int nA, int d, int two_nu, T sigma2, T tau2, T tau,
                              double& ld_acc, double& q_acc, int& bad, int& low) {
  const T diag0 = sigma2 + tau2;
  SBV_PROF_DECL
  if (kLateCov<T>) {
    __syncthreads();  // Ga: covariance column 0 staged
    __syncthreads();  // Gb: column 0 added, diagonal tile 0 published
  } else {
    for (int j0 = 0; j0 < nt;) {
      const int j1 = group_end(j0, nt, Smem<T, NTM, false, true>::kStageTiles);
      gen_group<T, NTHR>(sm, sm.panel, lane, j0, j1, nt, nA, d, two_nu, sigma2, tau2);
      __syncthreads();  // G1
      __syncthreads();  // G2
      j0 = j1;
    }
  }
  constexpr int KP = Smem<T, NTM, false, true>::kPanel;
  auto factor_step = [&](int k) {
    while (__atomic_load_n(&sm.la_flag, __ATOMIC_ACQUIRE) < k) __builtin_amdgcn_s_sleep(1);
    SBV_PROF(3, true);
    T piv, zr;
    __builtin_amdgcn_s_setprio(2);
    factor_diag<T>(sm, sm.negM, lane, k, nA - kTile * k, diag0, tau, piv, zr, bad, low);
    __builtin_amdgcn_s_setprio(0);
    const int rowg = kTile * k + lane;
    if (lane < 16) {
      sm.zk[kTile * (k & 1) + lane] = zr;
      if (rowg >= mi && rowg < nA) {
        ld_acc += log((double)piv);
        q_acc += (double)zr * (double)zr;
      }
    }
    SBV_PROF(4, true);
  };
  SBV_PROF(0, true);
  factor_step(0);
  __syncthreads();  // P0: step 0 factored
  SBV_PROF(5, true);
  // The forward-solve update of column k is split: the rows of tile k+1 go
  // right after S3 (factor k+1 needs them), the rows below after S4, from the
  // other column buffer, while the workers solve column k+1.
  for (int k = 0; k < nt; ++k) {
    if (k >= 1) y_update_buf<T, KP>(sm, (k - 1) & 1, lane, kTile * (k + 1), kTile * nt);
    SBV_PROF(2, true);
    __syncthreads();  // S3: column k of L published
    SBV_PROF(1, true);
    if (k + 1 < nt) {
      y_update_tile<T, KP>(sm, k & 1, lane, k + 1);
      SBV_PROF(2, true);
      factor_step(k + 1);
    }
    __syncthreads();  // S4: trailing update and next diagonal done
    SBV_PROF(5, true);
  }
}

template <typename T, int NTM, int NWK, int NTHR, class SM>
__device__ __forceinline__ void worker_waves_la(SM& sm, int wk, int lane, int nt, int nA, int d, int two_nu, T sigma2, T tau2) {
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
    ti[s] = __builtin_amdgcn_readfirstlane(i);
    tj[s] = __builtin_amdgcn_readfirstlane(j);
  }
  acc_t acc[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[s][t] = T(0);
  }
  // FP64: covariance column j is staged by the workers during step j-2 (after
  // their updates, while the panel wave factors) and added by its owners at
  // the start of step j-1, before that step's update and early publication
  // of the diagonal tile j; columns 0 and 1 are staged up front.  FP32
  // generates every column first (see worker_waves).
  constexpr int KP = Smem<T, NTM, false, true>::kPanel;
  T* stage = sm.panel + 2 * KP;
  const int wrank = wk == 3 ? NWK - 1 : (wk > 3 ? wk - 1 : wk);  // wave 4 last, as above
  const int wtid = 64 * wrank + lane;
  SBV_PROF_DECL
  auto add_staged = [&](int j) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] == j) {
        const T* src = stage + 256 * ti[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[s][t] += src[64 * t + lane];
      }
    }
  };
  if (kLateCov<T>) {
    gen_column<T, NTHR - 64>(sm, stage, wtid, 0, 0, nt, nA, d, two_nu, sigma2, tau2);
    __syncthreads();  // Ga
    refresh_slots<SLOTS>(ti, tj);
    add_staged(0);
  } else {
    for (int j0 = 0; j0 < nt;) {
      const int j1 = group_end(j0, nt, Smem<T, NTM, false, true>::kStageTiles);
      refresh_slots<SLOTS>(ti, tj);
      gen_group<T, NTHR>(sm, sm.panel, 64 * (wk + 1) + lane, j0, j1, nt, nA, d, two_nu, sigma2, tau2);
      __syncthreads();  // G1
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (tj[s] >= j0 && tj[s] < j1) {
          const int u = (tj[s] - j0) * nt - (tj[s] * (tj[s] - 1) - j0 * (j0 - 1)) / 2 + (ti[s] - tj[s]);
          const T* src = sm.panel + 256 * u;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[s][t] = src[64 * t + lane];
        }
      }
      __syncthreads();  // G2
      j0 = j1;
    }
  }
  auto publish_diag = [&](int s, int k) {
#pragma unroll
    for (int t = 0; t < 4; ++t) sm.diag[cl * kDiagLd + MF<T>::row(g, t)] = -acc[s][t];
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) __atomic_store_n(&sm.la_flag, k, __ATOMIC_RELEASE);
  };
#pragma unroll
  for (int s = 0; s < SLOTS; ++s)
    if (ti[s] == 0 && tj[s] == 0) publish_diag(s, 0);
  if (kLateCov<T>) {
    __syncthreads();  // Gb: stage free again
    if (nt > 1) gen_column<T, NTHR - 64>(sm, stage, wtid, 1, 1, nt, nA, d, two_nu, sigma2, tau2);
  }
  __syncthreads();  // P0
  SBV_PROF(8, wk == 0);
  for (int k = 0; k < nt; ++k) {
    refresh_slots<SLOTS>(ti, tj);
    if (kLateCov<T>) add_staged(k + 1);  // staged during the previous step (or up front)
    T* const Pk = sm.panel + KP * (k & 1);  // column k of L
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] == k && ti[s] > k) {
        // two independent MFMA chains (q even, q odd) halve the dependent latency
        acc_t o = {T(0), T(0), T(0), T(0)}, o2 = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 4; q += 2) {
          o = MF<T>::mma(acc[s][q], sm.negM[68 * q + oplane(lane)], o);
          o2 = MF<T>::mma(acc[s][q + 1], sm.negM[68 * (q + 1) + oplane(lane)], o2);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) o[t] += o2[t];
        acc[s] = o;
        T* P = Pk + kOpT * ti[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) P[opoff<T>(MF<T>::row(g, t), cl)] = o[t];
      }
    }
    SBV_PROF(9, wk == 0);
    __syncthreads();  // S3
    SBV_PROF(10, wk == 0);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] > k) {
        const T* Pj = Pk + kOpT * tj[s];
        const T* Pi = Pk + kOpT * ti[s];
        acc_t o = acc[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) o = MF<T>::mma(Pj[68 * q + oplane(lane)], Pi[68 * q + oplane(lane)], o);
        acc[s] = o;
        if (ti[s] == k + 1 && tj[s] == k + 1) publish_diag(s, k + 1);
      }
    }
    SBV_PROF(11, wk == 0);
    // covariance column k+2 while the panel wave factors diagonal tile k+1
    if (kLateCov<T> && k + 2 < nt)
      gen_column<T, NTHR - 64>(sm, stage, wtid, k + 2, k + 2, nt, nA, d, two_nu, sigma2, tau2);
    SBV_PROF(12, wk == 0);
    __syncthreads();  // S4
    SBV_PROF(13, wk == 0);
  }
}

// Right-hand sides of the adjoint solves, as one list of columns:
// column 0 is [z_J; 0] (its solution is e = [Sigma_J^{-1} y_J; 0]) and column
// c >= 1 is the unit vector of row mi + c - 1 (their solutions are the columns
// of Q = L^{-T} [0; I_b]).
template <typename T, int NTHR, class SM>
__device__ void rhs_init(SM& sm, int tid, int ch, int nt, int mi, int bi) {
  for (int e = tid; e < nt * kTile * kChunk; e += NTHR) {
    const int r = e / kChunk, c = e - r * kChunk;
    const int col = kChunk * ch + c;
    T v = T(0);
    if (col == 0) v = r < mi ? sm.zfull[r] : T(0);
    else if (col <= bi && r == mi + col - 1) v = T(1);
    sm.panel[r * kRS + c] = v;
  }
}

// After the solves of one chunk: accumulate g = Q z_B, write e / Q columns of
// this block to its slice of the adjoint buffer (e, g, then Q column-major,
// column stride ld: the joint size; a large block's trailing part writes rows
// from its prefix length on, through an offset `out`).
template <typename T, int NTHR, class SM>
__device__ void rhs_writeback(SM& sm, int tid, int ch, int mi, int nA, int bi, int ld, T* out) {
  for (int r = tid; r < nA; r += NTHR) {
    T gacc = sm.gv[r];
#pragma unroll 4
    for (int c = 0; c < kChunk; ++c) {
      const int col = kChunk * ch + c;
      if (col > bi) break;
      const T v = sm.panel[r * kRS + c];
      if (col == 0) {
        out[r] = v;
      } else {
        gacc += v * sm.zfull[mi + col - 1];
        out[(int64_t)(2 + col - 1) * ld + r] = v;
      }
    }
    sm.gv[r] = gacc;
  }
}

// Worker waves: own the register tiles, build them from the covariance, and
// run the column TRSMs and trailing MFMA updates of every step.  In GRAD mode
// the finished factor stays in the slots (diagonal slots take L_kk^{-1}) and
// the workers run the backward solves L^T X = R chunk by chunk.
template <typename T, int NTM, int NWK, int NTHR, bool GRAD, bool PRE, class SM>
__device__ __forceinline__ void worker_waves(SM& sm, int wk, int lane, int nt, int mi, int nA, int bi, int d,
                                             int two_nu, T sigma2, T tau2, T* gout, int ld, int p, const T* Wp,
                                             const T* zp) {
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
    ti[s] = __builtin_amdgcn_readfirstlane(i);
    tj[s] = __builtin_amdgcn_readfirstlane(j);
  }
  // A slot holds G = sum_k L_ik L_jk^T - Sigma_ij.  In FP64 (kLateCov) the
  // two parts are added in any order: slots start at zero and tile column j of
  // Sigma is generated just before it is needed -- column 0 up front, column
  // k+1 while the panel wave factors diagonal tile k (the workers would
  // otherwise wait there).  In FP32 every column is generated first, so that
  // the running sums shrink towards the Schur complement instead of growing
  // towards Sigma (FP32 rounding of the updates stays relative to the smaller
  // value).
  acc_t acc[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[s][t] = T(0);
  }
  SBV_PROF_DECL
  if (!kLateCov<T>) {
    // every thread of the workgroup builds groups of whole columns into LDS,
    // owners copy theirs in
    for (int j0 = 0; j0 < nt;) {
      const int j1 = group_end(j0, nt, Smem<T, NTM, GRAD>::kStageTiles);
      refresh_slots<SLOTS>(ti, tj);
      gen_group<T, NTHR>(sm, sm.panel, 64 * (wk + 1) + lane, j0, j1, nt, nA, d, two_nu, sigma2, tau2);
      __syncthreads();  // G1: columns j0..j1-1 staged
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (tj[s] >= j0 && tj[s] < j1) {
          // tiles before column tj[s] in the group: sum_{j=j0}^{tj-1} (nt - j)
          const int u = (tj[s] - j0) * nt - (tj[s] * (tj[s] - 1) - j0 * (j0 - 1)) / 2 + (ti[s] - tj[s]);
          const T* src = sm.panel + 256 * u;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[s][t] = src[64 * t + lane];
        }
      }
      __syncthreads();  // G2: staging area free
      j0 = j1;
    }
  }
  if (PRE) {
    // large block: G += L_RP L_RP^T, one prefix column tile at a time
    for (int k = 0; k < p; ++k) {
      load_prefix<T, NTHR>(sm, 64 * (wk + 1) + lane, k, nt, Wp, zp);
      __syncthreads();  // P1
      refresh_slots<SLOTS>(ti, tj);
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (tj[s] >= 0) {
          const T* Pj = sm.panel + kOpT * tj[s];
          const T* Pi = sm.panel + kOpT * ti[s];
          acc_t o = acc[s];
#pragma unroll
          for (int q = 0; q < 4; ++q) o = MF<T>::mma(Pj[68 * q + oplane(lane)], Pi[68 * q + oplane(lane)], o);
          acc[s] = o;
        }
      }
      __syncthreads();  // P2
    }
  }
  // covariance column j is staged by the workers in the second half of the
  // panel (`stage`) and added by the owners of its tiles
  T* stage = sm.panel + Smem<T, NTM, GRAD>::kPanel;
  // generation work goes to worker 3 (wave 4, which shares its SIMD with the
  // panel wave's diagonal factorisations) last
  const int wrank = wk == 3 ? NWK - 1 : (wk > 3 ? wk - 1 : wk);
  const int wtid = 64 * wrank + lane;
  if (kLateCov<T>) {
    gen_column<T, NTHR - 64>(sm, stage, wtid, 0, 0, nt, nA, d, two_nu, sigma2, tau2);
    __syncthreads();  // G0: covariance column 0 staged
    refresh_slots<SLOTS>(ti, tj);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] == 0) {
        const T* src = stage + 256 * ti[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[s][t] += src[64 * t + lane];
      }
    }
  }
  SBV_PROF(8, wk == 0);
  for (int k = 0; k < nt; ++k) {
    refresh_slots<SLOTS>(ti, tj);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (ti[s] == k && tj[s] == k) {
#pragma unroll
        for (int t = 0; t < 4; ++t) sm.diag[cl * kDiagLd + MF<T>::row(g, t)] = -acc[s][t];
      }
    }
    __syncthreads();  // S1
    SBV_PROF(9, wk == 0);
    // covariance column k+1 while the panel wave factors diagonal tile k
    if (kLateCov<T> && k + 1 < nt)
      gen_column<T, NTHR - 64>(sm, stage, wtid, k + 1, k + 1, nt, nA, d, two_nu, sigma2, tau2);
    SBV_PROF(15, wk == 0);
    __syncthreads();  // S2
    SBV_PROF(10, wk == 0);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (kLateCov<T> && tj[s] == k + 1) {
        const T* src = stage + 256 * ti[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[s][t] += src[64 * t + lane];
      }
    }
    // column-k TRSM: L_ik = A_ik L_kk^{-T}, published in operand layout
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] == k && ti[s] > k) {
        // two independent MFMA chains (q even, q odd) halve the dependent
        // latency (one chain in the large-block variant: fewer live registers)
        acc_t o = {T(0), T(0), T(0), T(0)}, o2 = {T(0), T(0), T(0), T(0)};
        if (PRE) {
#pragma unroll
          for (int q = 0; q < 4; ++q) o = MF<T>::mma(acc[s][q], sm.negM[68 * q + oplane(lane)], o);
        } else {
#pragma unroll
          for (int q = 0; q < 4; q += 2) {
            o = MF<T>::mma(acc[s][q], sm.negM[68 * q + oplane(lane)], o);
            o2 = MF<T>::mma(acc[s][q + 1], sm.negM[68 * (q + 1) + oplane(lane)], o2);
          }
#pragma unroll
          for (int t = 0; t < 4; ++t) o[t] += o2[t];
        }
        acc[s] = o;
        T* P = sm.panel + kOpT * ti[s];
#pragma unroll
        for (int t = 0; t < 4; ++t) P[opoff<T>(MF<T>::row(g, t), cl)] = o[t];
      }
      if (GRAD && tj[s] == k && ti[s] == k) {
        // keep X_kk = L_kk^{-1} in accumulator layout: X[a][b] = -negM[opoff(a, b)]
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[s][t] = -sm.negM[opoff<T>(MF<T>::row(g, t), cl)];
      }
    }
    SBV_PROF(11, wk == 0);
    __syncthreads();  // S3
    SBV_PROF(12, wk == 0);
    // trailing update G_ij += L_jk L_ik^T
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (tj[s] > k) {
        const T* Pj = sm.panel + kOpT * tj[s];
        const T* Pi = sm.panel + kOpT * ti[s];
        acc_t o = acc[s];
#pragma unroll
        for (int q = 0; q < 4; ++q) o = MF<T>::mma(Pj[68 * q + oplane(lane)], Pi[68 * q + oplane(lane)], o);
        acc[s] = o;
      }
    }
    SBV_PROF(13, wk == 0);
  }
  if (!GRAD) return;
  // ---- adjoint solves L^T X = R, right-hand sides in chunks of 32 columns
  const int nch = (bi + 1 + kChunk - 1) / kChunk;
  const int tid = 64 * (wk + 1) + lane;
  __syncthreads();  // B0: forward finished everywhere
  for (int r = tid; r < nt * kTile; r += NTHR) sm.gv[r] = T(0);
  for (int ch = 0; ch < nch; ++ch) {
    rhs_init<T, NTHR>(sm, tid, ch, nt, mi, bi);
    __syncthreads();  // B1
    for (int k = nt - 1; k >= 0; --k) {
      refresh_slots<SLOTS>(ti, tj);
      // X_k = L_kk^{-T} R_k by the diagonal owner
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (ti[s] == k && tj[s] == k) {
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            acc_t o = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < 4; ++q)
              o = MF<T>::mma(acc[s][q], sm.panel[(kTile * k + MF<T>::row(g, q)) * kRS + 16 * cb + cl], o);
#pragma unroll
            for (int t = 0; t < 4; ++t) sm.panel[(kTile * k + MF<T>::row(g, t)) * kRS + 16 * cb + cl] = o[t];
          }
        }
      }
      __syncthreads();  // B2
      // R_j -= L_kj^T X_k for j < k by the owners of row k of L
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (ti[s] == k && tj[s] < k && tj[s] >= 0) {
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            acc_t o = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < 4; ++q)
              o = MF<T>::mma(acc[s][q], sm.panel[(kTile * k + MF<T>::row(g, q)) * kRS + 16 * cb + cl], o);
            T* R = sm.panel + (kTile * tj[s]) * kRS + 16 * cb + cl;
#pragma unroll
            for (int t = 0; t < 4; ++t) R[MF<T>::row(g, t) * kRS] -= o[t];
          }
        }
      }
      __syncthreads();  // B3
    }
    rhs_writeback<T, NTHR>(sm, tid, ch, mi, nA, bi, ld, gout);
    __syncthreads();  // B4
  }
  for (int r = tid; r < nA; r += NTHR) gout[ld + r] = sm.gv[r];
}

// The panel wave's share of the adjoint solves: same barriers, plus its part
// of the set-up and write-back loops.
template <typename T, int NTHR, class SM>
__device__ __forceinline__ void panel_adjoint(SM& sm, int lane, int nt, int mi, int nA, int bi, int ld, T* gout) {
  const int nch = (bi + 1 + kChunk - 1) / kChunk;
  __syncthreads();  // B0
  for (int r = lane; r < nt * kTile; r += NTHR) sm.gv[r] = T(0);
  for (int ch = 0; ch < nch; ++ch) {
    rhs_init<T, NTHR>(sm, lane, ch, nt, mi, bi);
    __syncthreads();  // B1
    for (int k = nt - 1; k >= 0; --k) {
      __syncthreads();  // B2
      __syncthreads();  // B3
    }
    rhs_writeback<T, NTHR>(sm, lane, ch, mi, nA, bi, ld, gout);
    __syncthreads();  // B4
  }
  for (int r = lane; r < nA; r += NTHR) gout[ld + r] = sm.gv[r];
}

// PRE: large-block mode.  The block's first p = ceil(nA/16) - NTM tile rows
// were eliminated by k_block_prefix, which left L_RP and z_P in the workspace
// window L; this kernel factors the trailing NTM tiles (local point l is joint
// point l + 16p) after applying the p prefix updates.
template <typename T, int NTM, int NW, bool GRAD, bool SAMPLE = false, bool LA = false, bool PRE = false,
          int OCC = 1>
__global__ __launch_bounds__(NW * 64, OCC > 1 ? OCC * NW / 4 : 1) void k_block_loglik(const SetDesc* __restrict__ sets,
                                                          const double* __restrict__ theta,
                                                          const WorkItem* __restrict__ items,
                                                          const int* __restrict__ count,
                                                          double piv_tau, LargeArgs L) {
  static_assert(!PRE || (!SAMPLE && !LA && NTM == kLargeNTM), "large-block mode: no simulation, no lookahead");
  __shared__ Smem<T, NTM, GRAD, LA, SAMPLE> sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int total = PRE ? min(max(*count - L.off, 0), L.nb) : *count;
  const WorkItem* itm = PRE ? items + L.off : items;
#ifdef SBV_PHASE_PROFILE
  if (tid < 16) sm.prof[tid] = 0ull;
  __syncthreads();
#endif

  int isc_set = -1;  // set whose coordinate scales sm.isc holds
  // next item: grid stride, or one atomic increment of the queue per item
  auto take = [&](int cur) -> int {
    if (PRE || !L.queue) return cur + gridDim.x;
    if (tid == 0) sm.next_item = atomicAdd(L.queue, 1);
    __syncthreads();
    const int v = sm.next_item;
    __syncthreads();
    return v;
  };
  for (int it = (PRE || !L.queue) ? (int)blockIdx.x : take(0); it < total; it = take(it)) {
    const WorkItem w = itm[it];
    const SetDesc S = sets[w.set];
    const int d = S.d;
    const double* th = theta + S.theta_off;
    if (w.set != isc_set) {  // uniform over the workgroup
      if (tid < d) sm.isc[tid] = exp(-th[tid]);
      __syncthreads();
      isc_set = w.set;
    }
    const int b0 = S.bptr[w.block], b1 = S.bptr[w.block + 1];
    const int64_t n0 = S.nptr[w.block], n1 = S.nptr[w.block + 1];
    const int mi = (int)(n1 - n0), bi = b1 - b0, nA = mi + bi;
    int pre = 0;
    if (PRE) {
      pre = (nA + kTile - 1) / kTile - NTM;
      if (pre < 1 || pre > kMaxPrefix || kTile * pre > mi) {
        // not a large-path block (the host never queues one): mark it failed
        if (tid == 0) {
          S.llb[w.block] = -__builtin_inf();
          S.flag[w.block] = 2;
        }
        continue;
      }
    }
    const int off = kTile * pre;
    const int nAl = nA - off, mil = mi - off;  // local joint size and conditioning count
    const int nt = (nAl + kTile - 1) / kTile;
    const T sigma2 = T(exp(th[d]));
    const T tau2 = T(exp(th[d + 1]));
    T* gout = GRAD ? reinterpret_cast<T*>(S.qbuf) + S.qoff[w.block] + off : nullptr;
    const T* Wp = PRE ? reinterpret_cast<const T*>(L.W) + (int64_t)it * kLargeW : nullptr;
    const T* zp = PRE ? reinterpret_cast<const T*>(L.z) + (int64_t)it * kLargeZ : nullptr;

    // gather A = J u B (J first), one point per thread: scaled coordinates
    // (rows of zld(d), zero padded) and observations
    const int ld = zld<T>(d);
    if (PRE) {
      // (the large-block variant keeps the element-wise gather, which costs it
      // fewer register spills than the per-point one)
      for (int e = tid; e < nAl * ld; e += NW * 64) {
        const int pl = e / ld, k = e - pl * ld;
        const int pa = pl + off;
        const int pos = pa < mi ? S.nidx[n0 + pa] : b0 + (pa - mi);
        sm.z[pl * ld + k] = k < d ? T(S.X[(int64_t)pos * d + k] * exp(-th[k])) : T(0);
      }
    }
    for (int pl = tid; pl < nt * kTile; pl += NW * 64) {
      const int pa = pl + off;
      const bool real = pl < nAl;
      const int pos = real ? (pa < mi ? S.nidx[n0 + pa] : b0 + (pa - mi)) : 0;
      if (real && !PRE) {
        const double* xr = S.X + (int64_t)pos * d;
        for (int k = 0; k < ld; ++k) sm.z[pl * ld + k] = k < d ? T(xr[k] * sm.isc[k]) : T(0);
      }
      T v = T(0);
      if (real && (!SAMPLE || pa < mi)) v = T(S.y[pos]);
      sm.yv[pl] = v;
      if constexpr (SAMPLE) {
        sm.xi[pl] = (pa >= mi && real && S.xi) ? T(S.xi[b0 - S.out_off + (pa - mi)]) : T(0);
        sm.vacc[pl] = T(0);
      }
    }
    if (tid == 0) sm.la_flag = -1;
    __syncthreads();
#ifdef SBV_PHASE_PROFILE
    if (tid == 0) sm.prof[14] += 1ull;  // blocks processed
#endif

    if (wave == 0) {
      double ld_acc = 0.0, q_acc = 0.0;
      int bad = 0, low = 0;
      if (LA)
        panel_wave_la<T, NTM, NW * 64>(sm, lane, nt, mi, nA, d, S.two_nu, sigma2, tau2, T(piv_tau), ld_acc, q_acc,
                                       bad, low);
      else
        panel_wave<T, NTM, NW * 64, GRAD, SAMPLE, PRE>(
            sm, lane, nt, mil, nAl, d, S.two_nu, sigma2, tau2, T(piv_tau), ld_acc, q_acc, bad, low,
            SAMPLE ? S.y_out + (b0 - S.out_off) : nullptr, pre, Wp, zp,
            (SAMPLE && S.var_out) ? S.var_out + (b0 - S.out_off) : nullptr);
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
        S.flag[w.block] = PRE ? (S.flag[w.block] | fb) : fb;  // PRE: keep the prefix kernel's flags
      }
      if (GRAD) panel_adjoint<T, NW * 64>(sm, lane, nt, mil, nAl, bi, nA, gout);
    } else {
      if (LA)
        worker_waves_la<T, NTM, NW - 1, NW * 64>(sm, wave - 1, lane, nt, nA, d, S.two_nu, sigma2, tau2);
      else
        worker_waves<T, NTM, NW - 1, NW * 64, GRAD, PRE>(sm, wave - 1, lane, nt, mil, nAl, bi, d, S.two_nu,
                                                         sigma2, tau2, gout, nA, pre, Wp, zp);
    }
    __syncthreads();
  }
#ifdef SBV_PHASE_PROFILE
  __syncthreads();
  if (tid < 16) atomicAdd(&g_phase[tid], sm.prof[tid]);
#endif
}

// ---- large blocks: elimination of the prefix --------------------------------
// A block whose joint size nA exceeds 16 * kLargeNTM is split as A = [P; R]:
// P the first p = ceil(nA/16) - kLargeNTM tile rows (conditioning points only,
// 16p <= m_i) and R the last kLargeNTM tiles.  Block Cholesky gives
//   L = [L_PP, 0; L_RP, chol(T)],  L_RP = Sigma_RP L_PP^{-T},
//   T = Sigma_RR - L_RP L_RP^T,  z_P = L_PP^{-1} y_P,  z_R = chol(T)^{-1} (y_R - L_RP z_P),
// and every pivot and z entry of the block's own rows lies in the R part, so
// the block term of Alg. 5 follows from T and y_R - L_RP z_P alone.  This
// kernel factors Sigma_PP once into register tiles, keeps the inverses of its
// diagonal tiles in LDS, and builds L_RP in chunks of kLargeNTM - p tile rows:
// each chunk's Sigma_RP tiles are generated into the slots below P and
// eliminated column by column against the resident L_PP.  L_RP goes to the
// workspace tile by tile in the operand layout of the register kernel's panel,
// z_P beside it; k_block_loglik<..., PRE> consumes both.
template <typename T>
struct SmemP {
  alignas(16) T z[kLargeNTM * kTile * kMaxDim];  // scaled coordinates (rows of zld(d)): P, then a chunk of R
  T yv[kLargeNTM * kTile];           // observations of P, overwritten by the forward solve
  T panel[kLargeNTM * kOpT];         // generation staging / column k of L (operand layout)
  T diag[16 * kDiagLd];              // diagonal tile to factor (row-major, padded rows)
  T negMs[kMaxPrefix * kOpT];        // -(L_kk^{-T}) of every diagonal tile of P
  T zk[kTile];
  T xi[1];  // unused: factor_diag's simulation branch is not instantiated here
};

// Scaled coordinates (and, with yv, observations) of local points [lo, hi);
// local point l is joint point l + shift (J first); points past nA are zero.
template <typename T, int NTHR>
__device__ __forceinline__ void gather_points(T* z, T* yv, int tid, int lo, int hi, int shift, int d, int mi,
                                              int nA, const SetDesc& S, int b0, int64_t n0, const double* th) {
  const int ld = zld<T>(d);
  for (int e = tid; e < (hi - lo) * ld; e += NTHR) {
    const int pl = lo + e / ld, k = e % ld;
    const int pa = pl + shift;
    T v = T(0);
    if (pa < nA && k < d) {
      const int pos = pa < mi ? S.nidx[n0 + pa] : b0 + (pa - mi);
      v = T(S.X[(int64_t)pos * d + k] * exp(-th[k]));
    }
    z[pl * ld + k] = v;
  }
  if (yv)
    for (int pl = lo + tid; pl < hi; pl += NTHR) {
      const int pa = pl + shift;
      yv[pl] = pa < nA ? T(S.y[pa < mi ? S.nidx[n0 + pa] : b0 + (pa - mi)]) : T(0);
    }
}

// Panel wave of the prefix kernel: factors the diagonal tiles of P (first
// chunk only), solves z_P and writes it out; otherwise it takes part in the
// gathers and the generation and keeps the barrier count of the workers.
template <typename T, int NTHR, class SM>
__device__ __forceinline__ void prefix_panel_wave(SM& sm, int lane, int p, int c, const SetDesc& S, int b0,
                                                  int64_t n0, int mi, int nA, int d, const double* th, T sigma2,
                                                  T tau2, T tau, int& bad, int& low, T* zout) {
  const T diag0 = sigma2 + tau2;
  const int nch = (kLargeNTM + c - 1) / c;
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = ch * c, cc = min(c, kLargeNTM - r0), ntl = p + cc, nAl = nA - kTile * r0;
    gather_points<T, NTHR>(sm.z, (T*)nullptr, lane, kTile * p, kTile * ntl, kTile * r0, d, mi, nA, S, b0, n0,
                           th);
    __syncthreads();  // C0: chunk coordinates staged
    for (int j = 0; j < p; ++j) {
      gen_column<T, NTHR>(sm, sm.panel, lane, j, ch == 0 ? j : p, ntl, nAl, d, S.two_nu, sigma2, tau2);
      __syncthreads();  // G1
      __syncthreads();  // G2
    }
    for (int k = 0; k < p; ++k) {
      if (ch == 0) {
        __syncthreads();  // S1: diagonal tile published
        T piv, zr;
        factor_diag<T>(sm, sm.negMs + kOpT * k, lane, k, kTile, diag0, tau, piv, zr, bad, low);
        if (lane < kTile) {
          sm.zk[lane] = zr;
          zout[kTile * k + lane] = zr;
        }
        __syncthreads();  // S2: inverse of the diagonal tile published
        __syncthreads();  // S3: column k of L published
        y_update<T>(sm, lane, kTile * (k + 1), p);
      } else {
        __syncthreads();  // S3
        __syncthreads();  // S4
      }
    }
  }
}

// Worker waves of the prefix kernel.  Slots are numbered over the full
// kLargeNTM x kLargeNTM tile grid exactly as in the register kernel (p + c =
// kLargeNTM), so tiles of P stay in the same slots across chunks while the
// slots of rows p.. are regenerated for every chunk of R.
template <typename T, int NTM, int NWK, int NTHR, class SM>
__device__ __forceinline__ void prefix_worker_waves(SM& sm, int wk, int lane, int p, int c, const SetDesc& S,
                                                    int b0, int64_t n0, int mi, int nA, int d, const double* th,
                                                    T sigma2, T tau2, T* Wout, T* Lout) {
  typedef typename MF<T>::acc acc_t;
  constexpr int NTT = NTM * (NTM + 1) / 2;
  constexpr int SLOTS = (NTT + NWK - 1) / NWK;
  const int g = lane >> 4;
  const int cl = lane & 15;
  const int tid = 64 * (wk + 1) + lane;
  int ti[SLOTS], tj[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    int t = s * NWK + wk;
    int i = -1, j = -1;
    if (t < NTT) {
      j = 0;
      while (t >= NTM - j) {
        t -= NTM - j;
        ++j;
      }
      i = j + t;
    }
    ti[s] = __builtin_amdgcn_readfirstlane(i);
    tj[s] = __builtin_amdgcn_readfirstlane(j);
  }
  acc_t acc[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[s][t] = T(0);
  }
  const int nch = (NTM + c - 1) / c;
  for (int ch = 0; ch < nch; ++ch) {
    const int r0 = ch * c, cc = min(c, NTM - r0), ntl = p + cc, nAl = nA - kTile * r0;
    gather_points<T, NTHR>(sm.z, (T*)nullptr, tid, kTile * p, kTile * ntl, kTile * r0, d, mi, nA, S, b0, n0, th);
    __syncthreads();  // C0
    for (int j = 0; j < p; ++j) {
      refresh_slots<SLOTS>(ti, tj);
      const int i0 = ch == 0 ? j : p;
      gen_column<T, NTHR>(sm, sm.panel, tid, j, i0, ntl, nAl, d, S.two_nu, sigma2, tau2);
      __syncthreads();  // G1: column j staged
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (tj[s] == j && ti[s] >= i0 && ti[s] < ntl) {
          const T* src = sm.panel + 256 * ti[s];
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[s][t] = src[64 * t + lane];
        }
      }
      __syncthreads();  // G2
    }
    for (int k = 0; k < p; ++k) {
      refresh_slots<SLOTS>(ti, tj);
      const T* nM = sm.negMs + kOpT * k;
      if (ch == 0) {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          if (ti[s] == k && tj[s] == k) {
#pragma unroll
            for (int t = 0; t < 4; ++t) sm.diag[cl * kDiagLd + MF<T>::row(g, t)] = -acc[s][t];
          }
        }
        __syncthreads();  // S1
        __syncthreads();  // S2
      } else {
        // L_PP column k is final: publish it for this chunk's updates
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
          if (tj[s] == k && ti[s] > k && ti[s] < p) {
            T* P = sm.panel + kOpT * ti[s];
#pragma unroll
            for (int t = 0; t < 4; ++t) P[opoff<T>(MF<T>::row(g, t), cl)] = acc[s][t];
          }
        }
      }
      // column-k solves: rows of P (first chunk) and of the current chunk of R
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (tj[s] == k && ti[s] < ntl && (ch == 0 ? ti[s] > k : ti[s] >= p)) {
          acc_t o = {T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int q = 0; q < 4; ++q) o = MF<T>::mma(acc[s][q], nM[68 * q + oplane(lane)], o);
          acc[s] = o;
          T* P = sm.panel + kOpT * ti[s];
#pragma unroll
          for (int t = 0; t < 4; ++t) P[opoff<T>(MF<T>::row(g, t), cl)] = o[t];
        }
      }
      __syncthreads();  // S3: column k of L published
      // L_RP tiles of this chunk to the workspace (contiguous, coalesced)
      {
        T* dst = Wout + ((int64_t)k * NTM + r0) * kOpT;
        const T* src = sm.panel + kOpT * p;
        for (int e = tid - 64; e < cc * kOpT; e += NTHR - 64) dst[e] = src[e];
      }
      // for the adjoint: column k of L_PP (tile (j, k) at slot k * kMaxPrefix + j,
      // operand layout) and -L_kk^{-T} in the diagonal slot
      if (Lout && ch == 0) {
        T* dst = Lout + (int64_t)k * kMaxPrefix * kOpT;
        for (int e = kOpT * k + tid - 64; e < p * kOpT; e += NTHR - 64)
          dst[e] = e < kOpT * (k + 1) ? sm.negMs[e] : sm.panel[e];
      }
      // trailing update restricted to columns of P (the R x R part is left to
      // the register kernel)
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (tj[s] > k && tj[s] < p && ti[s] < ntl && (ch == 0 || ti[s] >= p)) {
          const T* Pj = sm.panel + kOpT * tj[s];
          const T* Pi = sm.panel + kOpT * ti[s];
          acc_t o = acc[s];
#pragma unroll
          for (int q = 0; q < 4; ++q) o = MF<T>::mma(Pj[68 * q + oplane(lane)], Pi[68 * q + oplane(lane)], o);
          acc[s] = o;
        }
      }
      if (ch > 0) __syncthreads();  // S4: staging area free
    }
  }
}

template <typename T, int NW>
__global__ __launch_bounds__(NW * 64) void k_block_prefix(const SetDesc* __restrict__ sets,
                                                          const double* __restrict__ theta,
                                                          const WorkItem* __restrict__ items,
                                                          const int* __restrict__ count, double piv_tau,
                                                          LargeArgs L) {
  __shared__ SmemP<T> sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int total = min(max(*count - L.off, 0), L.nb);
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const WorkItem w = items[L.off + it];
    const SetDesc S = sets[w.set];
    const int d = S.d;
    const double* th = theta + S.theta_off;
    const int b0 = S.bptr[w.block], b1 = S.bptr[w.block + 1];
    const int64_t n0 = S.nptr[w.block], n1 = S.nptr[w.block + 1];
    const int mi = (int)(n1 - n0), nA = mi + (b1 - b0);
    const int p = (nA + kTile - 1) / kTile - kLargeNTM;
    if (p < 1 || p > kMaxPrefix || kTile * p > mi) continue;  // never queued by the host
    const int c = kLargeNTM - p;
    const T sigma2 = T(exp(th[d]));
    const T tau2 = T(exp(th[d + 1]));
    T* Wout = reinterpret_cast<T*>(L.W) + (int64_t)it * kLargeW;
    T* zout = reinterpret_cast<T*>(L.z) + (int64_t)it * kLargeZ;
    T* Lout = L.Lpp ? reinterpret_cast<T*>(L.Lpp) + (int64_t)it * kLargeL : nullptr;
    gather_points<T, NW * 64>(sm.z, sm.yv, tid, 0, kTile * p, 0, d, mi, nA, S, b0, n0, th);
    __syncthreads();
    if (wave == 0) {
      int bad = 0, low = 0;
      prefix_panel_wave<T, NW * 64>(sm, lane, p, c, S, b0, n0, mi, nA, d, th, sigma2, tau2, T(piv_tau), bad, low,
                                    zout);
      if (lane == 0) S.flag[w.block] = (bad ? 2 : 0) | (low ? 1 : 0);
    } else {
      prefix_worker_waves<T, kLargeNTM, NW - 1, NW * 64>(sm, wave - 1, lane, p, c, S, b0, n0, mi, nA, d, th,
                                                         sigma2, tau2, Wout, Lout);
    }
    __syncthreads();
  }
}

// ---- gradient contraction -------------------------------------------------
// For one block, with e, g and Q = L^{-T}[0; I_b] from the adjoint solves:
//   dl_i/dtheta_k = 1/2 sum_ab M_ab dSigma_ab/dtheta_k,
//   M = e g^T + g e^T + g g^T - Q Q^T,
// where Q Q^T is accumulated tile by tile on MFMA (register tiles over the
// lower triangle) and dSigma is recomputed from the scaled coordinates:
//   d/dlog beta_k: sigma^2 (-rho'(r)/r) s_k^2,  d/dlog sigma^2: sigma^2 rho(r),
//   d/dlog tau^2: tau^2 on the diagonal.
template <typename T>
__device__ __forceinline__ T mdrho_over_r(T r, int two_nu) {
  T e = t_exp(-r);
  if (two_nu == 5) return (T(1) + r) * e * T(1.0 / 3.0);
  if (two_nu == 3) return e;
  if (two_nu == 7) return (T(3) + T(3) * r + r * r) * e * T(1.0 / 15.0);
  return r > T(0) ? e / r : T(0);
}

template <typename T, int NTM>
struct SmemC {
  T z[NTM * kTile * kMaxDim];
  T q[NTM * kTile * kRS];
  T ev[NTM * kTile];
  T gv[NTM * kTile];
  double red[16][kMaxDim + 2];
};

template <typename T, int NTM, int NW>
__global__ __launch_bounds__(NW * 64) void k_block_contract(const SetDesc* __restrict__ sets,
                                                            const double* __restrict__ theta,
                                                            const WorkItem* __restrict__ items,
                                                            const int* __restrict__ count) {
  typedef typename MF<T>::acc acc_t;
  constexpr int NTT = NTM * (NTM + 1) / 2;
  constexpr int SLOTS = (NTT + NW - 1) / NW;
  constexpr int NTHR = NW * 64;
  __shared__ SmemC<T, NTM> sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, cl = lane & 15;
  const int total = *count;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const WorkItem w = items[it];
    const SetDesc S = sets[w.set];
    const int d = S.d, two_nu = S.two_nu;
    const double* th = theta + S.theta_off;
    const int b0 = S.bptr[w.block], b1 = S.bptr[w.block + 1];
    const int64_t n0 = S.nptr[w.block], n1 = S.nptr[w.block + 1];
    const int mi = (int)(n1 - n0), bi = b1 - b0, nA = mi + bi;
    const int nt = (nA + kTile - 1) / kTile;
    const int ntt = nt * (nt + 1) / 2;
    const T sigma2 = T(exp(th[d]));
    const T tau2 = T(exp(th[d + 1]));
    const T* src = reinterpret_cast<const T*>(S.qbuf) + S.qoff[w.block];
    for (int e = tid; e < nA * d; e += NTHR) {
      int p = e / d, k = e - p * d;
      int pos = p < mi ? S.nidx[n0 + p] : b0 + (p - mi);
      sm.z[p * d + k] = T(S.X[(int64_t)pos * d + k] * exp(-th[k]));
    }
    for (int r = tid; r < nt * kTile; r += NTHR) {
      sm.ev[r] = r < nA ? src[r] : T(0);
      sm.gv[r] = r < nA ? src[nA + r] : T(0);
    }
    int ti[SLOTS], tj[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      int t = s * NW + wave;
      int i = -1, j = -1;
      if (t < ntt) {
        j = 0;
        while (t >= nt - j) {
          t -= nt - j;
          ++j;
        }
        i = j + t;
      }
      ti[s] = __builtin_amdgcn_readfirstlane(i);
      tj[s] = __builtin_amdgcn_readfirstlane(j);
    }
    acc_t P[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) P[s] = acc_t{T(0), T(0), T(0), T(0)};
    // Q Q^T over chunks of 32 columns of Q
    for (int c0 = 0; c0 < bi; c0 += kChunk) {
      __syncthreads();
      for (int e = tid; e < nt * kTile * kChunk; e += NTHR) {
        const int c = e / (nt * kTile), r = e - c * (nt * kTile);
        T v = T(0);
        if (r < nA && c0 + c < bi) v = src[(int64_t)(2 + c0 + c) * nA + r];
        sm.q[r * kRS + c] = v;
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        if (ti[s] >= 0) {
          const T* Qi = sm.q + (kTile * ti[s] + cl) * kRS;
          const T* Qj = sm.q + (kTile * tj[s] + cl) * kRS;
          acc_t o = P[s];
#pragma unroll
          for (int q = 0; q < kChunk / 4; ++q) o = MF<T>::mma(Qi[4 * q + g], Qj[4 * q + g], o);
          P[s] = o;
        }
      }
    }
    __syncthreads();
    // contraction with the recomputed covariance derivatives
    double gacc[kMaxDim + 2];
#pragma unroll
    for (int k = 0; k < kMaxDim + 2; ++k) gacc[k] = 0.0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      if (ti[s] < 0) continue;
      const double wgt = ti[s] == tj[s] ? 1.0 : 2.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int a = kTile * ti[s] + MF<T>::row(g, t);
        const int b = kTile * tj[s] + cl;
        if (a >= nA || b >= nA) continue;
        const T M = sm.ev[a] * sm.gv[b] + sm.gv[a] * sm.ev[b] + sm.gv[a] * sm.gv[b] - P[s][t];
        T r2 = T(0);
        for (int k = 0; k < d; ++k) {
          T df = sm.z[a * d + k] - sm.z[b * d + k];
          r2 += df * df;
        }
        const T r = t_sqrt(r2);
        const double wm = wgt * (double)M;
        const double f = wm * (double)(sigma2 * mdrho_over_r<T>(r, two_nu));
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
          if (k < d) {
            T df = sm.z[a * d + k] - sm.z[b * d + k];
            gacc[k] += f * (double)(df * df);
          }
        }
        gacc[kMaxDim] += wm * (double)(sigma2 * matern<T>(r, two_nu));
        if (a == b) gacc[kMaxDim + 1] += wm * (double)tau2;
      }
    }
    // fixed-order reduction: lanes, then waves
#pragma unroll
    for (int k = 0; k < kMaxDim + 2; ++k) {
      double v = gacc[k];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) sm.red[wave][k] = v;
    }
    __syncthreads();
    if (tid < d + 2) {
      const int k = tid < d ? tid : kMaxDim + (tid - d);
      double v = 0.0;
      for (int wv = 0; wv < NW; ++wv) v += sm.red[wv][k];
      S.gradb[(int64_t)w.block * (d + 2) + tid] = 0.5 * v;
    }
    __syncthreads();
  }
}

// ---- large blocks: prefix part of the adjoint ---------------------------------
// With L = [L_PP, 0; L_RP, L_T] the adjoint solves L^T X = Rhs split into
//   L_T^T X_R = Rhs_R                       (the trailing kernel, GRAD mode),
//   L_PP^T X_P = Rhs_P - L_RP^T X_R,
// for the columns e (Rhs_P = z_P), g and those of Q (Rhs_P = 0).  This kernel
// forms the second right-hand side 32 columns at a time and solves it
// backwards with the stored L_PP tiles and inverted diagonal tiles; X_P goes to
// rows 0..16p-1 of the block's adjoint buffer, which then holds e, g and Q
// over the whole joint set.
template <typename T>
struct SmemPA {
  T xr[kLargeNTM * kTile * kRS];   // chunk of X_R (rows of R)
  T rp[kMaxPrefix * kTile * kRS];  // right-hand side, then solution, of the prefix rows
  T xk[kTile * kRS];               // solved tile row k
};

template <typename T, int NW>
__global__ __launch_bounds__(NW * 64) void k_block_prefix_adjoint(const SetDesc* __restrict__ sets,
                                                                  const WorkItem* __restrict__ items,
                                                                  const int* __restrict__ count, LargeArgs L) {
  constexpr int NTHR = NW * 64;
  __shared__ SmemPA<T> sm;
  const int tid = threadIdx.x;
  const int total = min(max(*count - L.off, 0), L.nb);
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const WorkItem w = items[L.off + it];
    const SetDesc S = sets[w.set];
    const int b0 = S.bptr[w.block], b1 = S.bptr[w.block + 1];
    const int64_t n0 = S.nptr[w.block], n1 = S.nptr[w.block + 1];
    const int mi = (int)(n1 - n0), bi = b1 - b0, nA = mi + bi;
    const int p = (nA + kTile - 1) / kTile - kLargeNTM;
    if (p < 1 || p > kMaxPrefix || kTile * p > mi) continue;  // never queued by the host
    const int np = kTile * p, nR = nA - np;
    T* qb = reinterpret_cast<T*>(S.qbuf) + S.qoff[w.block];
    const T* Wp = reinterpret_cast<const T*>(L.W) + (int64_t)it * kLargeW;
    const T* Lp = reinterpret_cast<const T*>(L.Lpp) + (int64_t)it * kLargeL;
    const T* zp = reinterpret_cast<const T*>(L.z) + (int64_t)it * kLargeZ;
    const int ncol = bi + 2;  // e, g, then the columns of Q (column c at c * nA)
    for (int c0 = 0; c0 < ncol; c0 += kChunk) {
      for (int e = tid; e < nR * kChunk; e += NTHR) {
        const int r = e / kChunk, c = e - r * kChunk;
        sm.xr[r * kRS + c] = c0 + c < ncol ? qb[(int64_t)(c0 + c) * nA + np + r] : T(0);
      }
      __syncthreads();
      // Rhs_P - L_RP^T X_R; workspace tile (k, i) holds L[16p + 16i + a][16k + b] at opoff(a, b)
      for (int e = tid; e < np * kChunk; e += NTHR) {
        const int rr = e / kChunk, c = e - rr * kChunk;
        const T* Wk = Wp + (int64_t)(rr >> 4) * kLargeNTM * kOpT;
        const int cc = rr & 15;
        T acc = T(0);
        for (int r = 0; r < nR; ++r) acc += Wk[(r >> 4) * kOpT + opoff<T>(r & 15, cc)] * sm.xr[r * kRS + c];
        sm.rp[rr * kRS + c] = (c0 + c == 0 ? zp[rr] : T(0)) - acc;
      }
      __syncthreads();
      for (int k = p - 1; k >= 0; --k) {
        // X_k = L_kk^{-T} Rhs_k; the diagonal slot holds -(L_kk^{-1})[a][b] at opoff(a, b)
        const T* nM = Lp + ((int64_t)k * kMaxPrefix + k) * kOpT;
        for (int e = tid; e < kTile * kChunk; e += NTHR) {
          const int a = e / kChunk, c = e - a * kChunk;
          T acc = T(0);
          for (int b = 0; b < kTile; ++b) acc -= nM[opoff<T>(b, a)] * sm.rp[(kTile * k + b) * kRS + c];
          sm.xk[a * kRS + c] = acc;
        }
        __syncthreads();
        for (int e = tid; e < kTile * kChunk; e += NTHR) {
          const int a = e / kChunk, c = e - a * kChunk;
          sm.rp[(kTile * k + a) * kRS + c] = sm.xk[a * kRS + c];
        }
        // Rhs_j -= L_kj^T X_k for j < k; tile (k, j) sits in slot j * kMaxPrefix + k
        for (int e = tid; e < kTile * k * kChunk; e += NTHR) {
          const int rr = e / kChunk, c = e - rr * kChunk;
          const T* Lkj = Lp + ((int64_t)(rr >> 4) * kMaxPrefix + k) * kOpT;
          const int b = rr & 15;
          T acc = T(0);
          for (int a = 0; a < kTile; ++a) acc += Lkj[opoff<T>(a, b)] * sm.xk[a * kRS + c];
          sm.rp[rr * kRS + c] -= acc;
        }
        __syncthreads();
      }
      for (int e = tid; e < np * kChunk; e += NTHR) {
        const int rr = e / kChunk, c = e - rr * kChunk;
        if (c0 + c < ncol) qb[(int64_t)(c0 + c) * nA + rr] = sm.rp[rr * kRS + c];
      }
      __syncthreads();
    }
  }
}

// ---- large blocks: streamed gradient contraction -----------------------------
// The same contraction as k_block_contract over the whole joint set, with the
// tiles of the lower triangle taken one at a time by the waves (Q Q^T of a
// tile on MFMA, operands read from the adjoint buffer) instead of held in
// registers.
template <typename T>
struct SmemCS {
  T z[(kLargeNTM + kMaxPrefix) * kTile * kMaxDim];
  T ev[(kLargeNTM + kMaxPrefix) * kTile];
  T gv[(kLargeNTM + kMaxPrefix) * kTile];
  double red[8][kMaxDim + 2];
};

template <typename T, int NW>
__global__ __launch_bounds__(NW * 64) void k_block_contract_stream(const SetDesc* __restrict__ sets,
                                                                   const double* __restrict__ theta,
                                                                   const WorkItem* __restrict__ items,
                                                                   const int* __restrict__ count, LargeArgs L) {
  static_assert(NW <= 8, "reduction buffer holds 8 waves");
  typedef typename MF<T>::acc acc_t;
  constexpr int NTHR = NW * 64;
  __shared__ SmemCS<T> sm;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, cl = lane & 15;
  const int total = min(max(*count - L.off, 0), L.nb);
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const WorkItem w = items[L.off + it];
    const SetDesc S = sets[w.set];
    const int d = S.d, two_nu = S.two_nu;
    const double* th = theta + S.theta_off;
    const int b0 = S.bptr[w.block], b1 = S.bptr[w.block + 1];
    const int64_t n0 = S.nptr[w.block], n1 = S.nptr[w.block + 1];
    const int mi = (int)(n1 - n0), bi = b1 - b0, nA = mi + bi;
    const int nt = (nA + kTile - 1) / kTile;
    if (nt > kLargeNTM + kMaxPrefix) continue;  // never queued by the host
    const int ntt = nt * (nt + 1) / 2;
    const T sigma2 = T(exp(th[d]));
    const T tau2 = T(exp(th[d + 1]));
    const T* src = reinterpret_cast<const T*>(S.qbuf) + S.qoff[w.block];
    for (int e = tid; e < nA * d; e += NTHR) {
      const int pa = e / d, k = e - pa * d;
      const int pos = pa < mi ? S.nidx[n0 + pa] : b0 + (pa - mi);
      sm.z[pa * d + k] = T(S.X[(int64_t)pos * d + k] * exp(-th[k]));
    }
    for (int r = tid; r < nt * kTile; r += NTHR) {
      sm.ev[r] = r < nA ? src[r] : T(0);
      sm.gv[r] = r < nA ? src[nA + r] : T(0);
    }
    __syncthreads();
    double gacc[kMaxDim + 2];
#pragma unroll
    for (int k = 0; k < kMaxDim + 2; ++k) gacc[k] = 0.0;
    for (int t = wave; t < ntt; t += NW) {
      int i, j = 0, tt = t;
      while (tt >= nt - j) {
        tt -= nt - j;
        ++j;
      }
      i = j + tt;
      const int ra = kTile * i + cl, rb = kTile * j + cl;
      acc_t P = {T(0), T(0), T(0), T(0)};
      for (int q0 = 0; q0 < bi; q0 += 4) {
        const int c = q0 + g;
        const T qa = (c < bi && ra < nA) ? src[(int64_t)(2 + c) * nA + ra] : T(0);
        const T qc = (c < bi && rb < nA) ? src[(int64_t)(2 + c) * nA + rb] : T(0);
        P = MF<T>::mma(qa, qc, P);
      }
      const double wgt = i == j ? 1.0 : 2.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = kTile * i + MF<T>::row(g, q);
        const int b = kTile * j + cl;
        if (a >= nA || b >= nA) continue;
        const T M = sm.ev[a] * sm.gv[b] + sm.gv[a] * sm.ev[b] + sm.gv[a] * sm.gv[b] - P[q];
        T r2 = T(0);
        for (int k = 0; k < d; ++k) {
          const T df = sm.z[a * d + k] - sm.z[b * d + k];
          r2 += df * df;
        }
        const T r = t_sqrt(r2);
        const double wm = wgt * (double)M;
        const double f = wm * (double)(sigma2 * mdrho_over_r<T>(r, two_nu));
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
          if (k < d) {
            const T df = sm.z[a * d + k] - sm.z[b * d + k];
            gacc[k] += f * (double)(df * df);
          }
        }
        gacc[kMaxDim] += wm * (double)(sigma2 * matern<T>(r, two_nu));
        if (a == b) gacc[kMaxDim + 1] += wm * (double)tau2;
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxDim + 2; ++k) {
      double v = gacc[k];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) sm.red[wave][k] = v;
    }
    __syncthreads();
    if (tid < d + 2) {
      const int k = tid < d ? tid : kMaxDim + (tid - d);
      double v = 0.0;
      for (int wv = 0; wv < NW; ++wv) v += sm.red[wv][k];
      S.gradb[(int64_t)w.block * (d + 2) + tid] = 0.5 * v;
    }
    __syncthreads();
  }
}

// ---- variants -------------------------------------------------------------
// Sorted by tile capacity; for a capacity, the 8-wave kernel comes first (the
// default), the 16-wave one after it (FP32 only: more waves per SIMD to hide
// latency, 128 registers each; the FP64 tiles do not fit 128 registers, so an
// FP64 request for it runs the 8-wave kernel).  The autotuner may pick any
// variant at or above a bucket's smallest fitting one.
// The occupancy-2 variants (FP32 only, like the 16-wave ones) cap an 8-wave
// workgroup at 128 registers per lane so that two blocks share a compute
// unit and one block's serial diagonal factorisations run beside the other's
// trailing updates.
static const Variant kVariants[] = {{4, 2},      {8, 4},  {12, 8},     {14, 8},  {14, 16},
                                    {14, 8, 2},  {16, 8}, {16, 16},    {16, 8, 2}, {17, 8}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int n_variants() { return kNumVariants; }
Variant variant(int v) { return kVariants[v]; }
int variant_for(int nA) {
  for (int v = 0; v < kNumVariants; ++v)
    if (nA <= kVariants[v].ntm * kTile) return v;
  return -1;
}

// Waves of the kernel actually launched for a variant: 16-wave variants exist
// for FP32 only, and the gradient, contraction and simulation kernels always
// use the 8-wave layout.
template <typename T, int NW>
constexpr int nw_of() {
  return (NW > 8 && sizeof(T) == 8) ? 8 : NW;
}

template <typename T, int NTM, int NW, int OCC = 1>
static hipError_t launch_t(int grid, bool grad, bool la, const SetDesc* sets, const double* theta,
                           const WorkItem* items, const int* count, double piv_tau, hipStream_t s, int* queue) {
  if constexpr (nw_of<T, NW>() != NW || (OCC > 1 && sizeof(T) == 8)) {
    return launch_t<T, NTM, nw_of<T, NW>(), 1>(grid, grad, la, sets, theta, items, count, piv_tau, s, queue);
  } else {
    constexpr int NWG = NW > 8 ? 8 : NW;  // the gradient kernels keep the 8-wave layout
    const LargeArgs q{0, 0, nullptr, nullptr, nullptr, queue};
    if (la && !grad)
      hipLaunchKernelGGL((k_block_loglik<T, NTM, NW, false, false, true, false, OCC>), dim3(grid), dim3(NW * 64), 0,
                         s, sets, theta, items, count, piv_tau, q);
    else if (grad)
      hipLaunchKernelGGL((k_block_loglik<T, NTM, NWG, true>), dim3(grid), dim3(NWG * 64), 0, s, sets, theta, items,
                         count, piv_tau, q);
    else
      hipLaunchKernelGGL((k_block_loglik<T, NTM, NW, false, false, false, false, OCC>), dim3(grid), dim3(NW * 64), 0,
                         s, sets, theta, items, count, piv_tau, q);
    return hipGetLastError();
  }
}

template <typename T, int NTM, int NW>
static hipError_t launch_s(int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                           const int* count, hipStream_t s) {
  if constexpr (NW > 8) return launch_s<T, NTM, 8>(grid, sets, theta, items, count, s);
  hipLaunchKernelGGL((k_block_loglik<T, NTM, NW, false, true>), dim3(grid), dim3(NW * 64), 0, s, sets, theta,
                     items, count, 0.0, LargeArgs{});
  return hipGetLastError();
}

template <typename T, int NTM, int NW>
static hipError_t launch_c(int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                           const int* count, hipStream_t s) {
  if constexpr (NW > 8) return launch_c<T, NTM, 8>(grid, sets, theta, items, count, s);
  hipLaunchKernelGGL((k_block_contract<T, NTM, NW>), dim3(grid), dim3(NW * 64), 0, s, sets, theta, items, count);
  return hipGetLastError();
}

#define SBV_VARIANT_SWITCH(T, CALL)      \
  switch (v) {                           \
    case 0: return CALL(T, 4, 2, 1);     \
    case 1: return CALL(T, 8, 4, 1);     \
    case 2: return CALL(T, 12, 8, 1);    \
    case 3: return CALL(T, 14, 8, 1);    \
    case 4: return CALL(T, 14, 16, 1);   \
    case 5: return CALL(T, 14, 8, 2);    \
    case 6: return CALL(T, 16, 8, 1);    \
    case 7: return CALL(T, 16, 16, 1);   \
    case 8: return CALL(T, 16, 8, 2);    \
    case 9: return CALL(T, 17, 8, 1);    \
  }

hipError_t launch_loglik(int prec, int v, int grid, const SetDesc* sets, const double* theta,
                         const WorkItem* items, const int* count, double piv_tau, hipStream_t s, bool grad,
                         bool lookahead, int* queue) {
  if (grid <= 0) return hipSuccess;
#define SBV_CALL(T, A, B, C) launch_t<T, A, B, C>(grid, grad, lookahead, sets, theta, items, count, piv_tau, s, queue)
  if (prec == 0) {
    SBV_VARIANT_SWITCH(double, SBV_CALL)
  } else {
    SBV_VARIANT_SWITCH(float, SBV_CALL)
  }
#undef SBV_CALL
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_large_t(int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                                 const int* count, double piv_tau, const LargeArgs& L, hipStream_t s) {
  hipLaunchKernelGGL((k_block_prefix<T, 8>), dim3(grid), dim3(512), 0, s, sets, theta, items, count, piv_tau, L);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL((k_block_loglik<T, kLargeNTM, 8, false, false, false, true>), dim3(grid), dim3(512), 0, s,
                     sets, theta, items, count, piv_tau, L);
  return hipGetLastError();
}

hipError_t launch_large(int prec, int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                        const int* count, double piv_tau, const LargeArgs& L, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (prec == 0) return launch_large_t<double>(grid, sets, theta, items, count, piv_tau, L, s);
  return launch_large_t<float>(grid, sets, theta, items, count, piv_tau, L, s);
}

template <typename T>
static hipError_t launch_large_grad_t(int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                                      const int* count, double piv_tau, const LargeArgs& L, hipStream_t s) {
  if (!L.Lpp) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_block_prefix<T, 8>), dim3(grid), dim3(512), 0, s, sets, theta, items, count, piv_tau, L);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL((k_block_loglik<T, kLargeNTM, 8, true, false, false, true>), dim3(grid), dim3(512), 0, s,
                     sets, theta, items, count, piv_tau, L);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL((k_block_prefix_adjoint<T, 8>), dim3(grid), dim3(512), 0, s, sets, items, count, L);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL((k_block_contract_stream<T, 8>), dim3(grid), dim3(512), 0, s, sets, theta, items, count, L);
  return hipGetLastError();
}

hipError_t launch_large_grad(int prec, int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                             const int* count, double piv_tau, const LargeArgs& L, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (prec == 0) return launch_large_grad_t<double>(grid, sets, theta, items, count, piv_tau, L, s);
  return launch_large_grad_t<float>(grid, sets, theta, items, count, piv_tau, L, s);
}

hipError_t launch_sample(int v, int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                         const int* count, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define SBV_CALL(T, A, B, C) launch_s<T, A, B>(grid, sets, theta, items, count, s)
  SBV_VARIANT_SWITCH(double, SBV_CALL)
#undef SBV_CALL
  return hipErrorInvalidValue;
}

hipError_t launch_contract(int prec, int v, int grid, const SetDesc* sets, const double* theta,
                           const WorkItem* items, const int* count, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define SBV_CALL(T, A, B, C) launch_c<T, A, (B < 4 ? 4 : B)>(grid, sets, theta, items, count, s)
  if (prec == 0) {
    SBV_VARIANT_SWITCH(double, SBV_CALL)
  } else {
    SBV_VARIANT_SWITCH(float, SBV_CALL)
  }
#undef SBV_CALL
  return hipErrorInvalidValue;
}

#ifdef SBV_PHASE_PROFILE
hipError_t read_phase_profile(unsigned long long* out) {
  hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase), sizeof(unsigned long long) * 16);
  if (e) return e;
  unsigned long long z[16] = {};
  return hipMemcpyToSymbol(HIP_SYMBOL(g_phase), z, sizeof(z));
}
#endif

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

// Per-set gradient: sum of the per-block terms in a fixed order, one
// workgroup per set, one pass per parameter.  A set whose log-likelihood
// reduction found a block that is not positive definite (bad != 0) gets NaN.
__global__ __launch_bounds__(256) void k_reduce_grad(const SetDesc* __restrict__ sets,
                                                     double* __restrict__ out, const int* __restrict__ bad) {
  __shared__ double red[256];
  const SetDesc S = sets[blockIdx.x];
  const int np = S.d + 2;
  for (int k = 0; k < np; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < S.K; i += 256) s += S.gradb[(int64_t)i * np + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[S.theta_off + k] = (bad && bad[blockIdx.x]) ? __builtin_nan("") : red[0];
    __syncthreads();
  }
}

hipError_t launch_reduce_grad(const SetDesc* sets, int n_sets, double* out, const int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_grad, dim3(n_sets), dim3(256), 0, s, sets, out, bad);
  return hipGetLastError();
}

// ---- dense covariance matrix (Eq. (maternkernel) between two point lists) --
// out[a * nb + b] = sigma^2 rho(r_ab) (+ tau^2 when same and a == b), with the
// coordinates scaled as in the block kernels (x * exp(-theta_k)).  One thread
// per entry, rows of out contiguous.
__global__ void k_cov_matrix(const double* __restrict__ Xa, int64_t na, const double* __restrict__ Xb, int64_t nb,
                             int d, const double* __restrict__ theta, int two_nu, int same, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= na * nb) return;
  const int64_t a = e / nb, b = e - a * nb;
  double r2 = 0.0;
  for (int k = 0; k < d; ++k) {
    const double sc = exp(-theta[k]);
    const double df = Xa[a * d + k] * sc - Xb[b * d + k] * sc;
    r2 += df * df;
  }
  double v = exp(theta[d]) * matern<double>(g_sqrt(r2), two_nu);
  if (same && a == b) v += exp(theta[d + 1]);
  out[e] = v;
}

hipError_t launch_cov_matrix(const double* Xa, int64_t na, const double* Xb, int64_t nb, int d, const double* theta,
                             int two_nu, int same, double* out, hipStream_t s) {
  const int64_t n = na * nb;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cov_matrix, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Xa, na, Xb, nb, d, theta,
                     two_nu, same, out);
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
