// sbv_build_blocks: the block structure of Alg. 1 Steps 1-3 on one GPU.
//
//   1. scale z = x / beta_build                                   (Alg. 2)
//   2. K random anchors (SplitMix64 + partial Fisher-Yates)        (Alg. 3)
//   3. nearest-anchor assignment on the device (FP64)              (Alg. 3)
//   4. optional Lloyd passes: means on the host in point order,
//      empty clusters re-seeded with the point farthest from its
//      centre, re-assignment on the device, stop when nothing moves
//   5. size bounds: split clusters above max_bs along their largest-variance
//      axis into ceil(s/max_bs) near-equal chunks; merge clusters below min_bs
//      into the nearest (by centre) cluster with room
//   6. uniformly random block order (Fisher-Yates, seed + 1)        (Alg. 1)
//   7. points ordered by (block rank, id); centroids in scaled space (Alg. 4)
//   8. exact m nearest points of strictly earlier blocks to each centroid,
//      brute force on the device (Alg. 4 without the distance threshold)
//   9. pack and upload (the handle's contiguous device layout)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/sbv.h"
#include "sbv_internal.h"

namespace sbv {
hipError_t launch_assign(const double* Z, int64_t n, int d, const double* C, int K, int32_t* lab,
                         double* best_d2, hipStream_t s);

}  // namespace sbv

sbv_status sbv_internal_fail(sbv_status st, const char* msg);
void sbv_internal_set_build(sbv_blocks h, const double* beta_build, int64_t K, int32_t m, const sbv_build_opts& o);
sbv_status sbv_internal_make_handle(const double* X, const double* y, int64_t n, int32_t d, int64_t K,
                                    const int64_t* block_ptr, const int64_t* block_pts,
                                    const int64_t* nn_ptr, const int64_t* nn_idx, sbv_blocks* out);

namespace {

using namespace sbv;

// Progress lines on stderr when the environment variable SBV_PROGRESS is set
// (builds of 1e7+ points take minutes).
void progress(const char* what, double a = -1.0, double b = -1.0) {
  static const bool on = std::getenv("SBV_PROGRESS") != nullptr;
  if (!on) return;
  if (b >= 0.0)
    std::fprintf(stderr, "[build] %s %.0f / %.0f\n", what, a, b);
  else if (a >= 0.0)
    std::fprintf(stderr, "[build] %s %.0f\n", what, a);
  else
    std::fprintf(stderr, "[build] %s\n", what);
  std::fflush(stderr);
}

struct Splitmix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // uniform in [0, n): high half of the 128-bit product of a draw and n
  uint64_t below(uint64_t n) { return (uint64_t)(((unsigned __int128)next() * n) >> 64); }
};

template <typename T>
struct Dev {
  T* p = nullptr;
  Dev() = default;
  Dev(const Dev&) = delete;
  Dev& operator=(const Dev&) = delete;
  ~Dev() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc((void**)&p, sizeof(T) * std::max<size_t>(n, 1)); }
};

#define BTRY(expr)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return sbv_internal_fail(e_ == hipErrorOutOfMemory ? SBV_E_NOMEM : SBV_E_DEVICE,       \
                               (std::string("HIP error in builder: ") + hipGetErrorString(e_)).c_str()); \
  } while (0)

double sqd(const double* a, const double* b, int d) {
  double s = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = a[k] - b[k];
    s += t * t;
  }
  return s;
}

// Cluster means in point-id order; returns sizes.
void cluster_means(const std::vector<double>& Z, int64_t n, int d, const std::vector<int32_t>& lab, int64_t K,
                   std::vector<double>& C, std::vector<int64_t>& cnt) {
  C.assign((size_t)K * d, 0.0);
  cnt.assign(K, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t c = lab[i];
    ++cnt[c];
    for (int k = 0; k < d; ++k) C[c * d + k] += Z[i * d + k];
  }
  for (int64_t c = 0; c < K; ++c)
    if (cnt[c])
      for (int k = 0; k < d; ++k) C[c * d + k] /= (double)cnt[c];
}

// Alg. 3 on one point set: K random anchors (partial Fisher-Yates with
// SplitMix64(seed)), nearest-anchor assignment on the device, Lloyd passes
// (empty clusters re-seeded with the point farthest from its centre), the
// size bounds, and empty clusters dropped; lab receives cluster ids 0..K-1
// and K the final count.
sbv_status cluster_points(const std::vector<double>& Z, int64_t n, int d, int64_t& K, const sbv_build_opts& o,
                          uint64_t seed, int lloyd, std::vector<int32_t>& lab) {
  Dev<double> dZ, dC;
  Dev<int32_t> dlab;
  Dev<double> dbest;
  BTRY(dZ.alloc((size_t)n * d));
  BTRY(dlab.alloc(n));
  BTRY(dbest.alloc(n));
  BTRY(hipMemcpy(dZ.p, Z.data(), sizeof(double) * n * d, hipMemcpyHostToDevice));

  // 2. anchors
  std::vector<double> C((size_t)K * d);
  {
    std::vector<int64_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    Splitmix rs{seed};
    for (int64_t i = 0; i < K; ++i) {
      int64_t j = i + (int64_t)rs.below((uint64_t)(n - i));
      std::swap(perm[i], perm[j]);
      std::memcpy(&C[i * d], &Z[perm[i] * d], sizeof(double) * d);
    }
  }
  // 3.-4. assignment and Lloyd passes
  lab.assign(n, 0);
  std::vector<int32_t> prev(n);
  std::vector<double> best(n);
  std::vector<int64_t> cnt;
  BTRY(dC.alloc((size_t)K * d));
  auto assign = [&]() -> sbv_status {
    BTRY(hipMemcpy(dC.p, C.data(), sizeof(double) * K * d, hipMemcpyHostToDevice));
    BTRY(launch_assign(dZ.p, n, d, dC.p, (int)K, dlab.p, dbest.p, nullptr));
    BTRY(hipMemcpy(lab.data(), dlab.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    BTRY(hipMemcpy(best.data(), dbest.p, sizeof(double) * n, hipMemcpyDeviceToHost));
    return SBV_OK;
  };
  sbv_status st = assign();
  if (st) return st;
  progress("anchor assignment done, clusters", (double)K);
  for (int it = 0; it < lloyd; ++it) {
    cluster_means(Z, n, d, lab, K, C, cnt);
    for (int64_t c = 0; c < K; ++c) {
      if (cnt[c]) continue;
      // re-seed an empty cluster with the point farthest from its own centre
      double far = -1.0;
      int64_t fi = -1;
      for (int64_t i = 0; i < n; ++i) {
        if (cnt[lab[i]] <= 1) continue;
        double t = sqd(&Z[i * d], &C[(int64_t)lab[i] * d], d);
        if (t > far) {
          far = t;
          fi = i;
        }
      }
      if (fi < 0) continue;
      --cnt[lab[fi]];
      lab[fi] = (int32_t)c;
      cnt[c] = 1;
      std::memcpy(&C[c * d], &Z[fi * d], sizeof(double) * d);
    }
    prev = lab;
    st = assign();
    if (st) return st;
    progress("lloyd pass", (double)(it + 1), (double)lloyd);
    if (prev == lab) break;
  }
  // 5. size bounds
  for (int round = 0; round < 16; ++round) {
    bool changed = false;
    cluster_means(Z, n, d, lab, K, C, cnt);
    if (o.max_bs > 0) {
      std::vector<std::vector<int64_t>> members(K);
      for (int64_t i = 0; i < n; ++i)
        if (cnt[lab[i]] > o.max_bs) members[lab[i]].push_back(i);
      const int64_t K0 = K;
      for (int64_t c = 0; c < K0; ++c) {
        auto& mem = members[c];
        if (mem.empty()) continue;
        int ax = 0;
        double bv = -1.0;
        for (int k = 0; k < d; ++k) {
          double v = 0.0;
          for (int64_t i : mem) {
            double t = Z[i * d + k] - C[c * d + k];
            v += t * t;
          }
          if (v > bv) {
            bv = v;
            ax = k;
          }
        }
        std::stable_sort(mem.begin(), mem.end(), [&](int64_t a, int64_t b) {
          double za = Z[a * d + ax], zb = Z[b * d + ax];
          return za < zb || (za == zb && a < b);
        });
        const int64_t s = (int64_t)mem.size(), pieces = (s + o.max_bs - 1) / o.max_bs;
        for (int64_t p = 1; p < pieces; ++p) {
          for (int64_t t = p * s / pieces; t < (p + 1) * s / pieces; ++t) lab[mem[t]] = (int32_t)K;
          ++K;
        }
        changed = true;
      }
      if (changed) cluster_means(Z, n, d, lab, K, C, cnt);
    }
    if (o.min_bs > 0) {
      std::vector<std::vector<int64_t>> members(K);
      for (int64_t i = 0; i < n; ++i)
        if (cnt[lab[i]] < o.min_bs) members[lab[i]].push_back(i);
      for (int64_t c = 0; c < K; ++c) {
        if (cnt[c] == 0 || cnt[c] >= o.min_bs) continue;
        double bestd = INFINITY;
        int64_t to = -1;
        for (int64_t t = 0; t < K; ++t) {
          if (t == c || cnt[t] == 0) continue;
          if (o.max_bs > 0 && cnt[t] + cnt[c] > o.max_bs) continue;
          double dd = sqd(&C[c * d], &C[t * d], d);
          if (dd < bestd) {
            bestd = dd;
            to = t;
          }
        }
        if (to < 0) continue;
        for (int64_t i : members[c]) lab[i] = (int32_t)to;
        if (cnt[to] < o.min_bs) members[to].insert(members[to].end(), members[c].begin(), members[c].end());
        members[c].clear();
        for (int k = 0; k < d; ++k)
          C[to * d + k] = (C[to * d + k] * cnt[to] + C[c * d + k] * cnt[c]) / (double)(cnt[to] + cnt[c]);
        cnt[to] += cnt[c];
        cnt[c] = 0;
        changed = true;
      }
    }
    if (!changed) break;
  }
  // drop empty clusters
  cluster_means(Z, n, d, lab, K, C, cnt);
  {
    std::vector<int64_t> remap(K, -1);
    int64_t Kf = 0;
    for (int64_t c = 0; c < K; ++c)
      if (cnt[c]) remap[c] = Kf++;
    for (int64_t i = 0; i < n; ++i) lab[i] = (int32_t)remap[lab[i]];
    K = Kf;
  }
  return SBV_OK;
}

// Filtered exact neighbour search (Alg. 4 with the distance threshold of
// Eq. (distancethreashold)).  Query block q (rank q, m_q neighbours among
// the n_q points of earlier blocks) starts from the radius lambda_q of a ball
// expected to hold alpha m_q of them:
//   lambda_q = (alpha m_q zeta_d V / n_q)^(1/d),  zeta_d = Gamma(d/2 + 1) / pi^(d/2),
// V the volume of the scaled inputs' bounding box.  Candidate blocks pass
// ||c_q - c_j|| <= lambda_q + radius_j, candidate points ||z - c_q|| <= lambda_q,
// and the answer is exact once at least m_q points lie within lambda_q.
// Queries that fall short retry with lambda_q 4^(1/d) (a ball expected to
// hold four times as many points), four times at most; what
// remains, queries whose candidate list overflows, and queries with fewer
// than 8 m_q earlier points go to the brute-force search.
sbv_status filtered_knn(const std::vector<double>& Zo, const std::vector<double>& cen, const std::vector<int32_t>& bp,
                        const std::vector<int64_t>& nptr, int64_t n, int d, int64_t K, double alpha, const double* dZo,
                        const double* dcen, const int32_t* dbp, const int64_t* dnp, int32_t* dpos) {
  // block radii and the bounding-box volume of the scaled inputs
  std::vector<double> rad(K, 0.0), lo(d, INFINITY), hi(d, -INFINITY);
  for (int64_t r = 0; r < K; ++r)
    for (int64_t t = bp[r]; t < bp[r + 1]; ++t) {
      double s2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double z = Zo[(size_t)t * d + k];
        const double df = z - cen[(size_t)r * d + k];
        s2 += df * df;
        lo[k] = std::min(lo[k], z);
        hi[k] = std::max(hi[k], z);
      }
      rad[r] = std::max(rad[r], std::sqrt(s2));
    }
  double logV = 0.0;
  for (int k = 0; k < d; ++k) logV += std::log(std::max(hi[k] - lo[k], 1e-300));
  const double log_zeta = std::lgamma(0.5 * d + 1.0) - 0.5 * d * std::log(M_PI);
  std::vector<int32_t> pending, brute;
  std::vector<double> lam(K, 0.0);
  for (int64_t q = 0; q < K; ++q) {
    const int64_t mq = nptr[q + 1] - nptr[q];
    if (mq == 0) continue;
    if (bp[q] < 8 * mq) {
      brute.push_back((int32_t)q);
      continue;
    }
    lam[q] = std::exp((std::log(alpha * (double)mq) + log_zeta + logV - std::log((double)bp[q])) / d);
    pending.push_back((int32_t)q);
  }
  constexpr int kCap = 16384;     // candidate blocks per query
  constexpr int kBatch = 8192;    // queries per pass
  Dev<double> drad, dlam;
  Dev<int32_t> dq, dcand, dcnt, dst;
  BTRY(drad.alloc(K));
  BTRY(hipMemcpy(drad.p, rad.data(), sizeof(double) * K, hipMemcpyHostToDevice));
  BTRY(dlam.alloc(kBatch));
  BTRY(dq.alloc(std::max<int64_t>(K, 1)));
  BTRY(dcand.alloc((size_t)kBatch * kCap));
  BTRY(dcnt.alloc(kBatch));
  BTRY(dst.alloc(kBatch));
  for (int attempt = 0; attempt < 5 && !pending.empty(); ++attempt) {
    std::vector<int32_t> failed;
    progress("filtered neighbour search, pass / queries", (double)attempt, (double)pending.size());
    for (size_t b0 = 0; b0 < pending.size(); b0 += kBatch) {
      if ((b0 / kBatch) % 16 == 15) progress("  queries done", (double)b0, (double)pending.size());
      const int nb = (int)std::min<size_t>(kBatch, pending.size() - b0);
      std::vector<double> lb(nb);
      for (int i = 0; i < nb; ++i) lb[i] = lam[pending[b0 + i]];
      BTRY(hipMemcpy(dq.p, pending.data() + b0, sizeof(int32_t) * nb, hipMemcpyHostToDevice));
      BTRY(hipMemcpy(dlam.p, lb.data(), sizeof(double) * nb, hipMemcpyHostToDevice));
      BTRY(launch_knn_coarse(dcen, drad.p, d, dq.p, nb, dlam.p, kCap, dcand.p, dcnt.p, nullptr));
      BTRY(launch_knn_fine(dZo, d, dcen, dbp, dq.p, nb, dlam.p, kCap, dcand.p, dcnt.p, dnp, dpos, dst.p, nullptr));
      std::vector<int32_t> sb(nb);
      BTRY(hipMemcpy(sb.data(), dst.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost));
      for (int i = 0; i < nb; ++i) {
        if (sb[i] == 1) failed.push_back(pending[b0 + i]);
        if (sb[i] == 2) brute.push_back(pending[b0 + i]);
      }
    }
    const double grow = std::pow(4.0, 1.0 / d);  // four times the expected points inside
    for (int32_t q : failed) lam[q] *= grow;
    pending.swap(failed);
  }
  brute.insert(brute.end(), pending.begin(), pending.end());
  std::sort(brute.begin(), brute.end());
  if (!brute.empty()) {
    int mmax = 0;
    for (int32_t q : brute) mmax = std::max<int>(mmax, (int)(nptr[q + 1] - nptr[q]));
    BTRY(hipMemcpy(dq.p, brute.data(), sizeof(int32_t) * brute.size(), hipMemcpyHostToDevice));
    BTRY(launch_knn(dZo, d, dcen, dbp, (int)K, mmax, dnp, dpos, nullptr, dq.p, (int)brute.size()));
  }
  return SBV_OK;
}

}  // namespace

extern "C" sbv_status sbv_build_blocks(const double* X, const double* y, int64_t n, int32_t d,
                                       const double* beta_build, int64_t n_blocks, int32_t m,
                                       const sbv_build_opts* opts, sbv_blocks* out) {
  if (!X || !beta_build || !out) return sbv_internal_fail(SBV_E_INVAL, "X, beta_build and out are required");
  if (n <= 0 || d <= 0 || d > kMaxDim || n_blocks <= 0 || n_blocks > n || m < 0)
    return sbv_internal_fail(SBV_E_INVAL, "need n > 0, 0 < d <= 20, 0 < n_blocks <= n, m >= 0");
  if (n > INT32_MAX - 1 || n_blocks > INT32_MAX / 2) return sbv_internal_fail(SBV_E_INVAL, "n too large");
  if (m > knn_max_m()) return sbv_internal_fail(SBV_E_INVAL, "m exceeds the neighbour-search capacity");
  sbv_build_opts o{SBV_KMEANS, 10, 0, 0, 0, 0, 0.0};
  if (opts) o = *opts;
  if (o.method != SBV_KMEANS && o.method != SBV_RAC) return sbv_internal_fail(SBV_E_INVAL, "unknown method");
  if (o.min_bs < 0 || o.max_bs < 0 || (o.max_bs > 0 && o.min_bs > o.max_bs))
    return sbv_internal_fail(SBV_E_INVAL, "bad size bounds");
  for (int k = 0; k < d; ++k)
    if (!(beta_build[k] > 0.0) || !std::isfinite(beta_build[k]))
      return sbv_internal_fail(SBV_E_INVAL, "beta_build must be positive and finite");
  for (int64_t i = 0; i < n * d; ++i)
    if (!std::isfinite(X[i])) return sbv_internal_fail(SBV_E_INVAL, "X has non-finite values");
  const int lloyd = o.method == SBV_RAC ? 0 : std::max(0, o.lloyd_iters);
  if (!(o.nns_alpha >= 0.0) && !(o.nns_alpha < 0.0)) return sbv_internal_fail(SBV_E_INVAL, "nns_alpha is NaN");
  int64_t K = n_blocks;

  // 1. scaling
  std::vector<double> Z((size_t)n * d);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < d; ++k) Z[i * d + k] = X[i * d + k] / beta_build[k];
  std::vector<int32_t> lab;
  sbv_status st = SBV_OK;
  if (o.n_slabs <= 1) {
    st = cluster_points(Z, n, d, K, o, o.seed, lloyd, lab);
    if (st) return st;
  } else {
    // Alg. 2: slabs of equal point count along the scaled dimension of largest
    // extent (the most relevant input); each slab is clustered on its own with
    // a share of the K blocks proportional to its size
    int ax = 0;
    double ext = -1.0;
    for (int k = 0; k < d; ++k) {
      double lo = INFINITY, hi = -INFINITY;
      for (int64_t i = 0; i < n; ++i) {
        lo = std::min(lo, Z[i * d + k]);
        hi = std::max(hi, Z[i * d + k]);
      }
      if (hi - lo > ext) {
        ext = hi - lo;
        ax = k;
      }
    }
    std::vector<int64_t> ids(n);
    std::iota(ids.begin(), ids.end(), 0);
    std::stable_sort(ids.begin(), ids.end(), [&](int64_t a, int64_t b) { return Z[a * d + ax] < Z[b * d + ax]; });
    const int S = (int)std::min<int64_t>(o.n_slabs, K);
    lab.assign(n, 0);
    int64_t koff = 0;
    for (int sl = 0; sl < S; ++sl) {
      const int64_t i0 = sl * n / S, i1 = (sl + 1) * n / S, ns = i1 - i0;
      int64_t Ks = std::max<int64_t>(1, (int64_t)std::llround((double)K * ns / n));
      Ks = std::min(Ks, ns);
      std::vector<double> Zs((size_t)ns * d);
      for (int64_t t = 0; t < ns; ++t) std::memcpy(&Zs[t * d], &Z[ids[i0 + t] * d], sizeof(double) * d);
      std::vector<int32_t> ls;
      st = cluster_points(Zs, ns, d, Ks, o, o.seed + 0x10000ull * (uint64_t)sl, lloyd, ls);
      if (st) return st;
      for (int64_t t = 0; t < ns; ++t) lab[ids[i0 + t]] = (int32_t)(koff + ls[t]);
      koff += Ks;
    }
    K = koff;
  }
  progress("clusters after size bounds", (double)K);
  // 6. random block order
  std::vector<int64_t> order(K), rank_of(K);
  std::iota(order.begin(), order.end(), 0);
  {
    Splitmix ro{o.seed + 1};
    for (int64_t i = K - 1; i > 0; --i) {
      int64_t j = (int64_t)ro.below((uint64_t)(i + 1));
      std::swap(order[i], order[j]);
    }
  }
  for (int64_t r = 0; r < K; ++r) rank_of[order[r]] = r;
  // 7. ordered points and centroids
  std::vector<int64_t> bptr(K + 1, 0), pts(n);
  for (int64_t i = 0; i < n; ++i) ++bptr[rank_of[lab[i]] + 1];
  for (int64_t r = 0; r < K; ++r) bptr[r + 1] += bptr[r];
  {
    std::vector<int64_t> fill(bptr.begin(), bptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) pts[fill[rank_of[lab[i]]]++] = i;
  }
  std::vector<double> cen((size_t)K * d, 0.0), Zo((size_t)n * d);
  for (int64_t r = 0; r < K; ++r) {
    for (int64_t t = bptr[r]; t < bptr[r + 1]; ++t)
      for (int k = 0; k < d; ++k) cen[r * d + k] += Z[pts[t] * d + k];
    for (int k = 0; k < d; ++k) cen[r * d + k] /= (double)(bptr[r + 1] - bptr[r]);
  }
  for (int64_t t = 0; t < n; ++t) std::memcpy(&Zo[t * d], &Z[pts[t] * d], sizeof(double) * d);
  std::vector<int64_t> nptr(K + 1, 0);
  for (int64_t r = 0; r < K; ++r) nptr[r + 1] = nptr[r] + std::min<int64_t>(m, bptr[r]);
  const int64_t nnz = nptr[K];
  if (nnz > INT32_MAX) return sbv_internal_fail(SBV_E_INVAL, "too many conditioning entries");
  // 8. neighbours on the device: the filtered search (expansion factor alpha;
  //    0 = automatic: 3 from 2048 blocks on, brute force below; < 0 = brute force)
  const double alpha = o.nns_alpha > 0.0 ? o.nns_alpha : (o.nns_alpha == 0.0 && K >= 2048 ? 3.0 : 0.0);
  std::vector<int32_t> bp32(K + 1), npos(std::max<int64_t>(nnz, 1));
  for (int64_t r = 0; r <= K; ++r) bp32[r] = (int32_t)bptr[r];
  {
    Dev<double> dZo, dcen;
    Dev<int32_t> dbp, dpos;
    Dev<int64_t> dnp;
    BTRY(dZo.alloc((size_t)n * d));
    BTRY(dcen.alloc((size_t)K * d));
    BTRY(dbp.alloc(K + 1));
    BTRY(dnp.alloc(K + 1));
    BTRY(dpos.alloc(std::max<int64_t>(nnz, 1)));
    BTRY(hipMemcpy(dZo.p, Zo.data(), sizeof(double) * n * d, hipMemcpyHostToDevice));
    BTRY(hipMemcpy(dcen.p, cen.data(), sizeof(double) * K * d, hipMemcpyHostToDevice));
    BTRY(hipMemcpy(dbp.p, bp32.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice));
    BTRY(hipMemcpy(dnp.p, nptr.data(), sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice));
    if (alpha > 0.0) {
      st = filtered_knn(Zo, cen, bp32, nptr, n, d, K, alpha, dZo.p, dcen.p, dbp.p, dnp.p, dpos.p);
      if (st) return st;
    } else {
      BTRY(launch_knn(dZo.p, d, dcen.p, dbp.p, (int)K, m, dnp.p, dpos.p, nullptr));
    }
    BTRY(hipMemcpy(npos.data(), dpos.p, sizeof(int32_t) * std::max<int64_t>(nnz, 1), hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> nidx(std::max<int64_t>(nnz, 1));
  for (int64_t t = 0; t < nnz; ++t) nidx[t] = pts[npos[t]];
  progress("neighbours done");
  // 9. pack
  st = sbv_internal_make_handle(X, y, n, d, K, bptr.data(), pts.data(), nptr.data(), nidx.data(), out);
  if (st == SBV_OK) sbv_internal_set_build(*out, beta_build, n_blocks, m, o);
  return st;
}
