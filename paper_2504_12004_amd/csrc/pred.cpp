// Prediction by block-conditional distributions (Sec. 4.2's predictive
// product over new blocks, Sec. 5.5 GP Prediction).
//
// A prediction structure groups new inputs X* into blocks B*_j and gives each
// block its m_pred nearest observed points NN(B*_j).  For every block the
// joint covariance of [NN(B*_j); B*_j] is factored by the same register-tile
// kernel as the likelihood, in its conditional-simulation mode with zero
// innovations: the emitted values are the conditional mean mu_new of Alg. 5
// Step 1, and the squares of the trailing factor's rows give
// diag(Sigma_new) = diag(L' L'^T), the predictive variance of a new
// observation.  Draw summaries (1000 draws per point in the paper, 95 %
// intervals) run in their own kernel on the caller's innovations.
//
// The structure keeps one device copy of the observed inputs followed by the
// new ones, so that the kernel addresses both through one coordinate array;
// the observations are copied from the handle at every prediction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/sbv.h"
#include "sbv_internal.h"


sbv_status sbv_internal_fail(sbv_status st, const char* msg);
sbv_status sbv_internal_view(sbv_blocks h, sbv::HandleView* v);

using namespace sbv;

namespace {

#define PTRY(expr)                                                                                  \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess)                                                                           \
      return sbv_internal_fail(e_ == hipErrorOutOfMemory ? SBV_E_NOMEM : SBV_E_DEVICE,              \
                               (std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)) \
                                   .c_str());                                                       \
  } while (0)

template <typename T>
struct PBuf {
  T* p = nullptr;
  PBuf() = default;
  PBuf(const PBuf&) = delete;
  PBuf& operator=(const PBuf&) = delete;
  ~PBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc((void**)&p, sizeof(T) * std::max<size_t>(n, 1)); }
};

}  // namespace

struct sbv_pred_s {
  sbv_blocks h = nullptr;
  int64_t n_obs = 0, n_pred = 0, K = 0, nnz = 0;
  int32_t d = 0;
  // host, exchange format: blocks as prediction ids, neighbours as observed ids
  std::vector<int64_t> block_ptr, block_pts, nn_ptr, nn_idx;
  // device
  PBuf<double> X, y;        // (n_obs + n_pred) x d inputs and observations (new points: 0)
  PBuf<int32_t> bptr, nidx;  // block ranges (ordered positions, new points after the observed ones)
  PBuf<int64_t> nptr;
  PBuf<double> llb, mean, var, theta;
  PBuf<int32_t> flag;
  PBuf<SetDesc> desc;
  std::vector<int> b_variant, b_off, b_count;
  PBuf<WorkItem> items;
  PBuf<int> dcount;
};

namespace {

sbv_status check_theta(const double* theta, int d) {
  for (int k = 0; k < d + 2; ++k)
    if (!std::isfinite(theta[k])) return sbv_internal_fail(SBV_E_INVAL, "theta has non-finite values");
  return SBV_OK;
}

}  // namespace

extern "C" {

sbv_status sbv_pred_import(sbv_blocks h, const double* Xp, int64_t n_pred, int64_t K, const int64_t* block_ptr,
                           const int64_t* block_pts, const int64_t* nn_ptr, const int64_t* nn_idx, sbv_pred* out) {
  if (!h || !Xp || !block_ptr || !block_pts || !nn_ptr || !out)
    return sbv_internal_fail(SBV_E_INVAL, "handle, Xp, structure arrays and out are required");
  HandleView v{};
  sbv_status st = sbv_internal_view(h, &v);
  if (st) return st;
  const int d = v.d;
  if (n_pred <= 0 || K <= 0 || K > n_pred) return sbv_internal_fail(SBV_E_INVAL, "need 0 < K <= n_pred");
  if (v.n + n_pred > INT32_MAX - 1) return sbv_internal_fail(SBV_E_INVAL, "too many points");
  if (block_ptr[0] != 0 || block_ptr[K] != n_pred || nn_ptr[0] != 0)
    return sbv_internal_fail(SBV_E_INVAL, "block_ptr must run from 0 to n_pred and nn_ptr start at 0");
  if (nn_ptr[K] > 0 && !nn_idx) return sbv_internal_fail(SBV_E_INVAL, "nn_idx is required");
  for (int64_t i = 0; i < n_pred * d; ++i)
    if (!std::isfinite(Xp[i])) return sbv_internal_fail(SBV_E_INVAL, "Xp has non-finite values");
  std::vector<char> seen(n_pred, 0);
  std::vector<int32_t> pos_obs(v.n);
  for (int64_t t = 0; t < v.n; ++t) pos_obs[v.block_pts_host[t]] = (int32_t)t;
  const int cap = variant(n_variants() - 1).ntm * kTile;
  auto P = std::make_unique<sbv_pred_s>();
  P->h = h;
  P->n_obs = v.n;
  P->n_pred = n_pred;
  P->K = K;
  P->d = d;
  P->nnz = nn_ptr[K];
  std::vector<std::vector<std::pair<int32_t, int32_t>>> per(n_variants());
  for (int64_t r = 0; r < K; ++r) {
    if (block_ptr[r + 1] <= block_ptr[r] || nn_ptr[r + 1] < nn_ptr[r])
      return sbv_internal_fail(SBV_E_INVAL, "empty prediction block or decreasing nn_ptr");
    for (int64_t t = block_ptr[r]; t < block_ptr[r + 1]; ++t) {
      const int64_t p = block_pts[t];
      if (p < 0 || p >= n_pred || seen[p]) return sbv_internal_fail(SBV_E_INVAL, "block_pts is not a permutation");
      seen[p] = 1;
    }
    for (int64_t t = nn_ptr[r]; t < nn_ptr[r + 1]; ++t)
      if (nn_idx[t] < 0 || nn_idx[t] >= v.n) return sbv_internal_fail(SBV_E_INVAL, "neighbour id out of range");
    const int64_t joint = (nn_ptr[r + 1] - nn_ptr[r]) + (block_ptr[r + 1] - block_ptr[r]);
    if (joint > cap)
      return sbv_internal_fail(SBV_E_INVAL, ("prediction block " + std::to_string(r) + " has joint size " +
                                             std::to_string(joint) + "; prediction supports up to " +
                                             std::to_string(cap)).c_str());
    per[variant_for((int)joint)].push_back({(int32_t)joint, (int32_t)r});
  }
  P->block_ptr.assign(block_ptr, block_ptr + K + 1);
  P->block_pts.assign(block_pts, block_pts + n_pred);
  P->nn_ptr.assign(nn_ptr, nn_ptr + K + 1);
  P->nn_idx.assign(nn_idx, nn_idx + P->nnz);
  // device arrays: inputs (observed in rank order, then new points in block order)
  const int64_t nall = v.n + n_pred;
  std::vector<double> Xo((size_t)n_pred * d);
  for (int64_t t = 0; t < n_pred; ++t) std::memcpy(&Xo[(size_t)t * d], Xp + block_pts[t] * d, sizeof(double) * d);
  std::vector<int32_t> bp(K + 1), ni(std::max<int64_t>(P->nnz, 1), 0);
  for (int64_t r = 0; r <= K; ++r) bp[r] = (int32_t)(v.n + block_ptr[r]);
  for (int64_t t = 0; t < P->nnz; ++t) ni[t] = pos_obs[nn_idx[t]];
  PTRY(P->X.alloc((size_t)nall * d));
  PTRY(P->y.alloc(nall));
  PTRY(P->bptr.alloc(K + 1));
  PTRY(P->nptr.alloc(K + 1));
  PTRY(P->nidx.alloc(ni.size()));
  PTRY(P->llb.alloc(K));
  PTRY(P->flag.alloc(K));
  PTRY(P->mean.alloc(n_pred));
  PTRY(P->var.alloc(n_pred));
  PTRY(P->theta.alloc(d + 2));
  PTRY(P->desc.alloc(1));
  PTRY(hipMemcpy(P->X.p, v.X, sizeof(double) * v.n * d, hipMemcpyDeviceToDevice));
  PTRY(hipMemcpy(P->X.p + v.n * d, Xo.data(), sizeof(double) * n_pred * d, hipMemcpyHostToDevice));
  PTRY(hipMemset(P->y.p + v.n, 0, sizeof(double) * n_pred));
  PTRY(hipMemcpy(P->bptr.p, bp.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice));
  PTRY(hipMemcpy(P->nptr.p, nn_ptr, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice));
  PTRY(hipMemcpy(P->nidx.p, ni.data(), sizeof(int32_t) * ni.size(), hipMemcpyHostToDevice));
  // work lists per register variant, longest first
  std::vector<WorkItem> it;
  for (int vv = n_variants() - 1; vv >= 0; --vv) {
    if (per[vv].empty()) continue;
    std::stable_sort(per[vv].begin(), per[vv].end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    P->b_variant.push_back(vv);
    P->b_off.push_back((int)it.size());
    P->b_count.push_back((int)per[vv].size());
    for (const auto& e : per[vv]) it.push_back(WorkItem{0, e.second});
  }
  PTRY(P->items.alloc(it.size()));
  PTRY(hipMemcpy(P->items.p, it.data(), sizeof(WorkItem) * it.size(), hipMemcpyHostToDevice));
  PTRY(P->dcount.alloc(P->b_count.size()));
  PTRY(hipMemcpy(P->dcount.p, P->b_count.data(), sizeof(int) * P->b_count.size(), hipMemcpyHostToDevice));
  *out = P.release();
  return SBV_OK;
}

sbv_status sbv_pred_build(sbv_blocks h, const double* Xp, int64_t n_pred, const double* beta_build, int64_t n_blocks,
                          int32_t m_pred, const sbv_build_opts* opts, sbv_pred* out) {
  if (!h || !Xp || !beta_build || !out) return sbv_internal_fail(SBV_E_INVAL, "handle, Xp, beta_build and out are required");
  HandleView v{};
  sbv_status st = sbv_internal_view(h, &v);
  if (st) return st;
  const int d = v.d;
  if (m_pred < 0 || m_pred > knn_max_m()) return sbv_internal_fail(SBV_E_INVAL, "m_pred out of range");
  // 1. blocks of the new points: the builder's clustering (scaling, anchors,
  //    Lloyd passes, size bounds) with no conditioning
  sbv_blocks tmp = nullptr;
  st = sbv_build_blocks(Xp, nullptr, n_pred, d, beta_build, n_blocks, 0, opts, &tmp);
  if (st) return st;
  int64_t nn = 0, K = 0;
  sbv_blocks_info(tmp, &nn, nullptr, &K, nullptr);
  std::vector<int64_t> bptr(K + 1), bpts(n_pred), dummy(K + 1);
  st = sbv_blocks_export(tmp, bptr.data(), bpts.data(), dummy.data(), nullptr);
  sbv_blocks_free(tmp);
  if (st) return st;
  // 2. neighbours: the m_pred observed points nearest each block centroid
  //    (scaled by beta_build), exact search over every observed point
  const int64_t mm = std::min<int64_t>(m_pred, v.n);
  std::vector<double> Xo((size_t)v.n * d), Zo((size_t)v.n * d), cen((size_t)K * d, 0.0);
  PTRY(hipMemcpy(Xo.data(), v.X, sizeof(double) * v.n * d, hipMemcpyDeviceToHost));
  for (int64_t t = 0; t < v.n; ++t)
    for (int k = 0; k < d; ++k) Zo[(size_t)t * d + k] = Xo[(size_t)t * d + k] / beta_build[k];
  for (int64_t r = 0; r < K; ++r) {
    for (int64_t t = bptr[r]; t < bptr[r + 1]; ++t)
      for (int k = 0; k < d; ++k) cen[(size_t)r * d + k] += Xp[bpts[t] * d + k] / beta_build[k];
    for (int k = 0; k < d; ++k) cen[(size_t)r * d + k] /= (double)(bptr[r + 1] - bptr[r]);
  }
  std::vector<int64_t> nptr(K + 1);
  for (int64_t r = 0; r <= K; ++r) nptr[r] = r * mm;
  std::vector<int32_t> pref(K, (int32_t)v.n), npos(std::max<int64_t>(K * mm, 1));
  {
    PBuf<double> dZ, dC;
    PBuf<int32_t> dpref, dpos;
    PBuf<int64_t> dnp;
    PTRY(dZ.alloc((size_t)v.n * d));
    PTRY(dC.alloc((size_t)K * d));
    PTRY(dpref.alloc(K));
    PTRY(dnp.alloc(K + 1));
    PTRY(dpos.alloc(npos.size()));
    PTRY(hipMemcpy(dZ.p, Zo.data(), sizeof(double) * v.n * d, hipMemcpyHostToDevice));
    PTRY(hipMemcpy(dC.p, cen.data(), sizeof(double) * K * d, hipMemcpyHostToDevice));
    PTRY(hipMemcpy(dpref.p, pref.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice));
    PTRY(hipMemcpy(dnp.p, nptr.data(), sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice));
    if (mm > 0) PTRY(launch_knn(dZ.p, d, dC.p, dpref.p, (int)K, (int)mm, dnp.p, dpos.p, nullptr));
    PTRY(hipMemcpy(npos.data(), dpos.p, sizeof(int32_t) * npos.size(), hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> nidx(std::max<int64_t>(K * mm, 1));
  for (int64_t t = 0; t < K * mm; ++t) nidx[t] = v.block_pts_host[npos[t]];
  return sbv_pred_import(h, Xp, n_pred, K, bptr.data(), bpts.data(), nptr.data(), nidx.data(), out);
}

sbv_status sbv_pred_info(sbv_pred p, int64_t* n_pred, int64_t* K, int64_t* nnz) {
  if (!p) return sbv_internal_fail(SBV_E_INVAL, "null prediction structure");
  if (n_pred) *n_pred = p->n_pred;
  if (K) *K = p->K;
  if (nnz) *nnz = p->nnz;
  return SBV_OK;
}

sbv_status sbv_pred_export(sbv_pred p, int64_t* block_ptr, int64_t* block_pts, int64_t* nn_ptr, int64_t* nn_idx) {
  if (!p) return sbv_internal_fail(SBV_E_INVAL, "null prediction structure");
  if (block_ptr) std::memcpy(block_ptr, p->block_ptr.data(), sizeof(int64_t) * (p->K + 1));
  if (block_pts) std::memcpy(block_pts, p->block_pts.data(), sizeof(int64_t) * p->n_pred);
  if (nn_ptr) std::memcpy(nn_ptr, p->nn_ptr.data(), sizeof(int64_t) * (p->K + 1));
  if (nn_idx && p->nnz) std::memcpy(nn_idx, p->nn_idx.data(), sizeof(int64_t) * p->nnz);
  return SBV_OK;
}

void sbv_pred_free(sbv_pred p) { delete p; }

sbv_status sbv_predict(sbv_pred p, const double* theta, int32_t two_nu, double* mean, double* var) {
  if (!p || !theta || !mean || !var) return sbv_internal_fail(SBV_E_INVAL, "structure, theta, mean and var are required");
  if (two_nu != 1 && two_nu != 3 && two_nu != 5 && two_nu != 7)
    return sbv_internal_fail(SBV_E_INVAL, "two_nu must be 1, 3, 5 or 7");
  sbv_status st = check_theta(theta, p->d);
  if (st) return st;
  HandleView v{};
  st = sbv_internal_view(p->h, &v);
  if (st) return st;
  if (v.n != p->n_obs || v.d != p->d) return sbv_internal_fail(SBV_E_INVAL, "the observed handle changed shape");
  PTRY(hipMemcpy(p->y.p, v.y, sizeof(double) * v.n, hipMemcpyDeviceToDevice));
  PTRY(hipMemcpy(p->theta.p, theta, sizeof(double) * (p->d + 2), hipMemcpyHostToDevice));
  SetDesc D{};
  D.X = p->X.p;
  D.y = p->y.p;
  D.bptr = p->bptr.p;
  D.nptr = p->nptr.p;
  D.nidx = p->nidx.p;
  D.llb = p->llb.p;
  D.flag = p->flag.p;
  D.xi = nullptr;  // zero innovations: the emitted values are the conditional means
  D.y_out = p->mean.p;
  D.var_out = p->var.p;
  D.d = p->d;
  D.two_nu = two_nu;
  D.theta_off = 0;
  D.K = (int32_t)p->K;
  D.out_off = (int32_t)p->n_obs;
  PTRY(hipMemcpy(p->desc.p, &D, sizeof(SetDesc), hipMemcpyHostToDevice));
  for (size_t b = 0; b < p->b_variant.size(); ++b)
    PTRY(launch_sample(p->b_variant[b], p->b_count[b], p->desc.p, p->theta.p, p->items.p + p->b_off[b],
                       p->dcount.p + b, nullptr));
  std::vector<double> m(p->n_pred), vv(p->n_pred);
  std::vector<int32_t> fl(p->K);
  PTRY(hipMemcpy(m.data(), p->mean.p, sizeof(double) * p->n_pred, hipMemcpyDeviceToHost));
  PTRY(hipMemcpy(vv.data(), p->var.p, sizeof(double) * p->n_pred, hipMemcpyDeviceToHost));
  PTRY(hipMemcpy(fl.data(), p->flag.p, sizeof(int32_t) * p->K, hipMemcpyDeviceToHost));
  int64_t bad = -1;
  for (int64_t r = 0; r < p->K; ++r) {
    const bool b = fl[r] & 2;
    if (b && bad < 0) bad = r;
    for (int64_t t = p->block_ptr[r]; t < p->block_ptr[r + 1]; ++t) {
      mean[p->block_pts[t]] = b ? NAN : m[t];
      var[p->block_pts[t]] = b ? NAN : vv[t];
    }
  }
  if (bad >= 0)
    return sbv_internal_fail(SBV_E_NOTPD, ("prediction block " + std::to_string(bad) +
                                           " is not positive definite in FP64").c_str());
  return SBV_OK;
}

sbv_status sbv_predict_draws_dev(const double* mean_dev, const double* var_dev, int64_t n_pred, const double* xi_dev,
                                 int32_t n_draws, double* stats_dev, void* stream) {
  if (!mean_dev || !var_dev || !xi_dev || !stats_dev || n_pred <= 0 || n_draws <= 0)
    return sbv_internal_fail(SBV_E_INVAL, "device buffers, n_pred > 0 and n_draws > 0 are required");
  PTRY(launch_pred_draws(mean_dev, var_dev, n_pred, xi_dev, n_draws, stats_dev, (hipStream_t)stream));
  return SBV_OK;
}

}  // extern "C"
