// C-ABI of libsbv.so: handles, structure import/export, evaluation plans.
//
// A handle holds one dataset resident on the device in block-rank order (the
// contiguous arrangement of blocks, neighbours and observations described in
// Sec. 5.3/5.4: copied to the device once, then every evaluation only moves
// parameters in and log-likelihoods out).  An evaluation plan groups the
// blocks of one or more handles into size buckets (joint size m_i + b_i), each
// served by a kernel variant whose register tiles fit that size, ordered
// longest first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/sbv.h"
#include "sbv_internal.h"

using namespace sbv;

namespace {

thread_local std::string g_err;

sbv_status fail(sbv_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? SBV_E_NOMEM : SBV_E_DEVICE,                  \
                  std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_));    \
  } while (0)

// Owning device buffer (move-only).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t alloc(size_t count) {
    reset();
    n = count;
    if (count == 0) return hipSuccess;
    return hipMalloc((void**)&p, sizeof(T) * count);
  }
};

}  // namespace

struct Plan;

struct sbv_blocks_s {
  int64_t n = 0, K = 0, nnz = 0;
  int32_t d = 0;
  int32_t max_joint = 0;
  // host copies in the exchange format
  std::vector<int64_t> block_ptr, block_pts, nn_ptr, nn_idx;
  std::vector<int32_t> joint;  // m_i + b_i per block
  // device, rank order
  DevBuf<double> X, y;
  DevBuf<int32_t> bptr, nidx, pos_of;
  DevBuf<int64_t> nptr;
  DevBuf<double> llb, gradb;
  DevBuf<int32_t> flag;
  int64_t last_fallback = 0;
  int32_t last_two_nu = 0;
};

// ---- evaluation plans ------------------------------------------------------
struct Bucket {
  int variant = -1;
  int count = 0;           // host copy of the item count
  DevBuf<WorkItem> items;  // sorted by joint size, longest first
  DevBuf<int> dcount;      // device copy of count
  DevBuf<WorkItem> fb_items;
  DevBuf<int> fb_count;
};

struct Plan {
  std::vector<sbv_blocks> sets;
  std::vector<int32_t> two_nu;
  std::vector<int32_t> theta_off;
  int theta_len = 0;
  DevBuf<SetDesc> dsets;
  std::vector<Bucket> buckets;
  DevBuf<double> theta, out;
  DevBuf<int> bad;
};

namespace {

std::mutex g_plan_mu;
std::vector<std::unique_ptr<Plan>> g_plans;

void drop_plans_of(sbv_blocks h) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.erase(std::remove_if(g_plans.begin(), g_plans.end(),
                               [h](const std::unique_ptr<Plan>& p) {
                                 return std::find(p->sets.begin(), p->sets.end(), h) != p->sets.end();
                               }),
                g_plans.end());
}

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

sbv_status check_sets(const sbv_blocks* sets, int32_t n_sets, const int32_t* two_nu) {
  if (!sets || n_sets <= 0 || !two_nu) return fail(SBV_E_INVAL, "sets, n_sets and two_nu are required");
  for (int i = 0; i < n_sets; ++i) {
    if (!sets[i]) return fail(SBV_E_INVAL, "null handle in sets");
    if (two_nu[i] != 1 && two_nu[i] != 3 && two_nu[i] != 5 && two_nu[i] != 7)
      return fail(SBV_E_INVAL, "two_nu must be 1, 3, 5 or 7");
  }
  return SBV_OK;
}

// Find or build the plan for this list of sets.
sbv_status get_plan(const sbv_blocks* sets, int32_t n_sets, const int32_t* two_nu, Plan** out) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (auto& p : g_plans) {
    if ((int)p->sets.size() != n_sets) continue;
    bool same = true;
    for (int i = 0; i < n_sets && same; ++i) same = p->sets[i] == sets[i] && p->two_nu[i] == two_nu[i];
    if (same) {
      *out = p.get();
      return SBV_OK;
    }
  }
  auto P = std::make_unique<Plan>();
  P->sets.assign(sets, sets + n_sets);
  P->two_nu.assign(two_nu, two_nu + n_sets);
  std::vector<SetDesc> hd(n_sets);
  int off = 0;
  std::vector<std::vector<std::pair<int32_t, WorkItem>>> per(n_variants());
  for (int s = 0; s < n_sets; ++s) {
    sbv_blocks h = sets[s];
    SetDesc& D = hd[s];
    D.X = h->X.p;
    D.y = h->y.p;
    D.bptr = h->bptr.p;
    D.nptr = h->nptr.p;
    D.nidx = h->nidx.p;
    D.llb = h->llb.p;
    D.flag = h->flag.p;
    D.gradb = h->gradb.p;
    D.d = h->d;
    D.two_nu = two_nu[s];
    D.theta_off = off;
    D.K = (int32_t)h->K;
    P->theta_off.push_back(off);
    off += h->d + 2;
    for (int64_t b = 0; b < h->K; ++b) {
      int v = variant_for(h->joint[b]);
      if (v < 0) return fail(SBV_E_INVAL, "block joint size exceeds the supported maximum");
      per[v].push_back({h->joint[b], WorkItem{s, (int32_t)b}});
    }
  }
  P->theta_len = off;
  HIP_TRY(P->dsets.alloc(n_sets));
  HIP_TRY(hipMemcpy(P->dsets.p, hd.data(), sizeof(SetDesc) * n_sets, hipMemcpyHostToDevice));
  HIP_TRY(P->theta.alloc(off));
  HIP_TRY(P->out.alloc(n_sets));
  HIP_TRY(P->bad.alloc(n_sets));
  // longest buckets first
  for (int v = n_variants() - 1; v >= 0; --v) {
    if (per[v].empty()) continue;
    auto& L = per[v];
    std::stable_sort(L.begin(), L.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    Bucket B;
    B.variant = v;
    B.count = (int)L.size();
    std::vector<WorkItem> it(L.size());
    for (size_t i = 0; i < L.size(); ++i) it[i] = L[i].second;
    HIP_TRY(B.items.alloc(it.size()));
    HIP_TRY(hipMemcpy(B.items.p, it.data(), sizeof(WorkItem) * it.size(), hipMemcpyHostToDevice));
    HIP_TRY(B.dcount.alloc(1));
    HIP_TRY(hipMemcpy(B.dcount.p, &B.count, sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(B.fb_items.alloc(it.size()));
    HIP_TRY(B.fb_count.alloc(1));
    P->buckets.push_back(std::move(B));
  }
  *out = P.get();
  g_plans.push_back(std::move(P));
  return SBV_OK;
}

// Piv threshold of the FP32 path: a block whose FP32 pivot falls to or below
// this fraction of the original diagonal is recomputed in FP64.
double g_piv_tau = 1e-3;

// Queue one evaluation of plan P (theta already in P->theta) on stream s;
// result in P->out.
sbv_status run_plan(Plan* P, int32_t prec, hipStream_t s) {
  for (auto& B : P->buckets) {
    HIP_TRY(launch_loglik(prec == SBV_FP32 ? 1 : 0, B.variant, B.count, P->dsets.p, P->theta.p,
                          B.items.p, B.dcount.p, prec == SBV_FP32 ? g_piv_tau : 0.0, s));
    if (prec == SBV_FP32) {
      HIP_TRY(launch_zero_int(B.fb_count.p, 1, s));
      HIP_TRY(launch_flag_compact(P->dsets.p, B.items.p, B.dcount.p, B.fb_items.p, B.fb_count.p, s));
      int grid = std::min(B.count, max_grid(0, B.variant));
      HIP_TRY(launch_loglik(0, B.variant, grid, P->dsets.p, P->theta.p, B.fb_items.p, B.fb_count.p,
                            0.0, s));
    }
  }
  HIP_TRY(launch_reduce(P->dsets.p, (int)P->sets.size(), nullptr, P->out.p, P->bad.p, s));
  return SBV_OK;
}

sbv_status validate_structure(int64_t n, int32_t d, int64_t K, const int64_t* block_ptr,
                              const int64_t* block_pts, const int64_t* nn_ptr, const int64_t* nn_idx,
                              std::vector<int64_t>& rank_of_pt, std::vector<int64_t>& pos_of) {
  if (n <= 0 || d <= 0 || K <= 0 || K > n) return fail(SBV_E_INVAL, "need n > 0, d > 0 and 0 < K <= n");
  if (d > kMaxDim) return fail(SBV_E_INVAL, "d exceeds the supported maximum dimension");
  if (n > INT32_MAX - 1) return fail(SBV_E_INVAL, "n too large");
  if (!block_ptr || !block_pts || !nn_ptr || (nn_ptr[K] > 0 && !nn_idx))
    return fail(SBV_E_INVAL, "structure arrays are required");
  if (block_ptr[0] != 0 || block_ptr[K] != n) return fail(SBV_E_INVAL, "block_ptr must run from 0 to n");
  if (nn_ptr[0] != 0) return fail(SBV_E_INVAL, "nn_ptr[0] must be 0");
  rank_of_pt.assign(n, -1);
  pos_of.assign(n, -1);
  for (int64_t r = 0; r < K; ++r) {
    if (block_ptr[r + 1] <= block_ptr[r]) return fail(SBV_E_INVAL, "empty or decreasing block");
    if (nn_ptr[r + 1] < nn_ptr[r]) return fail(SBV_E_INVAL, "decreasing nn_ptr");
    for (int64_t t = block_ptr[r]; t < block_ptr[r + 1]; ++t) {
      int64_t p = block_pts[t];
      if (p < 0 || p >= n || rank_of_pt[p] >= 0) return fail(SBV_E_INVAL, "block_pts is not a permutation");
      rank_of_pt[p] = r;
      pos_of[p] = t;
    }
  }
  if (nn_ptr[K] > INT32_MAX) return fail(SBV_E_INVAL, "too many conditioning entries");
  for (int64_t r = 0; r < K; ++r)
    for (int64_t t = nn_ptr[r]; t < nn_ptr[r + 1]; ++t) {
      int64_t p = nn_idx[t];
      if (p < 0 || p >= n) return fail(SBV_E_INVAL, "neighbour id out of range");
      if (rank_of_pt[p] >= r)
        return fail(SBV_E_INVAL, "neighbour of block " + std::to_string(r) + " is not in an earlier block");
    }
  return SBV_OK;
}

}  // namespace

// Internal entry used by the builder: take ownership of an already-ordered
// structure (exchange format) and upload it.
sbv_status sbv_internal_make_handle(const double* X, const double* y, int64_t n, int32_t d, int64_t K,
                                    const int64_t* block_ptr, const int64_t* block_pts,
                                    const int64_t* nn_ptr, const int64_t* nn_idx, sbv_blocks* out);

sbv_status sbv_internal_fail(sbv_status st, const char* msg) { return fail(st, msg); }

extern "C" {

const char* sbv_last_error(void) { return g_err.c_str(); }

int32_t sbv_max_joint_size(void) { return variant(n_variants() - 1).ntm * kTile; }

sbv_status sbv_blocks_import(const double* X, const double* y, int64_t n, int32_t d, int64_t K,
                             const int64_t* block_ptr, const int64_t* block_pts, const int64_t* nn_ptr,
                             const int64_t* nn_idx, sbv_blocks* out) {
  if (!out) return fail(SBV_E_INVAL, "out is required");
  if (!X) return fail(SBV_E_INVAL, "X is required");
  return sbv_internal_make_handle(X, y, n, d, K, block_ptr, block_pts, nn_ptr, nn_idx, out);
}

sbv_status sbv_blocks_info(sbv_blocks h, int64_t* n, int32_t* d, int64_t* K, int64_t* nnz_nn) {
  if (!h) return fail(SBV_E_INVAL, "null handle");
  if (n) *n = h->n;
  if (d) *d = h->d;
  if (K) *K = h->K;
  if (nnz_nn) *nnz_nn = h->nnz;
  return SBV_OK;
}

sbv_status sbv_blocks_export(sbv_blocks h, int64_t* block_ptr, int64_t* block_pts, int64_t* nn_ptr,
                             int64_t* nn_idx) {
  if (!h) return fail(SBV_E_INVAL, "null handle");
  if (block_ptr) std::memcpy(block_ptr, h->block_ptr.data(), sizeof(int64_t) * (h->K + 1));
  if (block_pts) std::memcpy(block_pts, h->block_pts.data(), sizeof(int64_t) * h->n);
  if (nn_ptr) std::memcpy(nn_ptr, h->nn_ptr.data(), sizeof(int64_t) * (h->K + 1));
  if (nn_idx && h->nnz) std::memcpy(nn_idx, h->nn_idx.data(), sizeof(int64_t) * h->nnz);
  return SBV_OK;
}

sbv_status sbv_blocks_set_y(sbv_blocks h, const double* y) {
  if (!h || !y) return fail(SBV_E_INVAL, "handle and y are required");
  if (!finite_all(y, h->n)) return fail(SBV_E_INVAL, "y has non-finite values");
  std::vector<double> yo(h->n);
  for (int64_t t = 0; t < h->n; ++t) yo[t] = y[h->block_pts[t]];
  HIP_TRY(hipMemcpy(h->y.p, yo.data(), sizeof(double) * h->n, hipMemcpyHostToDevice));
  return SBV_OK;
}

sbv_status sbv_blocks_set_y_dev(sbv_blocks h, const double* y_dev, void* stream) {
  if (!h || !y_dev) return fail(SBV_E_INVAL, "handle and y_dev are required");
  HIP_TRY(launch_scatter_y(y_dev, h->pos_of.p, h->y.p, h->n, (hipStream_t)stream));
  return SBV_OK;
}

void sbv_blocks_free(sbv_blocks h) {
  if (!h) return;
  drop_plans_of(h);
  delete h;
}

sbv_status sbv_loglik_dev(const sbv_blocks* sets, int32_t n_sets, const double* theta_dev,
                          const int32_t* two_nu, int32_t prec, double* loglik_dev, void* stream) {
  sbv_status st = check_sets(sets, n_sets, two_nu);
  if (st) return st;
  if (!theta_dev || !loglik_dev) return fail(SBV_E_INVAL, "theta_dev and loglik_dev are required");
  if (prec != SBV_FP64 && prec != SBV_FP32) return fail(SBV_E_INVAL, "prec must be SBV_FP64 or SBV_FP32");
  Plan* P = nullptr;
  st = get_plan(sets, n_sets, two_nu, &P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(P->theta.p, theta_dev, sizeof(double) * P->theta_len, hipMemcpyDeviceToDevice, s));
  st = run_plan(P, prec, s);
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(loglik_dev, P->out.p, sizeof(double) * n_sets, hipMemcpyDeviceToDevice, s));
  for (int i = 0; i < n_sets; ++i) sets[i]->last_two_nu = two_nu[i];
  return SBV_OK;
}

sbv_status sbv_loglik(const sbv_blocks* sets, int32_t n_sets, const double* theta, const int32_t* two_nu,
                      int32_t prec, double* loglik) {
  sbv_status st = check_sets(sets, n_sets, two_nu);
  if (st) return st;
  if (!theta || !loglik) return fail(SBV_E_INVAL, "theta and loglik are required");
  if (prec != SBV_FP64 && prec != SBV_FP32) return fail(SBV_E_INVAL, "prec must be SBV_FP64 or SBV_FP32");
  Plan* P = nullptr;
  st = get_plan(sets, n_sets, two_nu, &P);
  if (st) return st;
  if (!finite_all(theta, P->theta_len)) return fail(SBV_E_INVAL, "theta has non-finite values");
  HIP_TRY(hipMemcpy(P->theta.p, theta, sizeof(double) * P->theta_len, hipMemcpyHostToDevice));
  st = run_plan(P, prec, nullptr);
  if (st) return st;
  std::vector<double> out(n_sets);
  std::vector<int> bad(n_sets);
  HIP_TRY(hipMemcpy(out.data(), P->out.p, sizeof(double) * n_sets, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(bad.data(), P->bad.p, sizeof(int) * n_sets, hipMemcpyDeviceToHost));
  std::memcpy(loglik, out.data(), sizeof(double) * n_sets);
  for (int i = 0; i < n_sets; ++i) sets[i]->last_two_nu = two_nu[i];
  for (int i = 0; i < n_sets; ++i)
    if (bad[i]) {
      // name the first failing block
      std::vector<int32_t> fl(sets[i]->K);
      HIP_TRY(hipMemcpy(fl.data(), sets[i]->flag.p, sizeof(int32_t) * sets[i]->K, hipMemcpyDeviceToHost));
      int64_t b = 0;
      while (b < sets[i]->K && !(fl[b] & 2)) ++b;
      return fail(SBV_E_NOTPD, "set " + std::to_string(i) + ": block " + std::to_string(b) +
                                   " is not positive definite in FP64");
    }
  return SBV_OK;
}

sbv_status sbv_blocks_fallback_count(sbv_blocks h, int64_t* count) {
  if (!h || !count) return fail(SBV_E_INVAL, "handle and count are required");
  HIP_TRY(hipDeviceSynchronize());
  std::vector<int32_t> fl(h->K);
  HIP_TRY(hipMemcpy(fl.data(), h->flag.p, sizeof(int32_t) * h->K, hipMemcpyDeviceToHost));
  // After a fallback pass the FP64 kernel rewrote the flag of every recomputed
  // block, so count them through the plan's fallback lists instead.
  int64_t c = 0;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto& P : g_plans) {
      auto itp = std::find(P->sets.begin(), P->sets.end(), h);
      if (itp == P->sets.end()) continue;
      int si = (int)(itp - P->sets.begin());
      for (auto& B : P->buckets) {
        int nfb = 0;
        HIP_TRY(hipMemcpy(&nfb, B.fb_count.p, sizeof(int), hipMemcpyDeviceToHost));
        if (nfb <= 0) continue;
        std::vector<WorkItem> it(nfb);
        HIP_TRY(hipMemcpy(it.data(), B.fb_items.p, sizeof(WorkItem) * nfb, hipMemcpyDeviceToHost));
        for (auto& w : it) c += (w.set == si);
      }
      break;
    }
  }
  *count = c;
  return SBV_OK;
}

sbv_status sbv_blocks_terms(sbv_blocks h, double* terms) {
  if (!h || !terms) return fail(SBV_E_INVAL, "handle and terms are required");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(terms, h->llb.p, sizeof(double) * h->K, hipMemcpyDeviceToHost));
  return SBV_OK;
}

}  // extern "C"

sbv_status sbv_internal_make_handle(const double* X, const double* y, int64_t n, int32_t d, int64_t K,
                                    const int64_t* block_ptr, const int64_t* block_pts,
                                    const int64_t* nn_ptr, const int64_t* nn_idx, sbv_blocks* out) {
  std::vector<int64_t> rank_of, pos_of;
  sbv_status st = validate_structure(n, d, K, block_ptr, block_pts, nn_ptr, nn_idx, rank_of, pos_of);
  if (st) return st;
  if (!finite_all(X, n * d)) return fail(SBV_E_INVAL, "X has non-finite values");
  if (y && !finite_all(y, n)) return fail(SBV_E_INVAL, "y has non-finite values");
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count <= 0)
    return fail(SBV_E_DEVICE, "no HIP device available");
  auto h = std::make_unique<sbv_blocks_s>();
  h->n = n;
  h->d = d;
  h->K = K;
  h->nnz = nn_ptr[K];
  h->block_ptr.assign(block_ptr, block_ptr + K + 1);
  h->block_pts.assign(block_pts, block_pts + n);
  h->nn_ptr.assign(nn_ptr, nn_ptr + K + 1);
  h->nn_idx.assign(nn_idx, nn_idx + h->nnz);
  h->joint.resize(K);
  for (int64_t r = 0; r < K; ++r) {
    int64_t j = (nn_ptr[r + 1] - nn_ptr[r]) + (block_ptr[r + 1] - block_ptr[r]);
    if (j > sbv_max_joint_size())
      return fail(SBV_E_INVAL, "block " + std::to_string(r) + " has joint size " + std::to_string(j) +
                                   " above the supported maximum");
    h->joint[r] = (int32_t)j;
    h->max_joint = std::max<int32_t>(h->max_joint, (int32_t)j);
  }
  std::vector<double> Xo((size_t)n * d), yo(n, 0.0);
  for (int64_t t = 0; t < n; ++t) {
    std::memcpy(&Xo[(size_t)t * d], X + block_pts[t] * d, sizeof(double) * d);
    if (y) yo[t] = y[block_pts[t]];
  }
  std::vector<int32_t> bp(K + 1), ni(std::max<int64_t>(h->nnz, 1), 0), po(n);
  for (int64_t r = 0; r <= K; ++r) bp[r] = (int32_t)block_ptr[r];
  for (int64_t t = 0; t < h->nnz; ++t) ni[t] = (int32_t)pos_of[nn_idx[t]];
  for (int64_t i = 0; i < n; ++i) po[i] = (int32_t)pos_of[i];
  HIP_TRY(h->X.alloc((size_t)n * d));
  HIP_TRY(h->y.alloc(n));
  HIP_TRY(h->bptr.alloc(K + 1));
  HIP_TRY(h->nptr.alloc(K + 1));
  HIP_TRY(h->nidx.alloc(ni.size()));
  HIP_TRY(h->pos_of.alloc(n));
  HIP_TRY(h->llb.alloc(K));
  HIP_TRY(h->flag.alloc(K));
  HIP_TRY(h->gradb.alloc((size_t)K * (d + 2)));
  HIP_TRY(hipMemcpy(h->X.p, Xo.data(), sizeof(double) * Xo.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->y.p, yo.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->bptr.p, bp.data(), sizeof(int32_t) * (K + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->nptr.p, nn_ptr, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->nidx.p, ni.data(), sizeof(int32_t) * ni.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->pos_of.p, po.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(h->flag.p, 0, sizeof(int32_t) * K));
  *out = h.release();
  return SBV_OK;
}
