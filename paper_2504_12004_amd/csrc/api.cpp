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
#include <cstdlib>
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
  // conditional simulator: blocks grouped by dependency level
  struct SampleLevel {
    int variant;
    int count;
    DevBuf<WorkItem> items;
    DevBuf<int> dcount;
  };
  std::vector<SampleLevel> sample_levels;
  DevBuf<double> xi_ord, theta_s;
  DevBuf<SetDesc> sample_desc;
  // build recipe of a handle made by sbv_build_blocks (for rebuilds at new ranges)
  bool built = false;
  std::vector<double> beta_build;
  int64_t k_req = 0;
  int32_t m_req = 0;
  sbv_build_opts bopts{};
  // work lists made with the handle (register variants only): bucket v's
  // items are rl_items[rl_off[v] .. rl_off[v] + rl_count[v]), longest first
  bool has_large = false;
  std::vector<int> rl_variant, rl_off, rl_count;
  DevBuf<WorkItem> rl_items;
  DevBuf<int> rl_dcount;
};

// ---- evaluation plans ------------------------------------------------------
struct Bucket {
  int variant = -1;        // smallest variant holding the bucket's joint sizes
  int tuned[2] = {-1, -1};  // autotuned variant per precision (-1: use `variant`)
  bool la[2] = {false, false};  // lookahead schedule per precision (autotuned)
  int use(int prec) const { return tuned[prec] >= 0 ? tuned[prec] : variant; }
  int count = 0;           // host copy of the item count
  DevBuf<WorkItem> items;  // sorted by joint size, longest first
  DevBuf<int> dcount;      // device copy of count
  DevBuf<WorkItem> fb_items;
  DevBuf<int> fb_count;
  // large path (joint sizes above the register capacity): items are processed
  // in windows of nb with a workspace of nb slots (L_RP panel and z_P, FP64-sized)
  bool large = false;
  int nb = 0;
  DevBuf<double> W, Z, Lpp;  // Lpp: the prefix factor, allocated with the adjoint buffers
};

// Workspace slots of the large path (each kLargeW + kLargeZ elements, about
// 0.5 MB in FP64): windows of this many blocks share one workspace.  The
// environment variable SBV_LARGE_WINDOW overrides it for new plans.
int large_window() {
  const char* e = std::getenv("SBV_LARGE_WINDOW");
  const int v = e ? std::atoi(e) : 0;
  return v > 0 ? v : 2048;
}

struct Plan {
  std::vector<sbv_blocks> sets;
  // captured evaluations: index = 2 * grad + prec
  hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec[4] = {nullptr, nullptr, nullptr, nullptr};
  ~Plan() {
    for (int i = 0; i < 4; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
    }
  }
  std::vector<SetDesc> hdesc;      // host copy of the set descriptors
  std::vector<DevBuf<double>> qbuf;  // adjoint buffers (allocated on the first gradient call)
  std::vector<DevBuf<int64_t>> qoff;
  DevBuf<double> grad;
  std::vector<int32_t> two_nu;
  std::vector<int32_t> theta_off;
  int theta_len = 0;
  DevBuf<SetDesc> dsets;
  std::vector<Bucket> buckets;
  DevBuf<double> theta, out;
  DevBuf<int> bad;
  // persistent mode: every register-path item of every set in one list
  // (buckets concatenated, longest first), served by one launch whose
  // workgroups pull items from a device counter
  int all_n = 0;
  int persist[2] = {0, 0};  // per precision: 1 when the autotuner chose the persistent launch
  DevBuf<WorkItem> all_items, all_fb_items;
  DevBuf<int> all_count, all_fb_count, queue;
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
  // one list per register variant, plus the large path last
  std::vector<std::vector<std::pair<int32_t, WorkItem>>> per(n_variants() + 1);
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
      if (v < 0) {
        const int mi = (int)(h->nn_ptr[b + 1] - h->nn_ptr[b]);
        if (large_prefix(h->joint[b], mi) < 0) return fail(SBV_E_INVAL, "block joint size not supported");
        v = n_variants();
      }
      per[v].push_back({h->joint[b], WorkItem{s, (int32_t)b}});
    }
  }
  P->theta_len = off;
  P->hdesc = hd;
  HIP_TRY(P->dsets.alloc(n_sets));
  HIP_TRY(hipMemcpy(P->dsets.p, hd.data(), sizeof(SetDesc) * n_sets, hipMemcpyHostToDevice));
  HIP_TRY(P->theta.alloc(off));
  HIP_TRY(P->out.alloc(n_sets));
  HIP_TRY(P->bad.alloc(n_sets));
  // longest buckets first
  for (int v = n_variants(); v >= 0; --v) {
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
    if (v == n_variants()) {
      B.large = true;
      B.nb = std::min(B.count, large_window());
      HIP_TRY(B.W.alloc((size_t)B.nb * kLargeW));
      HIP_TRY(B.Z.alloc((size_t)B.nb * kLargeZ));
    }
    // SBV_LOOKAHEAD=1 selects the lookahead schedule for new plans (the
    // autotuner may change it per bucket later)
    const char* la = std::getenv("SBV_LOOKAHEAD");
    B.la[0] = B.la[1] = la && la[0] == '1';
    P->buckets.push_back(std::move(B));
  }
  {
    std::vector<WorkItem> all;
    for (int v = n_variants() - 1; v >= 0; --v)
      for (const auto& e : per[v]) all.push_back(e.second);  // per[v] is sorted longest first above
    P->all_n = (int)all.size();
    if (P->all_n > 0) {
      HIP_TRY(P->all_items.alloc(all.size()));
      HIP_TRY(hipMemcpy(P->all_items.p, all.data(), sizeof(WorkItem) * all.size(), hipMemcpyHostToDevice));
      HIP_TRY(P->all_count.alloc(1));
      HIP_TRY(hipMemcpy(P->all_count.p, &P->all_n, sizeof(int), hipMemcpyHostToDevice));
      HIP_TRY(P->all_fb_items.alloc(all.size()));
      HIP_TRY(P->all_fb_count.alloc(1));
      HIP_TRY(P->queue.alloc(1));
    }
  }
  *out = P.get();
  g_plans.push_back(std::move(P));
  return SBV_OK;
}

// Kernel timing mode: when on, every bucket launch is bracketed by HIP events
// recorded on the launch stream and the elapsed times are accumulated per
// (precision, variant) when the caller asks for them.
struct TimedLaunch {
  int prec, variant;
  hipEvent_t a, b;
};
bool g_timing = false;
std::vector<TimedLaunch> g_timed;

// Pivot threshold of the FP32 path: a block whose FP32 pivot falls to or below
// this fraction of the original diagonal is recomputed in FP64.  The
// environment variable SBV_PIV_TAU overrides it (read at every queued
// evaluation; a captured graph keeps the value of its capture).
#define g_piv_tau sbv::fp32_pivot_tau()

// Allocate the per-block adjoint buffers (e, g, Q: nA_i (b_i + 2) values per
// block) of every set of a plan, once.
sbv_status ensure_adjoint(Plan* P) {
  if (!P->qbuf.empty()) return SBV_OK;
  const int ns = (int)P->sets.size();
  P->qbuf.resize(ns);
  P->qoff.resize(ns);
  for (int s = 0; s < ns; ++s) {
    sbv_blocks h = P->sets[s];
    std::vector<int64_t> off(h->K + 1, 0);
    for (int64_t b = 0; b < h->K; ++b) {
      const int64_t bi = h->block_ptr[b + 1] - h->block_ptr[b];
      off[b + 1] = off[b] + (int64_t)h->joint[b] * (bi + 2);
    }
    HIP_TRY(P->qbuf[s].alloc(off[h->K]));
    HIP_TRY(P->qoff[s].alloc(h->K + 1));
    HIP_TRY(hipMemcpy(P->qoff[s].p, off.data(), sizeof(int64_t) * (h->K + 1), hipMemcpyHostToDevice));
    P->hdesc[s].qbuf = P->qbuf[s].p;
    P->hdesc[s].qoff = P->qoff[s].p;
  }
  HIP_TRY(hipMemcpy(P->dsets.p, P->hdesc.data(), sizeof(SetDesc) * ns, hipMemcpyHostToDevice));
  HIP_TRY(P->grad.alloc(P->theta_len));
  for (auto& B : P->buckets)
    if (B.large) HIP_TRY(B.Lpp.alloc((size_t)B.nb * kLargeL));
  return SBV_OK;
}

// Queue one evaluation of log-likelihood and gradient: per bucket the
// factor + adjoint-solve kernel, then the contraction kernel; FP32 blocks that
// trip the pivot test are redone in FP64 (both kernels).
sbv_status run_plan_grad(Plan* P, int32_t prec, hipStream_t s) {
  sbv_status st = ensure_adjoint(P);
  if (st) return st;
  const int pk = prec == SBV_FP32 ? 1 : 0;
  for (auto& B : P->buckets) {
    if (B.large) {
      for (int off = 0; off < B.count; off += B.nb)
        HIP_TRY(launch_large_grad(pk, std::min(B.nb, B.count - off), P->dsets.p, P->theta.p, B.items.p,
                                  B.dcount.p, pk ? g_piv_tau : 0.0, LargeArgs{off, B.nb, B.W.p, B.Z.p, B.Lpp.p},
                                  s));
      if (pk) {
        HIP_TRY(launch_zero_int(B.fb_count.p, 1, s));
        HIP_TRY(launch_flag_compact(P->dsets.p, B.items.p, B.dcount.p, B.fb_items.p, B.fb_count.p, s));
        for (int off = 0; off < B.count; off += B.nb)
          HIP_TRY(launch_large_grad(0, std::min(B.nb, B.count - off), P->dsets.p, P->theta.p, B.fb_items.p,
                                    B.fb_count.p, 0.0, LargeArgs{off, B.nb, B.W.p, B.Z.p, B.Lpp.p}, s));
      }
      continue;
    }
    HIP_TRY(launch_loglik(pk, B.variant, B.count, P->dsets.p, P->theta.p, B.items.p, B.dcount.p,
                          pk ? g_piv_tau : 0.0, s, true));
    HIP_TRY(launch_contract(pk, B.variant, B.count, P->dsets.p, P->theta.p, B.items.p, B.dcount.p, s));
    if (pk) {
      HIP_TRY(launch_zero_int(B.fb_count.p, 1, s));
      HIP_TRY(launch_flag_compact(P->dsets.p, B.items.p, B.dcount.p, B.fb_items.p, B.fb_count.p, s));
      int grid = std::min(B.count, max_grid(0, B.variant));
      HIP_TRY(launch_loglik(0, B.variant, grid, P->dsets.p, P->theta.p, B.fb_items.p, B.fb_count.p, 0.0, s, true));
      HIP_TRY(launch_contract(0, B.variant, grid, P->dsets.p, P->theta.p, B.fb_items.p, B.fb_count.p, s));
    }
  }
  HIP_TRY(launch_reduce(P->dsets.p, (int)P->sets.size(), nullptr, P->out.p, P->bad.p, s));
  HIP_TRY(launch_reduce_grad(P->dsets.p, (int)P->sets.size(), P->grad.p, P->bad.p, s));
  return SBV_OK;
}

// Persistent mode: the register-path blocks of all sets go through ONE launch
// of the largest kernel variant any bucket uses, longest first, each
// workgroup taking its next block from a device counter; the FP32 fallback
// pass is one such launch too.  The large-set bucket keeps its own launches.
// The autotuner chooses it per plan and precision; the environment variable
// SBV_PERSISTENT (read at every queued evaluation) forces it on (1) or off (0).
bool persistent_mode(const Plan* P, int pk, int force) {
  if (force >= 0) return force == 1;
  const char* e = std::getenv("SBV_PERSISTENT");
  if (e && (e[0] == '0' || e[0] == '1')) return e[0] == '1';
  return P->persist[pk] == 1;
}

sbv_status run_persistent(Plan* P, int pk, hipStream_t s) {
  int v = -1, la = 0;
  for (const auto& B : P->buckets)
    if (!B.large && B.use(pk) > v) {
      v = B.use(pk);
      la = B.la[pk];
    }
  if (v < 0) return SBV_OK;
  const int grid = std::min(P->all_n, 1024);
  TimedLaunch tl{pk, v, nullptr, nullptr};
  if (g_timing) {
    HIP_TRY(hipEventCreate(&tl.a));
    HIP_TRY(hipEventCreate(&tl.b));
    HIP_TRY(hipEventRecord(tl.a, s));
  }
  HIP_TRY(launch_zero_int(P->queue.p, 1, s));
  HIP_TRY(launch_loglik(pk, v, grid, P->dsets.p, P->theta.p, P->all_items.p, P->all_count.p,
                        pk ? g_piv_tau : 0.0, s, false, la != 0, P->queue.p));
  if (g_timing) {
    HIP_TRY(hipEventRecord(tl.b, s));
    g_timed.push_back(tl);
  }
  if (pk) {
    HIP_TRY(launch_zero_int(P->all_fb_count.p, 1, s));
    HIP_TRY(launch_flag_compact(P->dsets.p, P->all_items.p, P->all_count.p, P->all_fb_items.p, P->all_fb_count.p, s));
    HIP_TRY(launch_zero_int(P->queue.p, 1, s));
    HIP_TRY(launch_loglik(0, v, grid, P->dsets.p, P->theta.p, P->all_fb_items.p, P->all_fb_count.p, 0.0, s,
                          false, false, P->queue.p));
  }
  return SBV_OK;
}

// Queue one evaluation of plan P (theta already in P->theta) on stream s;
// result in P->out.  force_persistent: -1 follows the plan's choice (and the
// environment), 0 / 1 forces per-bucket launches / the persistent launch.
sbv_status run_plan(Plan* P, int32_t prec, hipStream_t s, int force_persistent = -1) {
  const bool pers = persistent_mode(P, prec == SBV_FP32 ? 1 : 0, force_persistent) && P->all_n > 0;
  if (pers) {
    sbv_status st = run_persistent(P, prec == SBV_FP32 ? 1 : 0, s);
    if (st) return st;
  }
  for (auto& B : P->buckets) {
    if (pers && !B.large) continue;
    TimedLaunch tl{prec == SBV_FP32 ? 1 : 0, B.variant, nullptr, nullptr};  // keyed by size bucket
    if (g_timing) {
      HIP_TRY(hipEventCreate(&tl.a));
      HIP_TRY(hipEventCreate(&tl.b));
      HIP_TRY(hipEventRecord(tl.a, s));
    }
    const int pk = prec == SBV_FP32 ? 1 : 0;
    if (B.large) {
      for (int off = 0; off < B.count; off += B.nb)
        HIP_TRY(launch_large(pk, std::min(B.nb, B.count - off), P->dsets.p, P->theta.p, B.items.p, B.dcount.p,
                             pk ? g_piv_tau : 0.0, LargeArgs{off, B.nb, B.W.p, B.Z.p, nullptr}, s));
    } else {
      HIP_TRY(launch_loglik(pk, B.use(pk), B.count, P->dsets.p, P->theta.p, B.items.p, B.dcount.p,
                            pk ? g_piv_tau : 0.0, s, false, B.la[pk]));
    }
    if (g_timing) {
      HIP_TRY(hipEventRecord(tl.b, s));
      g_timed.push_back(tl);
    }
    if (prec == SBV_FP32) {
      HIP_TRY(launch_zero_int(B.fb_count.p, 1, s));
      HIP_TRY(launch_flag_compact(P->dsets.p, B.items.p, B.dcount.p, B.fb_items.p, B.fb_count.p, s));
      if (B.large) {
        // the flagged count is only known on the device: every window is
        // queued and windows past it exit at once
        for (int off = 0; off < B.count; off += B.nb)
          HIP_TRY(launch_large(0, std::min(B.nb, B.count - off), P->dsets.p, P->theta.p, B.fb_items.p,
                               B.fb_count.p, 0.0, LargeArgs{off, B.nb, B.W.p, B.Z.p, nullptr}, s));
      } else {
        int grid = std::min(B.count, max_grid(0, B.use(0)));
        HIP_TRY(launch_loglik(0, B.use(0), grid, P->dsets.p, P->theta.p, B.fb_items.p, B.fb_count.p, 0.0, s));
      }
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

void sbv_internal_set_build(sbv_blocks h, const double* beta_build, int64_t K, int32_t m, const sbv_build_opts& o) {
  h->built = true;
  h->beta_build.assign(beta_build, beta_build + h->d);
  h->k_req = K;
  h->m_req = m;
  h->bopts = o;
}

bool sbv_internal_was_built(sbv_blocks h) { return h && h->built; }

// Replace h's structure by a fresh build of its own points and observations
// with the same recipe at new ranges beta_build (d values).  Plans that refer
// to h are dropped; the handle pointer stays valid.
sbv_status sbv_internal_rebuild(sbv_blocks h, const double* beta_build) {
  if (!h || !h->built) return fail(SBV_E_INVAL, "the handle was not made by sbv_build_blocks");
  const int64_t n = h->n;
  const int d = h->d;
  std::vector<double> Xo((size_t)n * d), yo(n), X((size_t)n * d), y(n);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(Xo.data(), h->X.p, sizeof(double) * n * d, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(yo.data(), h->y.p, sizeof(double) * n, hipMemcpyDeviceToHost));
  for (int64_t t = 0; t < n; ++t) {
    const int64_t p = h->block_pts[t];
    std::memcpy(&X[(size_t)p * d], &Xo[(size_t)t * d], sizeof(double) * d);
    y[p] = yo[t];
  }
  sbv_blocks nh = nullptr;
  sbv_status st = sbv_build_blocks(X.data(), y.data(), n, d, beta_build, h->k_req, h->m_req, &h->bopts, &nh);
  if (st) return st;
  drop_plans_of(h);
  drop_plans_of(nh);
  std::swap(*h, *nh);
  sbv_blocks_free(nh);  // now holds the old structure
  return SBV_OK;
}

double sbv::fp32_pivot_tau() {
  const char* e = std::getenv("SBV_PIV_TAU");
  return e ? std::atof(e) : 1e-4;
}

sbv_status sbv_internal_view(sbv_blocks h, HandleView* v) {
  if (!h || !v) return fail(SBV_E_INVAL, "null handle");
  v->X = h->X.p;
  v->y = h->y.p;
  v->bptr = h->bptr.p;
  v->nptr = h->nptr.p;
  v->nidx = h->nidx.p;
  v->d = h->d;
  v->K = h->K;
  v->max_joint = h->max_joint;
  v->has_large = h->has_large;
  v->n_buckets = (int)h->rl_variant.size();
  v->bucket_variant = h->rl_variant.data();
  v->bucket_off = h->rl_off.data();
  v->bucket_count = h->rl_count.data();
  v->items = h->rl_items.p;
  v->dcount = h->rl_dcount.p;
  v->block_pts_host = h->block_pts.data();
  v->n = h->n;
  return SBV_OK;
}

extern "C" {

const char* sbv_last_error(void) { return g_err.c_str(); }

int32_t sbv_max_joint_size(void) { return kTile * (kLargeNTM + kMaxPrefix); }

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

sbv_status sbv_loglik_grad_dev(const sbv_blocks* sets, int32_t n_sets, const double* theta_dev,
                               const int32_t* two_nu, int32_t prec, double* loglik_dev, double* grad_dev,
                               void* stream) {
  sbv_status st = check_sets(sets, n_sets, two_nu);
  if (st) return st;
  if (!theta_dev || !loglik_dev || !grad_dev) return fail(SBV_E_INVAL, "theta_dev, loglik_dev and grad_dev are required");
  if (prec != SBV_FP64 && prec != SBV_FP32) return fail(SBV_E_INVAL, "prec must be SBV_FP64 or SBV_FP32");
  Plan* P = nullptr;
  st = get_plan(sets, n_sets, two_nu, &P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(P->theta.p, theta_dev, sizeof(double) * P->theta_len, hipMemcpyDeviceToDevice, s));
  st = run_plan_grad(P, prec, s);
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(loglik_dev, P->out.p, sizeof(double) * n_sets, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(grad_dev, P->grad.p, sizeof(double) * P->theta_len, hipMemcpyDeviceToDevice, s));
  return SBV_OK;
}

sbv_status sbv_loglik_grad(const sbv_blocks* sets, int32_t n_sets, const double* theta, const int32_t* two_nu,
                           int32_t prec, double* loglik, double* grad) {
  sbv_status st = check_sets(sets, n_sets, two_nu);
  if (st) return st;
  if (!theta || !loglik || !grad) return fail(SBV_E_INVAL, "theta, loglik and grad are required");
  if (prec != SBV_FP64 && prec != SBV_FP32) return fail(SBV_E_INVAL, "prec must be SBV_FP64 or SBV_FP32");
  Plan* P = nullptr;
  st = get_plan(sets, n_sets, two_nu, &P);
  if (st) return st;
  if (!finite_all(theta, P->theta_len)) return fail(SBV_E_INVAL, "theta has non-finite values");
  HIP_TRY(hipMemcpy(P->theta.p, theta, sizeof(double) * P->theta_len, hipMemcpyHostToDevice));
  st = run_plan_grad(P, prec, nullptr);
  if (st) return st;
  std::vector<double> out(n_sets), g(P->theta_len);
  std::vector<int> bad(n_sets);
  HIP_TRY(hipMemcpy(out.data(), P->out.p, sizeof(double) * n_sets, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(g.data(), P->grad.p, sizeof(double) * P->theta_len, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(bad.data(), P->bad.p, sizeof(int) * n_sets, hipMemcpyDeviceToHost));
  std::memcpy(loglik, out.data(), sizeof(double) * n_sets);
  for (int i = 0; i < n_sets; ++i) {
    const int off = P->theta_off[i], np = sets[i]->d + 2;
    for (int k = 0; k < np; ++k) grad[off + k] = bad[i] ? NAN : g[off + k];
  }
  for (int i = 0; i < n_sets; ++i)
    if (bad[i]) return fail(SBV_E_NOTPD, "set " + std::to_string(i) + " has a block that is not positive definite");
  return SBV_OK;
}

// Dependency levels of the conditional simulator: a block's level is one more
// than the highest level among the blocks holding its conditioning points, so
// every block of a level only reads observations of lower levels.
static sbv_status ensure_sampler(sbv_blocks h, int32_t two_nu) {
  if (h->max_joint > variant(n_variants() - 1).ntm * kTile)
    return fail(SBV_E_INVAL, "the conditional simulator supports joint sizes up to " +
                                 std::to_string(variant(n_variants() - 1).ntm * kTile));
  if (h->sample_levels.empty()) {
    const int64_t K = h->K;
    std::vector<int32_t> block_of(h->n);
    for (int64_t r = 0; r < K; ++r)
      for (int64_t t = h->block_ptr[r]; t < h->block_ptr[r + 1]; ++t) block_of[t] = (int32_t)r;
    std::vector<int32_t> pos_of(h->n);
    for (int64_t t = 0; t < h->n; ++t) pos_of[h->block_pts[t]] = (int32_t)t;
    std::vector<int32_t> level(K, 0);
    int32_t maxl = 0;
    for (int64_t r = 0; r < K; ++r) {
      int32_t l = 0;
      for (int64_t t = h->nn_ptr[r]; t < h->nn_ptr[r + 1]; ++t)
        l = std::max(l, level[block_of[pos_of[h->nn_idx[t]]]] + 1);
      level[r] = l;
      maxl = std::max(maxl, l);
    }
    const int nv = n_variants();
    std::vector<std::vector<WorkItem>> lists((size_t)(maxl + 1) * nv);
    for (int64_t r = 0; r < K; ++r)
      lists[(size_t)level[r] * nv + variant_for(h->joint[r])].push_back(WorkItem{0, (int32_t)r});
    for (size_t li = 0; li < lists.size(); ++li) {
      if (lists[li].empty()) continue;
      sbv_blocks_s::SampleLevel L;
      L.variant = (int)(li % nv);
      L.count = (int)lists[li].size();
      HIP_TRY(L.items.alloc(L.count));
      HIP_TRY(hipMemcpy(L.items.p, lists[li].data(), sizeof(WorkItem) * L.count, hipMemcpyHostToDevice));
      HIP_TRY(L.dcount.alloc(1));
      HIP_TRY(hipMemcpy(L.dcount.p, &L.count, sizeof(int), hipMemcpyHostToDevice));
      h->sample_levels.push_back(std::move(L));
    }
    HIP_TRY(h->xi_ord.alloc(h->n));
    HIP_TRY(h->theta_s.alloc(h->d + 2));
    HIP_TRY(h->sample_desc.alloc(1));
  }
  SetDesc D{};
  D.X = h->X.p;
  D.y = h->y.p;
  D.bptr = h->bptr.p;
  D.nptr = h->nptr.p;
  D.nidx = h->nidx.p;
  D.llb = h->llb.p;
  D.flag = h->flag.p;
  D.gradb = h->gradb.p;
  D.d = h->d;
  D.two_nu = two_nu;
  D.theta_off = 0;
  D.K = (int32_t)h->K;
  D.xi = h->xi_ord.p;
  D.y_out = h->y.p;
  HIP_TRY(hipMemcpy(h->sample_desc.p, &D, sizeof(SetDesc), hipMemcpyHostToDevice));
  return SBV_OK;
}

sbv_status sbv_sample_dev(sbv_blocks h, const double* theta_dev, int32_t two_nu, const double* xi_dev,
                          double* y_dev, void* stream) {
  if (!h || !theta_dev || !xi_dev) return fail(SBV_E_INVAL, "handle, theta_dev and xi_dev are required");
  if (two_nu != 1 && two_nu != 3 && two_nu != 5 && two_nu != 7) return fail(SBV_E_INVAL, "two_nu must be 1, 3, 5 or 7");
  sbv_status st = ensure_sampler(h, two_nu);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(h->theta_s.p, theta_dev, sizeof(double) * (h->d + 2), hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_scatter_y(xi_dev, h->pos_of.p, h->xi_ord.p, h->n, s));
  for (auto& L : h->sample_levels)
    HIP_TRY(launch_sample(L.variant, L.count, h->sample_desc.p, h->theta_s.p, L.items.p, L.dcount.p, s));
  if (y_dev) HIP_TRY(launch_gather_y(h->y.p, h->pos_of.p, y_dev, h->n, s));
  return SBV_OK;
}

sbv_status sbv_sample(sbv_blocks h, const double* theta, int32_t two_nu, const double* xi, double* y) {
  if (!h || !theta || !xi) return fail(SBV_E_INVAL, "handle, theta and xi are required");
  if (!finite_all(theta, h->d + 2) || !finite_all(xi, h->n)) return fail(SBV_E_INVAL, "non-finite theta or xi");
  DevBuf<double> th, x, yy;
  HIP_TRY(th.alloc(h->d + 2));
  HIP_TRY(x.alloc(h->n));
  HIP_TRY(yy.alloc(h->n));
  HIP_TRY(hipMemcpy(th.p, theta, sizeof(double) * (h->d + 2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(x.p, xi, sizeof(double) * h->n, hipMemcpyHostToDevice));
  sbv_status st = sbv_sample_dev(h, th.p, two_nu, x.p, yy.p, nullptr);
  if (st) return st;
  if (y) HIP_TRY(hipMemcpy(y, yy.p, sizeof(double) * h->n, hipMemcpyDeviceToHost));
  HIP_TRY(hipDeviceSynchronize());
  return SBV_OK;
}

// ---- autotuner: per size bucket, time every kernel variant that can hold the
// bucket's largest joint size and keep the fastest.
sbv_status sbv_autotune(const sbv_blocks* sets, int32_t n_sets, const int32_t* two_nu, const double* theta,
                        int32_t prec, int32_t reps, int32_t* chosen_tiles, int32_t* chosen_lookahead,
                        int32_t* chosen_waves, int32_t* chosen_persistent) {
  sbv_status st = check_sets(sets, n_sets, two_nu);
  if (st) return st;
  if (!theta || reps <= 0) return fail(SBV_E_INVAL, "theta and reps > 0 are required");
  Plan* P = nullptr;
  st = get_plan(sets, n_sets, two_nu, &P);
  if (st) return st;
  HIP_TRY(hipMemcpy(P->theta.p, theta, sizeof(double) * P->theta_len, hipMemcpyHostToDevice));
  const int pk = prec == SBV_FP32 ? 1 : 0;
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  int bi = 0;
  for (auto& B : P->buckets) {
    if (B.large) {  // one kernel pair, nothing to choose
      if (chosen_tiles) chosen_tiles[bi] = kLargeNTM + kMaxPrefix;
      if (chosen_lookahead) chosen_lookahead[bi] = 0;
      if (chosen_waves) chosen_waves[bi] = 8;
      ++bi;
      continue;
    }
    // the bucket's own variant is the smallest that fits; candidates are it and all larger ones
    const int base = B.variant;
    float best = INFINITY;
    int bestv = base;
    bool bestla = false;
    for (int v = base; v < n_variants(); ++v)
      for (int la = 0; la < 2; ++la) {
        HIP_TRY(launch_loglik(pk, v, B.count, P->dsets.p, P->theta.p, B.items.p, B.dcount.p, 0.0, nullptr, false,
                              la != 0));
        HIP_TRY(hipEventRecord(a, nullptr));
        for (int r = 0; r < reps; ++r)
          HIP_TRY(launch_loglik(pk, v, B.count, P->dsets.p, P->theta.p, B.items.p, B.dcount.p, 0.0, nullptr,
                                false, la != 0));
        HIP_TRY(hipEventRecord(b, nullptr));
        HIP_TRY(hipEventSynchronize(b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, a, b));
        if (ms < best) {
          best = ms;
          bestv = v;
          bestla = la != 0;
        }
      }
    B.tuned[pk] = bestv;
    B.la[pk] = bestla;
    if (chosen_tiles) chosen_tiles[bi] = variant(bestv).ntm;
    if (chosen_lookahead) chosen_lookahead[bi] = bestla ? 1 : 0;
    // waves per compute unit: waves per workgroup times workgroups per unit
    // (FP64 requests for the 16-wave and occupancy-2 variants run the 8-wave kernel)
    if (chosen_waves)
      chosen_waves[bi] = pk == 0 ? std::min(variant(bestv).nw, 8) : variant(bestv).nw * std::max(variant(bestv).occ, 1);
    ++bi;
  }
  // whole evaluations: per-bucket launches against the persistent launch
  if (P->all_n > 0) {
    float best_t = INFINITY;
    int best_p = 0;
    for (int pm = 0; pm < 2; ++pm) {
      sbv_status rs = run_plan(P, prec, nullptr, pm);
      if (rs) return rs;
      HIP_TRY(hipEventRecord(a, nullptr));
      for (int r = 0; r < reps; ++r) {
        rs = run_plan(P, prec, nullptr, pm);
        if (rs) return rs;
      }
      HIP_TRY(hipEventRecord(b, nullptr));
      HIP_TRY(hipEventSynchronize(b));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, a, b));
      if (ms < best_t) {
        best_t = ms;
        best_p = pm;
      }
    }
    P->persist[pk] = best_p;
  }
  if (chosen_persistent) *chosen_persistent = P->persist[pk];
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  // captured graphs may hold the old choice
  for (int i = 0; i < 4; ++i) {
    if (P->exec[i]) (void)hipGraphExecDestroy(P->exec[i]);
    if (P->graph[i]) (void)hipGraphDestroy(P->graph[i]);
    P->exec[i] = nullptr;
    P->graph[i] = nullptr;
  }
  return SBV_OK;
}

// ---- graph-captured evaluation of a whole plan ------------------------------
// The kernels of one evaluation (every bucket of every set, the FP32 fallback
// pass and the reductions) are captured once into a hipGraph; theta enters
// through the plan's fixed device buffer and results leave through the plan's
// output buffers, so the graph's parameters never change.
sbv_status sbv_eval_graph_dev(const sbv_blocks* sets, int32_t n_sets, const double* theta_dev,
                              const int32_t* two_nu, int32_t prec, int32_t with_grad, double* loglik_dev,
                              double* grad_dev, void* stream) {
  sbv_status st = check_sets(sets, n_sets, two_nu);
  if (st) return st;
  if (!theta_dev || !loglik_dev || (with_grad && !grad_dev)) return fail(SBV_E_INVAL, "device buffers required");
  if (prec != SBV_FP64 && prec != SBV_FP32) return fail(SBV_E_INVAL, "prec must be SBV_FP64 or SBV_FP32");
  Plan* P = nullptr;
  st = get_plan(sets, n_sets, two_nu, &P);
  if (st) return st;
  if (with_grad) {
    st = ensure_adjoint(P);
    if (st) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  const int gi = 2 * (with_grad ? 1 : 0) + (prec == SBV_FP32 ? 1 : 0);
  if (!P->exec[gi]) {
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    sbv_status rs = with_grad ? run_plan_grad(P, prec, cs) : run_plan(P, prec, cs);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rs) return rs;
    if (ce != hipSuccess) return fail(SBV_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(ce));
    P->graph[gi] = g;
    HIP_TRY(hipGraphInstantiate(&P->exec[gi], g, nullptr, nullptr, 0));
  }
  HIP_TRY(hipMemcpyAsync(P->theta.p, theta_dev, sizeof(double) * P->theta_len, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipGraphLaunch(P->exec[gi], s));
  HIP_TRY(hipMemcpyAsync(loglik_dev, P->out.p, sizeof(double) * n_sets, hipMemcpyDeviceToDevice, s));
  if (with_grad)
    HIP_TRY(hipMemcpyAsync(grad_dev, P->grad.p, sizeof(double) * P->theta_len, hipMemcpyDeviceToDevice, s));
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

sbv_status sbv_timing_enable(int32_t on) {
  for (auto& t : g_timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  g_timed.clear();
  g_timing = on != 0;
  return SBV_OK;
}

sbv_status sbv_timing_read(int32_t prec, int32_t* n_variants_out, double* ms_total, int64_t* launches) {
  HIP_TRY(hipDeviceSynchronize());
  const int nv = n_variants() + 1;  // size buckets: register variants, then the large path
  if (n_variants_out) *n_variants_out = nv;
  for (int v = 0; v < nv; ++v) {
    if (ms_total) ms_total[v] = 0.0;
    if (launches) launches[v] = 0;
  }
  for (auto& t : g_timed) {
    if (t.prec != (prec == SBV_FP32 ? 1 : 0)) continue;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    if (ms_total) ms_total[t.variant] += ms;
    if (launches) launches[t.variant] += 1;
  }
  return SBV_OK;
}

sbv_status sbv_plan_flops(const sbv_blocks* sets, int32_t n_sets, const int32_t* two_nu, double* flops,
                          int32_t* variant_of_bucket, int32_t* n_buckets) {
  sbv_status st = check_sets(sets, n_sets, two_nu);
  if (st) return st;
  Plan* P = nullptr;
  st = get_plan(sets, n_sets, two_nu, &P);
  if (st) return st;
  const int nv = n_variants();  // register variants; bucket nv is the large path
  for (int v = 0; v <= nv; ++v) flops[v] = 0.0;
  for (int s = 0; s < n_sets; ++s)
    for (int64_t b = 0; b < sets[s]->K; ++b) {
      const double nA = sets[s]->joint[b];
      const int v = variant_for(sets[s]->joint[b]);
      flops[v < 0 ? nv : v] += nA * nA * nA / 3.0 + nA * nA;
    }
  if (n_buckets) *n_buckets = nv + 1;
  if (variant_of_bucket) {
    for (int v = 0; v < nv; ++v) variant_of_bucket[v] = variant(v).ntm;
    variant_of_bucket[nv] = kLargeNTM + kMaxPrefix;
    for (const auto& B : P->buckets)
      if (!B.large) variant_of_bucket[B.variant] = variant(B.use(0)).ntm;
  }
  return SBV_OK;
}

sbv_status sbv_cov_matrix_dev(const double* Xa_dev, int64_t na, const double* Xb_dev, int64_t nb, int32_t d,
                              const double* theta_dev, int32_t two_nu, int32_t same, double* out_dev, void* stream) {
  if (!Xa_dev || !Xb_dev || !theta_dev || !out_dev || na <= 0 || nb <= 0 || d <= 0)
    return fail(SBV_E_INVAL, "device buffers and positive sizes are required");
  if (two_nu != 1 && two_nu != 3 && two_nu != 5 && two_nu != 7) return fail(SBV_E_INVAL, "two_nu must be 1, 3, 5 or 7");
  if (same && na != nb) return fail(SBV_E_INVAL, "same = 1 needs na == nb");
  HIP_TRY(launch_cov_matrix(Xa_dev, na, Xb_dev, nb, d, theta_dev, two_nu, same, out_dev, (hipStream_t)stream));
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
    const int64_t mi = nn_ptr[r + 1] - nn_ptr[r];
    int64_t j = mi + (block_ptr[r + 1] - block_ptr[r]);
    if (j > sbv_max_joint_size())
      return fail(SBV_E_INVAL, "block " + std::to_string(r) + " has joint size " + std::to_string(j) +
                                   " above the supported maximum");
    if (variant_for((int)j) < 0 && large_prefix((int)j, (int)mi) < 0)
      return fail(SBV_E_INVAL, "block " + std::to_string(r) + " has joint size " + std::to_string(j) +
                                   " but only " + std::to_string(mi) +
                                   " conditioning points; above 272 the first 16 * (ceil(size / 16) - 17) "
                                   "joint points must be conditioning points");
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
  // resident work lists: one bucket per register variant, longest first
  {
    const int nv = n_variants();
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per(nv);
    for (int64_t r = 0; r < K; ++r) {
      const int v = variant_for(h->joint[r]);
      if (v < 0)
        h->has_large = true;
      else
        per[v].push_back({h->joint[r], (int32_t)r});
    }
    std::vector<WorkItem> it;
    std::vector<int> cnt;
    for (int v = nv - 1; v >= 0; --v) {
      if (per[v].empty()) continue;
      std::stable_sort(per[v].begin(), per[v].end(), [](const auto& a, const auto& b) { return a.first > b.first; });
      h->rl_variant.push_back(v);
      h->rl_off.push_back((int)it.size());
      h->rl_count.push_back((int)per[v].size());
      for (const auto& e : per[v]) it.push_back(WorkItem{0, e.second});
    }
    if (!it.empty()) {
      HIP_TRY(h->rl_items.alloc(it.size()));
      HIP_TRY(hipMemcpy(h->rl_items.p, it.data(), sizeof(WorkItem) * it.size(), hipMemcpyHostToDevice));
      HIP_TRY(h->rl_dcount.alloc(h->rl_count.size()));
      HIP_TRY(hipMemcpy(h->rl_dcount.p, h->rl_count.data(), sizeof(int) * h->rl_count.size(),
                        hipMemcpyHostToDevice));
    }
  }
  *out = h.release();
  return SBV_OK;
}
