// Log-likelihood entry point that allocates no device memory.
//
// sbv_loglik_noalloc_dev evaluates one handle with the same kernels, size
// buckets and reduction as sbv_loglik_dev, but keeps everything the
// evaluation needs beyond its inputs and output -- the set descriptor, the
// per-block terms and flags, the FP32 fallback lists and their counters, the
// reduction's failure flag -- in one file-scope device array, `scratch`.  The
// work lists come from the handle (made when it was created).  No hipMalloc,
// hipFree or allocating library call is made, so the call suits callers that
// cannot allocate (code queued inside a capture region, tight serving loops).
//
// Each device holds its own copy of the array until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for the
// current device (kept per device at the first call), never through the
// array's name.  Calls that overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/sbv.h"
#include "sbv_internal.h"

sbv_status sbv_internal_fail(sbv_status st, const char* msg);
sbv_status sbv_internal_view(sbv_blocks h, sbv::HandleView* v);

namespace {

using sbv::SetDesc;
using sbv::WorkItem;

// Largest block count one call accepts.
constexpr int64_t kMaxBlocks = int64_t(1) << 18;
constexpr int kMaxBuckets = 32;

// Byte layout of the scratch array.
constexpr size_t kOffDesc = 0;                                      // SetDesc
constexpr size_t kOffBad = 256;                                     // int: not-PD flag of the reduction
constexpr size_t kOffFbCount = 512;                                 // int[kMaxBuckets]: fallback counts
constexpr size_t kOffLlb = 1024;                                    // double[kMaxBlocks]: block terms
constexpr size_t kOffFlag = kOffLlb + sizeof(double) * kMaxBlocks;  // int32[kMaxBlocks]: block flags
constexpr size_t kOffFb = kOffFlag + sizeof(int32_t) * kMaxBlocks;  // WorkItem[kMaxBlocks]: fallback list
constexpr size_t kScratchBytes = kOffFb + sizeof(WorkItem) * kMaxBlocks;
static_assert(sizeof(SetDesc) <= kOffBad, "set descriptor does not fit its scratch slot");
static_assert(sizeof(int) * kMaxBuckets <= kOffLlb - kOffFbCount, "fallback counters do not fit");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
sbv_status scratch_ptr(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return sbv_internal_fail(SBV_E_DEVICE, "no current HIP device for the allocation-free evaluation");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return sbv_internal_fail(SBV_E_DEVICE, (std::string("hipGetSymbolAddress(scratch) failed: ") +
                                              hipGetErrorString(e)).c_str());
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return SBV_OK;
}

__global__ void k_put_desc(SetDesc* dst, SetDesc v) { *dst = v; }

}  // namespace

#define NA_TRY(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return sbv_internal_fail(SBV_E_DEVICE, (std::string("HIP error in ") + #expr + ": " + \
                                              hipGetErrorString(e_)).c_str());               \
  } while (0)

extern "C" sbv_status sbv_loglik_noalloc_dev(sbv_blocks h, const double* theta_dev, int32_t two_nu, int32_t prec,
                                             double* loglik_dev, void* stream) {
  if (!h || !theta_dev || !loglik_dev)
    return sbv_internal_fail(SBV_E_INVAL, "handle, theta_dev and loglik_dev are required");
  if (two_nu != 1 && two_nu != 3 && two_nu != 5 && two_nu != 7)
    return sbv_internal_fail(SBV_E_INVAL, "two_nu must be 1, 3, 5 or 7");
  if (prec != SBV_FP64 && prec != SBV_FP32) return sbv_internal_fail(SBV_E_INVAL, "prec must be SBV_FP64 or SBV_FP32");
  sbv::HandleView v{};
  sbv_status st = sbv_internal_view(h, &v);
  if (st) return st;
  if (v.K > kMaxBlocks)
    return sbv_internal_fail(SBV_E_INVAL, ("the allocation-free evaluation takes at most " +
                                           std::to_string(kMaxBlocks) + " blocks; this handle has " +
                                           std::to_string(v.K)).c_str());
  if (v.has_large)
    return sbv_internal_fail(SBV_E_INVAL, ("the allocation-free evaluation takes joint sizes up to " +
                                           std::to_string(sbv::variant(sbv::n_variants() - 1).ntm * sbv::kTile) +
                                           "; this handle has " + std::to_string(v.max_joint)).c_str());
  if (v.n_buckets > kMaxBuckets) return sbv_internal_fail(SBV_E_INVAL, "too many size buckets");
  unsigned char* base = nullptr;
  st = scratch_ptr(&base);
  if (st) return st;
  SetDesc* desc = reinterpret_cast<SetDesc*>(base + kOffDesc);
  int* bad = reinterpret_cast<int*>(base + kOffBad);
  int* fb_count = reinterpret_cast<int*>(base + kOffFbCount);
  WorkItem* fb_items = reinterpret_cast<WorkItem*>(base + kOffFb);

  SetDesc D{};
  D.X = v.X;
  D.y = v.y;
  D.bptr = v.bptr;
  D.nptr = v.nptr;
  D.nidx = v.nidx;
  D.llb = reinterpret_cast<double*>(base + kOffLlb);
  D.flag = reinterpret_cast<int32_t*>(base + kOffFlag);
  D.d = v.d;
  D.two_nu = two_nu;
  D.theta_off = 0;
  D.K = (int32_t)v.K;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(1), 0, s, desc, D);
  NA_TRY(hipGetLastError());
  const int pk = prec == SBV_FP32 ? 1 : 0;
  const double tau = pk ? sbv::fp32_pivot_tau() : 0.0;
  for (int b = 0; b < v.n_buckets; ++b) {
    const int var = v.bucket_variant[b];
    const WorkItem* items = v.items + v.bucket_off[b];
    NA_TRY(sbv::launch_loglik(pk, var, v.bucket_count[b], desc, theta_dev, items, v.dcount + b, tau, s));
    if (pk) {
      NA_TRY(sbv::launch_zero_int(fb_count + b, 1, s));
      NA_TRY(sbv::launch_flag_compact(desc, items, v.dcount + b, fb_items, fb_count + b, s));
      const int grid = std::min(v.bucket_count[b], sbv::max_grid(0, var));
      NA_TRY(sbv::launch_loglik(0, var, grid, desc, theta_dev, fb_items, fb_count + b, 0.0, s));
    }
  }
  NA_TRY(sbv::launch_reduce(desc, 1, nullptr, loglik_dev, bad, s));
  return SBV_OK;
}
