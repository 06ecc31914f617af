// Internal types shared by the HIP kernels and the C-ABI layer of libsbv.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace sbv {

// Tile edge of every block factorisation (the 16x16 MFMA output tile).
constexpr int kTile = 16;
// Largest input dimension supported by the fused kernels.
constexpr int kMaxDim = 20;

// One dataset as the kernels see it: points in block-rank order.
struct SetDesc {
  const double* X;        // n x d, row-major, rank order
  const double* y;        // n, rank order
  const int32_t* bptr;    // K+1 block offsets into the ordered points
  const int64_t* nptr;    // K+1 offsets into nidx
  const int32_t* nidx;    // conditioning points as ordered positions
  double* llb;            // K per-block terms (output)
  int32_t* flag;          // K per-block status (output): bit0 fp32 pivot flag, bit1 not PD
  double* gradb;          // K x (d+2) per-block gradient terms (output, gradient kernels)
  double* qbuf;           // adjoint buffer: per block e, g, Q (elements of the kernel precision)
  const int64_t* qoff;    // K offsets into qbuf, in elements of the kernel precision
  const double* xi;       // n innovations, rank order (conditional simulation only; null: all 0)
  double* y_out;          // simulated observations, rank order (conditional simulation only)
  double* var_out;        // conditional variances of the block points (prediction only; may be null)
  int32_t d;
  int32_t two_nu;
  int32_t theta_off;      // offset of this set's d+2 parameters in the theta buffer
  int32_t K;
  int32_t out_off;        // xi, y_out and var_out are indexed by (ordered position - out_off)
};

// One unit of work: block `block` of set `set`.
struct WorkItem {
  int32_t set;
  int32_t block;
};

// Kernel variant: register-tile capacity NTM tiles per side, NW waves, and
// occ workgroups meant to share a compute unit (registers capped to fit).
struct Variant {
  int ntm;
  int nw;
  int occ = 1;
};

// Blocks whose joint size exceeds the register capacity of the largest
// variant (kLargeNTM tiles) take the two-kernel path: the first
// p = ceil(nA/16) - kLargeNTM tile rows (conditioning points, 16p <= m_i) are
// eliminated by the prefix kernel, which writes the panel of L below them and
// their part of z to a workspace; the trailing kLargeNTM tiles are then
// factored by the register kernel after p streamed rank-16 updates.
constexpr int kLargeNTM = 17;
// Elements of one 16x16 tile in the MFMA operand layout (the three padding
// elements per 16-row group keep the layout change of the column solves free
// of LDS bank conflicts).
constexpr int kOpT = 272;
constexpr int kMaxPrefix = 15;  // joint sizes up to 16 * (kLargeNTM + kMaxPrefix) = 512
constexpr int64_t kLargeW = (int64_t)kMaxPrefix * kLargeNTM * kOpT;  // panel elements per workspace slot
constexpr int64_t kLargeZ = (int64_t)kMaxPrefix * kTile;            // z elements per workspace slot
constexpr int64_t kLargeL = (int64_t)kMaxPrefix * kMaxPrefix * kOpT;  // L_PP elements per slot (gradient)

// Workspace window of one launch of the large-block kernels: they process
// items[off + i] for i < min(*count - off, nb), item i using workspace slot i
// (W + i * kLargeW, z + i * kLargeZ, Lpp + i * kLargeL, elements of the kernel
// precision).  Lpp (the prefix factor, kept for the adjoint) may be null on
// the forward path.
struct LargeArgs {
  int32_t off;
  int32_t nb;
  void* W;
  void* z;
  void* Lpp;
  // Register kernels only: when set, workgroups take their items from this
  // device counter (one atomic increment per item, starting at 0) instead of
  // striding by the grid size -- one persistent launch can then serve every
  // item of a list whatever the number of resident workgroups.
  int* queue;
};

// Prefix length p of a block with joint size nA and m_i conditioning points
// on the large path, or -1 when it does not qualify (fits a register variant,
// exceeds 512, or the prefix would reach into the block's own points).
inline int large_prefix(int nA, int mi) {
  const int nt = (nA + kTile - 1) / kTile;
  const int p = nt - kLargeNTM;
  if (p < 1 || p > kMaxPrefix || kTile * p > mi) return -1;
  return p;
}

// Launchers (kernels.hip).  `count` is a device int; the kernel loops over
// items[blockIdx.x + k*gridDim.x] while the index is below *count.
hipError_t launch_loglik(int prec, int variant, int grid, const SetDesc* sets, const double* theta,
                         const WorkItem* items, const int* count, double piv_tau, hipStream_t s,
                         bool grad = false, bool lookahead = false, int* queue = nullptr);
hipError_t launch_contract(int prec, int variant, int grid, const SetDesc* sets, const double* theta,
                           const WorkItem* items, const int* count, hipStream_t s);
hipError_t launch_sample(int variant, int grid, const SetDesc* sets, const double* theta,
                         const WorkItem* items, const int* count, hipStream_t s);
// bad (n_sets, may be null): the not-positive-definite flags written by
// launch_reduce; a flagged set's gradient is NaN.
hipError_t launch_reduce_grad(const SetDesc* sets, int n_sets, double* out, const int* bad, hipStream_t s);
int n_variants();
Variant variant(int v);
int variant_for(int nA);  // smallest variant holding a joint size nA, or -1
hipError_t launch_reduce(const SetDesc* sets, int n_sets, const int* set_k, double* out, int* bad,
                         hipStream_t s);
hipError_t launch_flag_compact(const SetDesc* sets, const WorkItem* items, const int* count,
                               WorkItem* out_items, int* out_count, hipStream_t s);
hipError_t launch_zero_int(int* p, int n, hipStream_t s);
int max_grid(int prec, int variant);
// Both kernels of the large path for one workspace window (prec 0 FP64, 1 FP32).
hipError_t launch_large(int prec, int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                        const int* count, double piv_tau, const LargeArgs& L, hipStream_t s);
// Large path with the gradient: prefix kernel (keeping L_PP), trailing factor
// with its adjoint solves, the prefix part of the adjoint, and the streamed
// contraction; per-block gradients land in gradb.  L.Lpp must be set.
hipError_t launch_large_grad(int prec, int grid, const SetDesc* sets, const double* theta, const WorkItem* items,
                             const int* count, double piv_tau, const LargeArgs& L, hipStream_t s);

}  // namespace sbv

namespace sbv {

// Read-only view of a handle for entry points outside the evaluation plans:
// its device arrays and the work lists made when the handle was created (one
// size bucket per register variant, longest joint size first, items of set 0,
// all in one device array with one device count per bucket).
struct HandleView {
  const double* X;
  const double* y;
  const int32_t* bptr;
  const int64_t* nptr;
  const int32_t* nidx;
  int32_t d;
  int64_t K;
  int32_t max_joint;
  bool has_large;                 // some block needs the large-joint-set path
  int n_buckets;
  const int* bucket_variant;      // host, n_buckets
  const int* bucket_off;          // host, n_buckets: offset into items
  const int* bucket_count;        // host, n_buckets
  const WorkItem* items;          // device, K items grouped by bucket
  const int* dcount;              // device, n_buckets counts
  const int64_t* block_pts_host;  // host, n: original id of each ordered position
  int64_t n;
};

// Neighbour search of the builder (build_kernels.hip): brute force over the
// points of earlier blocks for queries 0..K-1 or the ascending ranks in qlist,
// and the two steps of the filtered search (coarse candidate blocks, fine
// candidate points with its exactness status).
hipError_t launch_knn(const double* Z, int d, const double* cen, const int32_t* bptr, int K, int m,
                      const int64_t* nn_ptr, int32_t* nn_pos, hipStream_t s, const int32_t* qlist = nullptr,
                      int nq = 0);
hipError_t launch_knn_coarse(const double* cen, const double* rad, int d, const int32_t* qlist, int nq,
                             const double* lam, int cap, int32_t* cand, int32_t* ccount, hipStream_t s);
hipError_t launch_knn_fine(const double* Z, int d, const double* cen, const int32_t* bptr, const int32_t* qlist,
                           int nq, const double* lam, int cap, const int32_t* cand, const int32_t* ccount,
                           const int64_t* nn_ptr, int32_t* nn_pos, int32_t* status, hipStream_t s);
int knn_max_m();

// Dense covariance matrix between two point lists (device buffers; theta on
// the device, d + 2 log-parameters).
hipError_t launch_cov_matrix(const double* Xa, int64_t na, const double* Xb, int64_t nb, int d, const double* theta,
                             int two_nu, int same, double* out, hipStream_t s);

// Pivot threshold of the FP32 path (a block whose FP32 pivot falls to or
// below this fraction of its original diagonal is recomputed in FP64).
double fp32_pivot_tau();

// Summaries of n_draws draws mean_j + sqrt(var_j) xi[t * n + j] per point j:
// stats[j] sample mean, stats[n + j] sample variance (divisor n_draws - 1),
// stats[2n + j] / stats[3n + j] the 95 % interval mean -/+ z sd.
hipError_t launch_pred_draws(const double* mean, const double* var, int64_t n, const double* xi, int n_draws,
                             double* stats, hipStream_t s);

hipError_t launch_gather_y(const double* y_ord, const int32_t* pos_of, double* y, int64_t n, hipStream_t s);
hipError_t launch_scatter_y(const double* y, const int32_t* pos_of, double* y_ord, int64_t n,
                            hipStream_t s);
}  // namespace sbv
