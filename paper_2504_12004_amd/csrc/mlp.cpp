// Warm-start network: a fully connected in -> H (x L, GELU) -> out FP32 MLP
// trained on the device with the hand-written kernels of mlp_kernels.hip, and
// the per-dataset summary statistics it reads.
//
// Parameters are packed layer by layer as W (rows = outputs, row-major) then
// b.  Inputs and targets are standardised with the training set's column
// means and standard deviations, stored in the handle and applied by predict.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/sbv.h"
#include "sbv_internal.h"

sbv_status sbv_internal_fail(sbv_status st, const char* msg);

namespace sbv {
hipError_t launch_gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                       int64_t sbn, float* C, int64_t ldc, const float* bias, float* D, int mode, float beta,
                       hipStream_t s);
hipError_t launch_gelu_bwd(const float* Z, const float* dA, float* dZ, int64_t n, hipStream_t s);
hipError_t launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s);
hipError_t launch_mse(const float* yhat, const float* y, int64_t n, float* dy, float* loss, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t s);
hipError_t launch_affine_cols(const float* x, int64_t rows, int cols, const float* mu, const float* sd, float* y,
                              int inverse, hipStream_t s);
hipError_t launch_gather_rows(const float* in, const int32_t* idx, int rows, int cols, float* out, hipStream_t s);
hipError_t launch_knn16(const double* P, int ns, int d, int32_t* nn, hipStream_t s);
}  // namespace sbv

using namespace sbv;

#define MTRY(expr)                                                                                  \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess)                                                                           \
      return sbv_internal_fail(e_ == hipErrorOutOfMemory ? SBV_E_NOMEM : SBV_E_DEVICE,              \
                               (std::string("HIP error in mlp: ") + hipGetErrorString(e_)).c_str()); \
  } while (0)

namespace {

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t c) {
    if (c <= n && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = c;
    return hipMalloc((void**)&p, sizeof(T) * std::max<size_t>(c, 1));
  }
};

struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  // Box-Muller
  double normal() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(6.283185307179586 * uniform()); }
  uint64_t below(uint64_t n) { return (uint64_t)(((unsigned __int128)next() * n) >> 64); }
};

}  // namespace

struct sbv_mlp_s {
  int in = 0, H = 0, L = 0, out = 0;
  int64_t np = 0;
  std::vector<int64_t> off;  // offset of each layer's W (L + 1 layers)
  DBuf<float> p, g, m, v;
  std::vector<float> mu_x, sd_x, mu_y, sd_y;
  DBuf<float> dmu_x, dsd_x, dmu_y, dsd_y;
  int64_t adam_t = 0;
  // work buffers for a batch of B rows
  int B = 0;
  DBuf<float> X0, Z, A, dA, dZ, Yh, dY, Yt, loss;
  hipError_t work(int b) {
    if (b <= B) return hipSuccess;
    B = b;
    hipError_t e;
    if ((e = X0.alloc((size_t)b * in))) return e;
    if ((e = Z.alloc((size_t)b * H * L))) return e;
    if ((e = A.alloc((size_t)b * H * L))) return e;
    if ((e = dA.alloc((size_t)b * std::max(H, in)))) return e;
    if ((e = dZ.alloc((size_t)b * H))) return e;
    if ((e = Yh.alloc((size_t)b * out))) return e;
    if ((e = dY.alloc((size_t)b * out))) return e;
    if ((e = Yt.alloc((size_t)b * out))) return e;
    return loss.alloc(1);
  }
  int din(int l) const { return l == 0 ? in : H; }
};

namespace {

// Forward on b standardised rows in M->X0; output (standardised) in M->Yh.
hipError_t forward(sbv_mlp_s* M, int b, hipStream_t s) {
  const float* x = M->X0.p;
  for (int l = 0; l < M->L; ++l) {
    const int di = M->din(l);
    const float* W = M->p.p + M->off[l];
    const float* bias = W + (int64_t)M->H * di;
    float* Z = M->Z.p + (int64_t)l * b * M->H;
    float* Aout = M->A.p + (int64_t)l * b * M->H;
    hipError_t e = launch_gemm(b, M->H, di, x, di, 1, W, 1, di, Z, M->H, bias, Aout, 1, 0.f, s);
    if (e) return e;
    x = Aout;
  }
  const int dl = M->din(M->L);
  const float* W = M->p.p + M->off[M->L];
  return launch_gemm(b, M->out, dl, x, dl, 1, W, 1, dl, M->Yh.p, M->out, W + (int64_t)M->out * dl, nullptr, 2, 0.f,
                     s);
}

// Backward from dY (b x out) into M->g (overwritten).
hipError_t backward(sbv_mlp_s* M, int b, hipStream_t s) {
  hipError_t e;
  const int L = M->L, H = M->H;
  const int dl = M->din(L);
  const float* hin = L > 0 ? M->A.p + (int64_t)(L - 1) * b * H : M->X0.p;
  float* gWo = M->g.p + M->off[L];
  const float* Wo = M->p.p + M->off[L];
  if ((e = launch_gemm(M->out, dl, b, M->dY.p, 1, M->out, hin, dl, 1, gWo, dl, nullptr, nullptr, 0, 0.f, s))) return e;
  if ((e = launch_colsum(M->dY.p, b, M->out, gWo + (int64_t)M->out * dl, s))) return e;
  if (L == 0) return hipSuccess;
  if ((e = launch_gemm(b, dl, M->out, M->dY.p, M->out, 1, Wo, dl, 1, M->dA.p, dl, nullptr, nullptr, 0, 0.f, s)))
    return e;
  for (int l = L - 1; l >= 0; --l) {
    const int di = M->din(l);
    const float* Z = M->Z.p + (int64_t)l * b * H;
    if ((e = launch_gelu_bwd(Z, M->dA.p, M->dZ.p, (int64_t)b * H, s))) return e;
    const float* xin = l > 0 ? M->A.p + (int64_t)(l - 1) * b * H : M->X0.p;
    float* gW = M->g.p + M->off[l];
    if ((e = launch_gemm(H, di, b, M->dZ.p, 1, H, xin, di, 1, gW, di, nullptr, nullptr, 0, 0.f, s))) return e;
    if ((e = launch_colsum(M->dZ.p, b, H, gW + (int64_t)H * di, s))) return e;
    if (l > 0) {
      const float* W = M->p.p + M->off[l];
      if ((e = launch_gemm(b, di, H, M->dZ.p, H, 1, W, di, 1, M->dA.p, di, nullptr, nullptr, 0, 0.f, s))) return e;
    }
  }
  return hipSuccess;
}

void col_stats(const float* X, int64_t n, int c, std::vector<float>& mu, std::vector<float>& sd) {
  mu.assign(c, 0.f);
  sd.assign(c, 1.f);
  for (int k = 0; k < c; ++k) {
    double s = 0.0, q = 0.0;
    for (int64_t i = 0; i < n; ++i) s += X[i * c + k];
    s /= (double)n;
    for (int64_t i = 0; i < n; ++i) {
      double t = X[i * c + k] - s;
      q += t * t;
    }
    q = std::sqrt(q / (double)n);
    mu[k] = (float)s;
    sd[k] = q > 1e-12 ? (float)q : 1.f;
  }
}

sbv_status upload_stats(sbv_mlp_s* M) {
  MTRY(M->dmu_x.alloc(M->in));
  MTRY(M->dsd_x.alloc(M->in));
  MTRY(M->dmu_y.alloc(M->out));
  MTRY(M->dsd_y.alloc(M->out));
  MTRY(hipMemcpy(M->dmu_x.p, M->mu_x.data(), sizeof(float) * M->in, hipMemcpyHostToDevice));
  MTRY(hipMemcpy(M->dsd_x.p, M->sd_x.data(), sizeof(float) * M->in, hipMemcpyHostToDevice));
  MTRY(hipMemcpy(M->dmu_y.p, M->mu_y.data(), sizeof(float) * M->out, hipMemcpyHostToDevice));
  MTRY(hipMemcpy(M->dsd_y.p, M->sd_y.data(), sizeof(float) * M->out, hipMemcpyHostToDevice));
  return SBV_OK;
}

}  // namespace

extern "C" {

sbv_status sbv_mlp_create(int32_t in, int32_t hidden, int32_t layers, int32_t out, uint64_t seed, sbv_mlp* h) {
  if (!h || in <= 0 || hidden <= 0 || layers < 0 || out <= 0 || layers > 16)
    return sbv_internal_fail(SBV_E_INVAL, "bad network shape");
  auto M = new sbv_mlp_s();
  M->in = in;
  M->H = hidden;
  M->L = layers;
  M->out = out;
  int64_t o = 0;
  for (int l = 0; l <= layers; ++l) {
    M->off.push_back(o);
    const int di = M->din(l), dout = l < layers ? hidden : out;
    o += (int64_t)dout * di + dout;
  }
  M->np = o;
  std::vector<float> p(o, 0.f);
  Rng r{seed};
  for (int l = 0; l <= layers; ++l) {  // He initialisation, zero biases
    const int di = M->din(l), dout = l < layers ? hidden : out;
    const double sdv = std::sqrt(2.0 / di);
    for (int64_t i = 0; i < (int64_t)dout * di; ++i) p[M->off[l] + i] = (float)(sdv * r.normal());
  }
  M->mu_x.assign(in, 0.f);
  M->sd_x.assign(in, 1.f);
  M->mu_y.assign(out, 0.f);
  M->sd_y.assign(out, 1.f);
  if (M->p.alloc(o) || M->g.alloc(o) || M->m.alloc(o) || M->v.alloc(o)) {
    delete M;
    return sbv_internal_fail(SBV_E_NOMEM, "mlp allocation failed");
  }
  MTRY(hipMemcpy(M->p.p, p.data(), sizeof(float) * o, hipMemcpyHostToDevice));
  MTRY(hipMemset(M->m.p, 0, sizeof(float) * o));
  MTRY(hipMemset(M->v.p, 0, sizeof(float) * o));
  sbv_status st = upload_stats(M);
  if (st) {
    delete M;
    return st;
  }
  *h = M;
  return SBV_OK;
}

void sbv_mlp_free(sbv_mlp h) { delete h; }

int64_t sbv_mlp_num_params(sbv_mlp h) { return h ? h->np : 0; }

sbv_status sbv_mlp_get_params(sbv_mlp h, float* params) {
  if (!h || !params) return sbv_internal_fail(SBV_E_INVAL, "handle and params required");
  MTRY(hipMemcpy(params, h->p.p, sizeof(float) * h->np, hipMemcpyDeviceToHost));
  return SBV_OK;
}

sbv_status sbv_mlp_set_params(sbv_mlp h, const float* params) {
  if (!h || !params) return sbv_internal_fail(SBV_E_INVAL, "handle and params required");
  MTRY(hipMemcpy(h->p.p, params, sizeof(float) * h->np, hipMemcpyHostToDevice));
  return SBV_OK;
}

// Loss and gradient of one batch of raw (unstandardised-by-the-handle) rows:
// the standardisation is NOT applied here, so this is the bare network.
sbv_status sbv_mlp_loss_grad(sbv_mlp h, const float* X, const float* Y, int32_t n, float* loss, float* grad) {
  if (!h || !X || !Y || n <= 0) return sbv_internal_fail(SBV_E_INVAL, "bad arguments");
  MTRY(h->work(n));
  MTRY(hipMemcpy(h->X0.p, X, sizeof(float) * n * h->in, hipMemcpyHostToDevice));
  MTRY(hipMemcpy(h->Yt.p, Y, sizeof(float) * n * h->out, hipMemcpyHostToDevice));
  MTRY(forward(h, n, nullptr));
  MTRY(launch_mse(h->Yh.p, h->Yt.p, (int64_t)n * h->out, h->dY.p, h->loss.p, nullptr));
  MTRY(backward(h, n, nullptr));
  if (loss) MTRY(hipMemcpy(loss, h->loss.p, sizeof(float), hipMemcpyDeviceToHost));
  if (grad) MTRY(hipMemcpy(grad, h->g.p, sizeof(float) * h->np, hipMemcpyDeviceToHost));
  return SBV_OK;
}

// Train with Adam on standardised data for `epochs` passes in shuffled
// mini-batches (SplitMix64(seed) Fisher-Yates per epoch).  The column
// statistics of X and Y are computed here and kept for predict.
sbv_status sbv_mlp_train(sbv_mlp h, const float* X, const float* Y, int64_t n, int32_t epochs, int32_t batch,
                         float lr, uint64_t seed, float* final_loss) {
  if (!h || !X || !Y || n <= 0 || epochs < 0 || batch <= 0) return sbv_internal_fail(SBV_E_INVAL, "bad arguments");
  col_stats(X, n, h->in, h->mu_x, h->sd_x);
  col_stats(Y, n, h->out, h->mu_y, h->sd_y);
  sbv_status st = upload_stats(h);
  if (st) return st;
  DBuf<float> xs, ys, xr, yr;
  DBuf<int32_t> idx;
  MTRY(xr.alloc((size_t)n * h->in));
  MTRY(yr.alloc((size_t)n * h->out));
  MTRY(xs.alloc((size_t)n * h->in));
  MTRY(ys.alloc((size_t)n * h->out));
  MTRY(idx.alloc(n));
  MTRY(hipMemcpy(xr.p, X, sizeof(float) * n * h->in, hipMemcpyHostToDevice));
  MTRY(hipMemcpy(yr.p, Y, sizeof(float) * n * h->out, hipMemcpyHostToDevice));
  MTRY(launch_affine_cols(xr.p, n, h->in, h->dmu_x.p, h->dsd_x.p, xs.p, 0, nullptr));
  MTRY(launch_affine_cols(yr.p, n, h->out, h->dmu_y.p, h->dsd_y.p, ys.p, 0, nullptr));
  const int b = (int)std::min<int64_t>(batch, n);
  MTRY(h->work(b));
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  Rng r{seed};
  double last = 0.0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)r.below((uint64_t)(i + 1))]);
    MTRY(hipMemcpy(idx.p, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    double sum = 0.0;
    int nb = 0;
    for (int64_t s0 = 0; s0 + b <= n; s0 += b) {
      MTRY(launch_gather_rows(xs.p, idx.p + s0, b, h->in, h->X0.p, nullptr));
      MTRY(launch_gather_rows(ys.p, idx.p + s0, b, h->out, h->Yt.p, nullptr));
      MTRY(forward(h, b, nullptr));
      MTRY(launch_mse(h->Yh.p, h->Yt.p, (int64_t)b * h->out, h->dY.p, h->loss.p, nullptr));
      MTRY(backward(h, b, nullptr));
      ++h->adam_t;
      MTRY(launch_adam(h->p.p, h->g.p, h->m.p, h->v.p, h->np, lr, 0.9f, 0.999f, 1e-8f, (int)h->adam_t, nullptr));
      if (ep == epochs - 1) {
        float lv;
        MTRY(hipMemcpy(&lv, h->loss.p, sizeof(float), hipMemcpyDeviceToHost));
        sum += lv;
        ++nb;
      }
    }
    if (ep == epochs - 1 && nb) last = sum / nb;
  }
  MTRY(hipDeviceSynchronize());
  if (final_loss) *final_loss = (float)last;
  return SBV_OK;
}

// Predict n rows (raw features in, raw targets out).
sbv_status sbv_mlp_predict(sbv_mlp h, const float* X, int64_t n, float* Yout) {
  if (!h || !X || !Yout || n <= 0) return sbv_internal_fail(SBV_E_INVAL, "bad arguments");
  DBuf<float> xr, yo;
  MTRY(xr.alloc((size_t)n * h->in));
  MTRY(yo.alloc((size_t)n * h->out));
  MTRY(hipMemcpy(xr.p, X, sizeof(float) * n * h->in, hipMemcpyHostToDevice));
  const int chunk = 1024;
  MTRY(h->work(chunk));
  for (int64_t s0 = 0; s0 < n; s0 += chunk) {
    const int b = (int)std::min<int64_t>(chunk, n - s0);
    MTRY(launch_affine_cols(xr.p + s0 * h->in, b, h->in, h->dmu_x.p, h->dsd_x.p, h->X0.p, 0, nullptr));
    MTRY(forward(h, b, nullptr));
    MTRY(launch_affine_cols(h->Yh.p, b, h->out, h->dmu_y.p, h->dsd_y.p, yo.p + s0 * h->out, 1, nullptr));
  }
  MTRY(hipMemcpy(Yout, yo.p, sizeof(float) * n * h->out, hipMemcpyDeviceToHost));
  return SBV_OK;
}

sbv_status sbv_mlp_save(sbv_mlp h, const char* path) {
  if (!h || !path) return sbv_internal_fail(SBV_E_INVAL, "handle and path required");
  std::vector<float> p(h->np);
  MTRY(hipMemcpy(p.data(), h->p.p, sizeof(float) * h->np, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) return sbv_internal_fail(SBV_E_INVAL, "cannot open file");
  const char magic[8] = {'S', 'B', 'V', 'M', 'L', 'P', '1', 0};
  int32_t shape[4] = {h->in, h->H, h->L, h->out};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(shape, 4, 4, f) == 4 &&
            std::fwrite(h->mu_x.data(), 4, h->in, f) == (size_t)h->in &&
            std::fwrite(h->sd_x.data(), 4, h->in, f) == (size_t)h->in &&
            std::fwrite(h->mu_y.data(), 4, h->out, f) == (size_t)h->out &&
            std::fwrite(h->sd_y.data(), 4, h->out, f) == (size_t)h->out &&
            std::fwrite(p.data(), 4, h->np, f) == (size_t)h->np;
  std::fclose(f);
  return ok ? SBV_OK : sbv_internal_fail(SBV_E_INVAL, "write failed");
}

sbv_status sbv_mlp_load(const char* path, sbv_mlp* out) {
  if (!path || !out) return sbv_internal_fail(SBV_E_INVAL, "path and out required");
  FILE* f = std::fopen(path, "rb");
  if (!f) return sbv_internal_fail(SBV_E_INVAL, "cannot open file");
  char magic[8];
  int32_t shape[4];
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "SBVMLP1", 7) != 0 || std::fread(shape, 4, 4, f) != 4) {
    std::fclose(f);
    return sbv_internal_fail(SBV_E_INVAL, "not a network file");
  }
  sbv_mlp h = nullptr;
  sbv_status st = sbv_mlp_create(shape[0], shape[1], shape[2], shape[3], 0, &h);
  if (st) {
    std::fclose(f);
    return st;
  }
  std::vector<float> p(h->np);
  bool ok = std::fread(h->mu_x.data(), 4, h->in, f) == (size_t)h->in &&
            std::fread(h->sd_x.data(), 4, h->in, f) == (size_t)h->in &&
            std::fread(h->mu_y.data(), 4, h->out, f) == (size_t)h->out &&
            std::fread(h->sd_y.data(), 4, h->out, f) == (size_t)h->out &&
            std::fread(p.data(), 4, h->np, f) == (size_t)h->np;
  std::fclose(f);
  if (!ok) {
    sbv_mlp_free(h);
    return sbv_internal_fail(SBV_E_INVAL, "truncated network file");
  }
  st = upload_stats(h);
  if (!st) st = sbv_mlp_set_params(h, p.data());
  if (st) {
    sbv_mlp_free(h);
    return st;
  }
  *out = h;
  return SBV_OK;
}

// Summary statistics of one dataset (4 + 5 (d + 2) values; 64 for d = 10),
// on a subsample of min(n, sub_n) points drawn by SplitMix64(seed) partial
// Fisher-Yates and taken in increasing id order:
//   log var(y); log mean 1/2 (y_i - y_nn1(i))^2; for neighbour ranks
//   k in {1,2,4,8,16} (Euclidean, unscaled x, 16-NN on the device): the
//   least-squares coefficients of 1/2 (y_i - y_nnk(i))^2 / var(y) on
//   [1, dx_1^2, ..., dx_d^2] and the fit's R^2; then d/10 and 1.
sbv_status sbv_features(const double* X, const double* y, int64_t n, int32_t d, int64_t sub_n, uint64_t seed,
                        double* feat) {
  if (!X || !y || !feat || n < 32 || d <= 0 || d > kMaxDim || sub_n < 32)
    return sbv_internal_fail(SBV_E_INVAL, "bad arguments");
  const int64_t ns = std::min(n, sub_n);
  std::vector<int64_t> sub(ns);
  {
    std::vector<int64_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    Rng r{seed};
    for (int64_t i = 0; i < ns; ++i) std::swap(perm[i], perm[i + (int64_t)r.below((uint64_t)(n - i))]);
    std::copy(perm.begin(), perm.begin() + ns, sub.begin());
    std::sort(sub.begin(), sub.end());
  }
  std::vector<double> P((size_t)ns * d);
  for (int64_t i = 0; i < ns; ++i) std::memcpy(&P[i * d], X + sub[i] * d, sizeof(double) * d);
  std::vector<int32_t> nn((size_t)ns * 16);
  {
    DBuf<double> dP;
    DBuf<int32_t> dnn;
    MTRY(dP.alloc(P.size()));
    MTRY(dnn.alloc(nn.size()));
    MTRY(hipMemcpy(dP.p, P.data(), sizeof(double) * P.size(), hipMemcpyHostToDevice));
    MTRY(launch_knn16(dP.p, (int)ns, d, dnn.p, nullptr));
    MTRY(hipMemcpy(nn.data(), dnn.p, sizeof(int32_t) * nn.size(), hipMemcpyDeviceToHost));
  }
  double mean = 0.0, var = 0.0;
  for (int64_t i = 0; i < ns; ++i) mean += y[sub[i]];
  mean /= (double)ns;
  for (int64_t i = 0; i < ns; ++i) var += (y[sub[i]] - mean) * (y[sub[i]] - mean);
  var /= (double)ns;
  int f = 0;
  feat[f++] = std::log(var);
  {
    double s = 0.0;
    for (int64_t i = 0; i < ns; ++i) {
      double t = y[sub[i]] - y[sub[nn[i * 16]]];
      s += 0.5 * t * t;
    }
    feat[f++] = std::log(s / (double)ns);
  }
  const int ranks[5] = {1, 2, 4, 8, 16};
  const int p = d + 1;
  for (int rk : ranks) {
    std::vector<double> A((size_t)p * p, 0.0), b(p, 0.0), row(p);
    double tmean = 0.0;
    for (int64_t i = 0; i < ns; ++i) {
      double t = y[sub[i]] - y[sub[nn[i * 16 + rk - 1]]];
      tmean += 0.5 * t * t / var;
    }
    tmean /= (double)ns;
    double tss = 0.0;
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t j = nn[i * 16 + rk - 1];
      double t = y[sub[i]] - y[sub[j]];
      double target = 0.5 * t * t / var;
      row[0] = 1.0;
      for (int c = 0; c < d; ++c) {
        double dx = P[i * d + c] - P[j * d + c];
        row[c + 1] = dx * dx;
      }
      for (int a = 0; a < p; ++a) {
        b[a] += row[a] * target;
        for (int c = 0; c < p; ++c) A[a * p + c] += row[a] * row[c];
      }
      tss += (target - tmean) * (target - tmean);
    }
    for (int a = 0; a < p; ++a) A[a * p + a] *= 1.0 + 1e-12;  // scale-free ridge
    // Cholesky solve of the normal equations
    std::vector<double> Lm(A), c(b);
    for (int j = 0; j < p; ++j) {
      double s = Lm[j * p + j];
      for (int k = 0; k < j; ++k) s -= Lm[j * p + k] * Lm[j * p + k];
      Lm[j * p + j] = std::sqrt(std::max(s, 1e-300));
      for (int i = j + 1; i < p; ++i) {
        double t = Lm[i * p + j];
        for (int k = 0; k < j; ++k) t -= Lm[i * p + k] * Lm[j * p + k];
        Lm[i * p + j] = t / Lm[j * p + j];
      }
    }
    for (int i = 0; i < p; ++i) {
      double t = c[i];
      for (int k = 0; k < i; ++k) t -= Lm[i * p + k] * c[k];
      c[i] = t / Lm[i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {
      double t = c[i];
      for (int k = i + 1; k < p; ++k) t -= Lm[k * p + i] * c[k];
      c[i] = t / Lm[i * p + i];
    }
    double rss = 0.0;
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t j = nn[i * 16 + rk - 1];
      double t = y[sub[i]] - y[sub[j]];
      double target = 0.5 * t * t / var, pred = c[0];
      for (int cc = 0; cc < d; ++cc) {
        double dx = P[i * d + cc] - P[j * d + cc];
        pred += c[cc + 1] * dx * dx;
      }
      rss += (target - pred) * (target - pred);
    }
    for (int a = 0; a < p; ++a) feat[f++] = c[a];
    feat[f++] = tss > 0 ? 1.0 - rss / tss : 0.0;
  }
  feat[f++] = d / 10.0;
  feat[f++] = 1.0;
  return SBV_OK;
}

}  // extern "C"
