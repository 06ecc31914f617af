/*
 * FP64 reference of the warm-start network and its summary statistics.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as sbv_oracle.c): used by the tests to
 * check the GPU training/inference kernels and feature kernel.
 *
 * Network: in -> H -> H -> H -> out, fully connected, GELU (exact erf form,
 * 0.5 x (1 + erf(x / sqrt 2))) after every hidden layer, identity output.
 * Parameters are packed layer by layer as W (out x in, row-major) then b (out).
 * Loss: mean squared error over the batch and the outputs,
 *   L = 1/(N * out) sum (yhat - y)^2.
 * Adam (Kingma & Ba 2015) with bias correction.
 *
 * The features and the network are not in the paper; they are the library's own
 * warm-start component, so their parity is pinned only by finite differences
 * and closed-form checks (no paper values exist).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }
static double gelu_d(double x) {
  return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * exp(-0.5 * x * x) / sqrt(2.0 * M_PI);
}

/* Forward pass of N samples: X (N x in) -> out (N x no).  Hidden width H,
 * L hidden layers.  Returns nothing; out must hold N*no doubles. */
void mlp_oracle_forward(const double* params, int in, const double* X, int N, int H, int L, int no,
                        double* out, double* unused) {
  (void)unused;
  double* a = (double*)malloc(sizeof(double) * H);
  double* b = (double*)malloc(sizeof(double) * H);
  for (int s = 0; s < N; ++s) {
    const double* p = params;
    const double* x = X + (int64_t)s * in;
    int din = in;
    for (int l = 0; l < L; ++l) {
      const double* W = p;
      const double* bias = p + (int64_t)H * din;
      for (int o = 0; o < H; ++o) {
        double t = bias[o];
        for (int k = 0; k < din; ++k) t += W[(int64_t)o * din + k] * x[k];
        b[o] = gelu(t);
      }
      p = bias + H;
      memcpy(a, b, sizeof(double) * H);
      x = a;
      din = H;
    }
    const double* W = p;
    const double* bias = p + (int64_t)no * din;
    for (int o = 0; o < no; ++o) {
      double t = bias[o];
      for (int k = 0; k < din; ++k) t += W[(int64_t)o * din + k] * x[k];
      out[(int64_t)s * no + o] = t;
    }
  }
  free(a);
  free(b);
}

/* MSE loss of a batch and its gradient w.r.t. every parameter (packed like
 * params), by back-propagation written out layer by layer. */
double mlp_oracle_loss_grad(const double* params, int in, const double* X, const double* Y, int N, int H, int L,
                            int no, double* grad) {
  int64_t np = 0;
  {
    int din = in;
    for (int l = 0; l < L; ++l) { np += (int64_t)H * din + H; din = H; }
    np += (int64_t)no * din + no;
  }
  memset(grad, 0, sizeof(double) * np);
  double* pre = (double*)malloc(sizeof(double) * L * H);   /* pre-activations */
  double* act = (double*)malloc(sizeof(double) * L * H);   /* activations */
  double* dcur = (double*)malloc(sizeof(double) * (H > no ? H : no));
  double* dnext = (double*)malloc(sizeof(double) * H);
  double loss = 0.0;
  for (int s = 0; s < N; ++s) {
    const double* x0 = X + (int64_t)s * in;
    /* forward, keeping pre-activations */
    const double* p = params;
    const double* x = x0;
    int din = in;
    for (int l = 0; l < L; ++l) {
      const double* W = p;
      const double* bias = p + (int64_t)H * din;
      for (int o = 0; o < H; ++o) {
        double t = bias[o];
        for (int k = 0; k < din; ++k) t += W[(int64_t)o * din + k] * x[k];
        pre[l * H + o] = t;
        act[l * H + o] = gelu(t);
      }
      p = bias + H;
      x = act + l * H;
      din = H;
    }
    const double* Wo = p;
    const double* bo = p + (int64_t)no * din;
    for (int o = 0; o < no; ++o) {
      double t = bo[o];
      for (int k = 0; k < din; ++k) t += Wo[(int64_t)o * din + k] * x[k];
      double e = t - Y[(int64_t)s * no + o];
      loss += e * e;
      dcur[o] = 2.0 * e / ((double)N * no); /* dL/dyhat */
    }
    /* backward: output layer */
    int64_t off = 0;
    int64_t offs[64];
    {
      int dd = in;
      for (int l = 0; l < L; ++l) { offs[l] = off; off += (int64_t)H * dd + H; dd = H; }
      offs[L] = off;
    }
    double* gWo = grad + offs[L];
    double* gbo = gWo + (int64_t)no * H;
    const double* hin = L > 0 ? act + (L - 1) * H : x0;
    int hdim = L > 0 ? H : in;
    for (int o = 0; o < no; ++o) {
      gbo[o] += dcur[o];
      for (int k = 0; k < hdim; ++k) gWo[(int64_t)o * hdim + k] += dcur[o] * hin[k];
    }
    /* delta into the last hidden activation */
    for (int k = 0; k < hdim; ++k) {
      double t = 0.0;
      for (int o = 0; o < no; ++o) t += Wo[(int64_t)o * hdim + k] * dcur[o];
      dnext[k] = t;
    }
    for (int l = L - 1; l >= 0; --l) {
      int dl = (l == 0) ? in : H;
      const double* W = params + offs[l];
      double* gW = grad + offs[l];
      double* gb = gW + (int64_t)H * dl;
      const double* xin = (l == 0) ? x0 : act + (l - 1) * H;
      for (int o = 0; o < H; ++o) dcur[o] = dnext[o] * gelu_d(pre[l * H + o]);
      for (int o = 0; o < H; ++o) {
        gb[o] += dcur[o];
        for (int k = 0; k < dl; ++k) gW[(int64_t)o * dl + k] += dcur[o] * xin[k];
      }
      if (l > 0)
        for (int k = 0; k < dl; ++k) {
          double t = 0.0;
          for (int o = 0; o < H; ++o) t += W[(int64_t)o * dl + k] * dcur[o];
          dnext[k] = t;
        }
    }
  }
  free(pre); free(act); free(dcur); free(dnext);
  return loss / ((double)N * no);
}

/* One Adam step (Kingma & Ba 2015) at step t >= 1. */
void mlp_oracle_adam(double* p, const double* g, double* m, double* v, int64_t n, int t, double lr, double b1,
                     double b2, double eps) {
  double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}

/* --------------------------------------------------------------------------
 * Summary statistics of one dataset (64 values for d = 10), computed on the
 * points listed in `sub` (a seeded subsample chosen by the caller):
 *   f0 = log var(y)
 *   f1 = log mean over points of 1/2 (y_i - y_nn1(i))^2
 *   for each neighbour rank k in {1, 2, 4, 8, 16} (Euclidean, unscaled x):
 *     least-squares fit of 1/2 (y_i - y_nnk(i))^2 / var(y) on
 *     [1, dx_1^2, ..., dx_d^2] -> d+1 coefficients, then the fit's R^2
 *   then d/10 and 1.
 * Length 2 + 5 (d + 2) + 2; the normal equations are solved by Cholesky with
 * each diagonal entry raised by 1e-12 of itself (a scale-free ridge).  Neighbour ties go to the lower subsample index.
 */
static int feat_ranks[5] = {1, 2, 4, 8, 16};

static int chol_solve(double* A, double* b, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0)) return 1;
    A[j * n + j] = sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / A[j * n + j];
    }
  }
  for (int i = 0; i < n; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= A[i * n + k] * b[k];
    b[i] = t / A[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = b[i];
    for (int k = i + 1; k < n; ++k) t -= A[k * n + i] * b[k];
    b[i] = t / A[i * n + i];
  }
  return 0;
}

int sbv_oracle_features(const double* X, const double* y, int64_t n, int d, const int64_t* sub, int64_t ns,
                        double* feat) {
  (void)n;
  if (d <= 0 || d > 32 || ns < 32) return 1;
  const int KMAX = 16;
  int64_t* nn = (int64_t*)malloc(sizeof(int64_t) * ns * KMAX);
  /* brute-force 16 nearest (excluding self) in the subsample */
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < ns; ++i) {
    double bd[16];
    int64_t bi[16];
    int cnt = 0;
    const double* xi = X + sub[i] * d;
    for (int64_t j = 0; j < ns; ++j) {
      if (j == i) continue;
      const double* xj = X + sub[j] * d;
      double s = 0.0;
      for (int k = 0; k < d; ++k) { double t = xi[k] - xj[k]; s += t * t; }
      if (cnt < KMAX || s < bd[cnt - 1]) {
        int p = cnt < KMAX ? cnt++ : KMAX - 1;
        while (p > 0 && bd[p - 1] > s) { bd[p] = bd[p - 1]; bi[p] = bi[p - 1]; --p; }
        bd[p] = s;
        bi[p] = j;
      }
    }
    for (int k = 0; k < KMAX; ++k) nn[i * KMAX + k] = bi[k];
  }
  double mean = 0.0, var = 0.0;
  for (int64_t i = 0; i < ns; ++i) mean += y[sub[i]];
  mean /= (double)ns;
  for (int64_t i = 0; i < ns; ++i) { double t = y[sub[i]] - mean; var += t * t; }
  var /= (double)ns;
  int f = 0;
  feat[f++] = log(var);
  {
    double s = 0.0;
    for (int64_t i = 0; i < ns; ++i) { double t = y[sub[i]] - y[sub[nn[i * KMAX]]]; s += 0.5 * t * t; }
    feat[f++] = log(s / (double)ns);
  }
  const int p = d + 1;
  double* A = (double*)malloc(sizeof(double) * p * p);
  double* b = (double*)malloc(sizeof(double) * p);
  double* row = (double*)malloc(sizeof(double) * p);
  for (int r = 0; r < 5; ++r) {
    const int k = feat_ranks[r] - 1;
    memset(A, 0, sizeof(double) * p * p);
    memset(b, 0, sizeof(double) * p);
    double tss = 0.0, tmean = 0.0;
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t j = nn[i * KMAX + k];
      double t = y[sub[i]] - y[sub[j]];
      tmean += 0.5 * t * t / var;
    }
    tmean /= (double)ns;
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t j = nn[i * KMAX + k];
      double t = y[sub[i]] - y[sub[j]];
      double target = 0.5 * t * t / var;
      row[0] = 1.0;
      for (int c = 0; c < d; ++c) { double dx = X[sub[i] * d + c] - X[sub[j] * d + c]; row[c + 1] = dx * dx; }
      for (int a = 0; a < p; ++a) {
        b[a] += row[a] * target;
        for (int c = 0; c < p; ++c) A[a * p + c] += row[a] * row[c];
      }
      tss += (target - tmean) * (target - tmean);
    }
    for (int a = 0; a < p; ++a) A[a * p + a] *= 1.0 + 1e-12;
    double* Ac = (double*)malloc(sizeof(double) * p * p);
    double* coef = (double*)malloc(sizeof(double) * p);
    memcpy(Ac, A, sizeof(double) * p * p);
    memcpy(coef, b, sizeof(double) * p);
    chol_solve(Ac, coef, p);
    double rss = 0.0;
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t j = nn[i * KMAX + k];
      double t = y[sub[i]] - y[sub[j]];
      double target = 0.5 * t * t / var, pred = coef[0];
      for (int c = 0; c < d; ++c) { double dx = X[sub[i] * d + c] - X[sub[j] * d + c]; pred += coef[c + 1] * dx * dx; }
      rss += (target - pred) * (target - pred);
    }
    for (int a = 0; a < p; ++a) feat[f++] = coef[a];
    feat[f++] = tss > 0 ? 1.0 - rss / tss : 0.0;
    free(Ac);
    free(coef);
  }
  feat[f++] = d / 10.0;
  feat[f++] = 1.0;
  free(A); free(b); free(row); free(nn);
  return 0;
}
