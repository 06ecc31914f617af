// Maximum-likelihood driver (host C++): minimise f(theta) = -l(theta).
//
//  - Nelder-Mead simplex search (Nelder & Mead 1965; reflection 1, expansion 2,
//    contraction 1/2, shrink 1/2), value-only.
//  - L-BFGS (Liu & Nocedal 1989): two-loop recursion over the last `lbfgs_m`
//    pairs, strong-Wolfe line search by bracketing and zoom with cubic
//    interpolation (Nocedal & Wright, Numerical Optimization, Alg. 3.5/3.6).
//  - A checkpoint file (JSON, rewritten after every iteration) holds the full
//    optimiser state; a run started with an existing checkpoint resumes from it
//    and follows the identical trajectory.
// The optimisers work on any objective through sbv_minimize; sbv_fit plugs in
// the device log-likelihood (and gradient) of a handle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/sbv.h"

sbv_status sbv_internal_fail(sbv_status st, const char* msg);
bool sbv_internal_was_built(sbv_blocks h);
sbv_status sbv_internal_rebuild(sbv_blocks h, const double* beta_build);

namespace {

// Progress lines on stderr when the environment variable SBV_PROGRESS is set
// (long fits at large n report every iteration).
bool progress_on() {
  static const bool on = std::getenv("SBV_PROGRESS") != nullptr;
  return on;
}

struct Objective {
  sbv_objective fn;
  void* ctx;
  int64_t evals = 0;
  double eval(const std::vector<double>& x, std::vector<double>* g) {
    ++evals;
    double f = fn(x.data(), g ? g->data() : nullptr, ctx);
    if (!std::isfinite(f)) f = INFINITY;
    return f;
  }
};

// ---- checkpoint (flat JSON of named number arrays) --------------------------
struct State {
  std::string kind;
  int64_t iter = 0, evals = 0;
  std::vector<double> x, fvals, simplex, s_hist, y_hist, g, extra;
  double f = INFINITY;
};

void put(std::ostringstream& o, const char* k, const std::vector<double>& v) {
  o << "\"" << k << "\":[";
  for (size_t i = 0; i < v.size(); ++i) {
    char b[40];
    std::snprintf(b, sizeof b, "%.17g", v[i]);
    o << (i ? "," : "") << b;
  }
  o << "]";
}

bool save_state(const char* path, const State& s) {
  if (!path || !*path) return true;
  std::ostringstream o;
  char b[64];
  std::snprintf(b, sizeof b, "%.17g", s.f);
  o << "{\"kind\":\"" << s.kind << "\",\"iter\":" << s.iter << ",\"evals\":" << s.evals << ",\"f\":" << b << ",";
  put(o, "x", s.x);
  o << ",";
  put(o, "fvals", s.fvals);
  o << ",";
  put(o, "simplex", s.simplex);
  o << ",";
  put(o, "s_hist", s.s_hist);
  o << ",";
  put(o, "y_hist", s.y_hist);
  o << ",";
  put(o, "g", s.g);
  o << ",";
  put(o, "extra", s.extra);
  o << "}\n";
  std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << o.str();
  }
  return std::rename(tmp.c_str(), path) == 0;
}

bool parse_array(const std::string& js, const char* key, std::vector<double>& out) {
  std::string k = std::string("\"") + key + "\":[";
  size_t p = js.find(k);
  if (p == std::string::npos) return false;
  p += k.size();
  size_t e = js.find(']', p);
  out.clear();
  std::string body = js.substr(p, e - p);
  std::stringstream ss(body);
  std::string tok;
  while (std::getline(ss, tok, ','))
    if (!tok.empty()) out.push_back(std::strtod(tok.c_str(), nullptr));
  return true;
}

bool parse_num(const std::string& js, const char* key, double& v) {
  std::string k = std::string("\"") + key + "\":";
  size_t p = js.find(k);
  if (p == std::string::npos) return false;
  v = std::strtod(js.c_str() + p + k.size(), nullptr);
  return true;
}

bool load_state(const char* path, State& s) {
  if (!path || !*path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream b;
  b << f.rdbuf();
  std::string js = b.str();
  size_t p = js.find("\"kind\":\"");
  if (p == std::string::npos) return false;
  size_t e = js.find('"', p + 8);
  s.kind = js.substr(p + 8, e - p - 8);
  double v;
  if (!parse_num(js, "iter", v)) return false;
  s.iter = (int64_t)v;
  if (!parse_num(js, "evals", v)) return false;
  s.evals = (int64_t)v;
  if (!parse_num(js, "f", s.f)) return false;
  parse_array(js, "x", s.x);
  parse_array(js, "fvals", s.fvals);
  parse_array(js, "simplex", s.simplex);
  parse_array(js, "s_hist", s.s_hist);
  parse_array(js, "y_hist", s.y_hist);
  parse_array(js, "g", s.g);
  parse_array(js, "extra", s.extra);
  return true;
}

// ---- Nelder-Mead -------------------------------------------------------------
sbv_status nelder_mead(Objective& obj, std::vector<double>& x, const sbv_fit_opts& o, double& fbest,
                       bool& converged) {
  const int n = (int)x.size();
  std::vector<std::vector<double>> P(n + 1, x);
  std::vector<double> F(n + 1);
  State st;
  st.kind = "nelder-mead";
  bool resumed = false;
  if (o.checkpoint_path && load_state(o.checkpoint_path, st) && st.kind == "nelder-mead" &&
      (int)st.simplex.size() == n * (n + 1) && (int)st.fvals.size() == n + 1) {
    for (int i = 0; i <= n; ++i) {
      for (int k = 0; k < n; ++k) P[i][k] = st.simplex[i * n + k];
      F[i] = st.fvals[i];
    }
    obj.evals = st.evals;
    resumed = true;
  } else {
    st.iter = 0;
    F[0] = obj.eval(P[0], nullptr);
    const double h = o.init_step > 0 ? o.init_step : 0.5;
    for (int i = 1; i <= n; ++i) {
      P[i][i - 1] += h;
      F[i] = obj.eval(P[i], nullptr);
    }
  }
  (void)resumed;
  converged = false;
  std::vector<int> idx(n + 1);
  while (obj.evals < o.max_evals) {
    for (int i = 0; i <= n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return F[a] < F[b]; });
    {
      std::vector<std::vector<double>> P2(n + 1);
      std::vector<double> F2(n + 1);
      for (int i = 0; i <= n; ++i) {
        P2[i] = P[idx[i]];
        F2[i] = F[idx[i]];
      }
      P.swap(P2);
      F.swap(F2);
    }
    // checkpoint the ordered simplex
    st.simplex.clear();
    for (int i = 0; i <= n; ++i) st.simplex.insert(st.simplex.end(), P[i].begin(), P[i].end());
    st.fvals = F;
    st.x = P[0];
    st.f = F[0];
    st.evals = obj.evals;
    save_state(o.checkpoint_path, st);
    ++st.iter;
    if (progress_on() && st.iter % 25 == 0)
      std::fprintf(stderr, "[fit] nelder-mead iteration %lld, %lld evaluations, f %.10g\n", (long long)st.iter,
                   (long long)obj.evals, F[0]);
    const double spread = F[n] - F[0];
    if (std::isfinite(F[n]) && spread <= o.ftol * (std::fabs(F[0]) + 1e-300)) {
      converged = true;
      break;
    }
    std::vector<double> c(n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) c[k] += P[i][k] / n;
    auto along = [&](double t) {
      std::vector<double> y(n);
      for (int k = 0; k < n; ++k) y[k] = c[k] + t * (P[n][k] - c[k]);
      return y;
    };
    std::vector<double> xr = along(-1.0);
    double fr = obj.eval(xr, nullptr);
    if (fr < F[0]) {
      std::vector<double> xe = along(-2.0);
      double fe = obj.eval(xe, nullptr);
      if (fe < fr) {
        P[n] = xe;
        F[n] = fe;
      } else {
        P[n] = xr;
        F[n] = fr;
      }
    } else if (fr < F[n - 1]) {
      P[n] = xr;
      F[n] = fr;
    } else {
      const bool outside = fr < F[n];
      std::vector<double> xc = along(outside ? -0.5 : 0.5);
      double fc = obj.eval(xc, nullptr);
      if (fc < (outside ? fr : F[n])) {
        P[n] = xc;
        F[n] = fc;
      } else {
        for (int i = 1; i <= n; ++i) {
          for (int k = 0; k < n; ++k) P[i][k] = P[0][k] + 0.5 * (P[i][k] - P[0][k]);
          F[i] = obj.eval(P[i], nullptr);
        }
      }
    }
  }
  int b = (int)(std::min_element(F.begin(), F.end()) - F.begin());
  x = P[b];
  fbest = F[b];
  return SBV_OK;
}

// ---- L-BFGS with a strong-Wolfe line search -----------------------------------
double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

double cubic_min(double a, double fa, double ga, double b, double fb, double gb) {
  // minimiser of the cubic interpolating (a, fa, ga), (b, fb, gb), safeguarded
  const double d1 = ga + gb - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - ga * gb;
  if (disc < 0.0 || !std::isfinite(disc)) return 0.5 * (a + b);
  const double d2 = std::copysign(std::sqrt(disc), b - a);
  double t = b - (b - a) * (gb + d2 - d1) / (gb - ga + 2.0 * d2);
  const double lo = std::min(a, b), hi = std::max(a, b);
  if (!std::isfinite(t) || t <= lo + 0.1 * (hi - lo) || t >= hi - 0.1 * (hi - lo)) t = 0.5 * (a + b);
  return t;
}

// Returns the accepted step (0 if none) and leaves x, f, g at the new point.
double wolfe_search(Objective& obj, std::vector<double>& x, double& f, std::vector<double>& g,
                    const std::vector<double>& p, double a1, int64_t max_evals, int max_trials = 30) {
  const double c1 = 1e-4, c2 = 0.9;
  const double f0 = f, g0 = dot(g, p);
  if (!(g0 < 0.0)) return 0.0;
  const int n = (int)x.size();
  std::vector<double> x0 = x, xt(n), gt(n);
  auto phi = [&](double a, double& fa, double& ga) {
    for (int i = 0; i < n; ++i) xt[i] = x0[i] + a * p[i];
    fa = obj.eval(xt, &gt);
    ga = std::isfinite(fa) ? dot(gt, p) : NAN;
  };
  double a_prev = 0.0, f_prev = f0, g_prev = g0, a = a1;
  auto accept = [&](double aa) {
    x = xt;
    g = gt;
    (void)aa;
  };
  auto zoom = [&](double lo, double flo, double glo, double hi, double fhi, double ghi) -> double {
    for (int it = 0; it < max_trials && obj.evals < max_evals; ++it) {
      double aj = std::isfinite(fhi) && std::isfinite(ghi) ? cubic_min(lo, flo, glo, hi, fhi, ghi) : 0.5 * (lo + hi);
      double fj, gj;
      phi(aj, fj, gj);
      if (!std::isfinite(fj) || fj > f0 + c1 * aj * g0 || fj >= flo) {
        hi = aj;
        fhi = fj;
        ghi = gj;
      } else {
        if (std::fabs(gj) <= -c2 * g0) {
          f = fj;
          accept(aj);
          return aj;
        }
        if (gj * (hi - lo) >= 0.0) {
          hi = lo;
          fhi = flo;
          ghi = glo;
        }
        lo = aj;
        flo = fj;
        glo = gj;
      }
    }
    // best sufficient-decrease point found
    if (lo > 0.0) {
      double fl, gl;
      phi(lo, fl, gl);
      if (std::isfinite(fl) && fl < f0) {
        f = fl;
        accept(lo);
        return lo;
      }
    }
    return 0.0;
  };
  for (int it = 0; it < max_trials && obj.evals < max_evals; ++it) {
    double fa, ga;
    phi(a, fa, ga);
    if (!std::isfinite(fa)) {  // outside the domain (e.g. not positive definite): back off
      a = 0.5 * (a_prev + a);
      continue;
    }
    if (fa > f0 + c1 * a * g0 || (it > 0 && fa >= f_prev)) return zoom(a_prev, f_prev, g_prev, a, fa, ga);
    if (std::fabs(ga) <= -c2 * g0) {
      f = fa;
      accept(a);
      return a;
    }
    if (ga >= 0.0) return zoom(a, fa, ga, a_prev, f_prev, g_prev);
    a_prev = a;
    f_prev = fa;
    g_prev = ga;
    a = 2.0 * a;
  }
  return 0.0;
}

// coarse: a phase that a finer one will finish (FP32 before an FP64 polish):
// line searches get a few trials and a failed one ends the phase instead of
// restarting along steepest descent.
sbv_status lbfgs(Objective& obj, std::vector<double>& x, const sbv_fit_opts& o, double& fbest, bool& converged,
                 bool coarse = false) {
  const int n = (int)x.size();
  const int M = o.lbfgs_m > 0 ? o.lbfgs_m : 10;
  std::vector<double> g(n);
  std::vector<std::vector<double>> S, Y;
  State st;
  st.kind = "lbfgs";
  double f;
  if (o.checkpoint_path && load_state(o.checkpoint_path, st) && st.kind == "lbfgs" && (int)st.x.size() == n &&
      (int)st.g.size() == n) {
    x = st.x;
    g = st.g;
    f = st.f;
    obj.evals = st.evals;
    const int h = (int)st.s_hist.size() / n;
    for (int i = 0; i < h; ++i) {
      S.emplace_back(st.s_hist.begin() + i * n, st.s_hist.begin() + (i + 1) * n);
      Y.emplace_back(st.y_hist.begin() + i * n, st.y_hist.begin() + (i + 1) * n);
    }
  } else {
    f = obj.eval(x, &g);
    st.iter = 0;
    if (!std::isfinite(f)) return sbv_internal_fail(SBV_E_NOTPD, "objective is not finite at the start point");
  }
  converged = false;
  while (obj.evals < o.max_evals) {
    st.x = x;
    st.g = g;
    st.f = f;
    st.evals = obj.evals;
    st.s_hist.clear();
    st.y_hist.clear();
    for (size_t i = 0; i < S.size(); ++i) {
      st.s_hist.insert(st.s_hist.end(), S[i].begin(), S[i].end());
      st.y_hist.insert(st.y_hist.end(), Y[i].begin(), Y[i].end());
    }
    save_state(o.checkpoint_path, st);
    ++st.iter;
    double gmax = 0.0;
    for (double v : g) gmax = std::max(gmax, std::fabs(v));
    if (progress_on())
      std::fprintf(stderr, "[fit] l-bfgs iteration %lld, %lld evaluations, f %.12g, max |g| %.3g\n",
                   (long long)st.iter, (long long)obj.evals, f, gmax);
    if (gmax <= o.gtol) {
      converged = true;
      break;
    }
    // two-loop recursion
    std::vector<double> q = g, alpha(S.size());
    for (int i = (int)S.size() - 1; i >= 0; --i) {
      alpha[i] = dot(S[i], q) / dot(Y[i], S[i]);
      for (int k = 0; k < n; ++k) q[k] -= alpha[i] * Y[i][k];
    }
    double gamma = S.empty() ? 1.0 / std::max(1.0, gmax) : dot(S.back(), Y.back()) / dot(Y.back(), Y.back());
    for (int k = 0; k < n; ++k) q[k] *= gamma;
    for (size_t i = 0; i < S.size(); ++i) {
      double beta = dot(Y[i], q) / dot(Y[i], S[i]);
      for (int k = 0; k < n; ++k) q[k] += S[i][k] * (alpha[i] - beta);
    }
    std::vector<double> p(n);
    for (int k = 0; k < n; ++k) p[k] = -q[k];
    if (!(dot(p, g) < 0.0)) {  // not a descent direction: restart from steepest descent
      S.clear();
      Y.clear();
      for (int k = 0; k < n; ++k) p[k] = -g[k] / std::max(1.0, gmax);
    }
    const std::vector<double> xold = x, gold = g;
    const double fold = f;
    double a = wolfe_search(obj, x, f, g, p, 1.0, o.max_evals, coarse ? 8 : 30);
    if (a == 0.0) {
      if (!S.empty() && !coarse) {  // retry once along steepest descent
        S.clear();
        Y.clear();
        continue;
      }
      break;
    }
    std::vector<double> s(n), y(n);
    for (int k = 0; k < n; ++k) {
      s[k] = x[k] - xold[k];
      y[k] = g[k] - gold[k];
    }
    if (dot(s, y) > 1e-12 * std::sqrt(dot(s, s) * dot(y, y))) {
      S.push_back(s);
      Y.push_back(y);
      if ((int)S.size() > M) {
        S.erase(S.begin());
        Y.erase(Y.begin());
      }
    }
    if (std::fabs(fold - f) <= o.ftol * std::max(std::fabs(f), 1e-300)) {
      converged = true;
      break;
    }
  }
  fbest = f;
  return SBV_OK;
}

sbv_status run_minimize(int32_t method, std::vector<double>& x, Objective& obj, const sbv_fit_opts& o,
                        double& fbest, bool& converged, bool coarse = false) {
  if (method == SBV_NELDER_MEAD) return nelder_mead(obj, x, o, fbest, converged);
  if (method == SBV_LBFGS) return lbfgs(obj, x, o, fbest, converged, coarse);
  return sbv_internal_fail(SBV_E_INVAL, "unknown optimizer");
}

// Device objective of sbv_fit: -l(theta) (and -grad) of one handle.
struct FitCtx {
  sbv_blocks h;
  int32_t two_nu;
  int32_t prec;
  sbv_status last = SBV_OK;
};

double fit_objective(const double* x, double* g, void* ctx) {
  FitCtx* c = (FitCtx*)ctx;
  double l = -INFINITY;
  sbv_status st;
  if (g) {
    int64_t n;
    int32_t d;
    sbv_blocks_info(c->h, &n, &d, nullptr, nullptr);
    st = sbv_loglik_grad(&c->h, 1, x, &c->two_nu, c->prec, &l, g);
    if (st == SBV_OK)
      for (int k = 0; k < d + 2; ++k) g[k] = -g[k];
  } else {
    st = sbv_loglik(&c->h, 1, x, &c->two_nu, c->prec, &l);
  }
  if (st != SBV_OK && st != SBV_E_NOTPD) c->last = st;
  if (st != SBV_OK) return INFINITY;
  return -l;
}

}  // namespace

extern "C" {

sbv_status sbv_minimize(int32_t method, int32_t n, double* x, sbv_objective fn, void* ctx,
                        const sbv_fit_opts* opts, double* fbest, int32_t* n_evals) {
  if (n <= 0 || !x || !fn || !opts) return sbv_internal_fail(SBV_E_INVAL, "n, x, fn and opts are required");
  Objective obj{fn, ctx};
  std::vector<double> xv(x, x + n);
  double fb = INFINITY;
  bool conv = false;
  sbv_status st = run_minimize(method, xv, obj, *opts, fb, conv);
  if (st) return st;
  std::memcpy(x, xv.data(), sizeof(double) * n);
  if (fbest) *fbest = fb;
  if (n_evals) *n_evals = (int32_t)obj.evals;
  return conv ? SBV_OK : SBV_E_NOCONV;
}

sbv_status sbv_fit(sbv_blocks set, const double* theta0, int32_t two_nu, const sbv_fit_opts* o, double* theta_hat,
                   double* loglik_fp64, int32_t* n_evals, double* seconds) {
  if (!set || !theta0 || !o || !theta_hat) return sbv_internal_fail(SBV_E_INVAL, "set, theta0, o, theta_hat required");
  if (o->rebuild_rounds < 0) return sbv_internal_fail(SBV_E_INVAL, "rebuild_rounds must be >= 0");
  if (o->rebuild_rounds > 0 && !sbv_internal_was_built(set))
    return sbv_internal_fail(SBV_E_INVAL, "rebuild_rounds > 0 needs a handle made by sbv_build_blocks");
  if (o->prec != SBV_FP64 && o->prec != SBV_FP32) return sbv_internal_fail(SBV_E_INVAL, "bad precision");
  int64_t n;
  int32_t d;
  sbv_blocks_info(set, &n, &d, nullptr, nullptr);
  for (int k = 0; k < d + 2; ++k)
    if (!std::isfinite(theta0[k])) return sbv_internal_fail(SBV_E_INVAL, "theta0 has non-finite values");
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> x(theta0, theta0 + d + 2);
  int64_t evals = 0;
  bool conv = false;
  // One optimisation on the handle's current structure, from x.
  auto one_fit = [&](const sbv_fit_opts& oo) -> sbv_status {
    FitCtx c{set, two_nu, oo.prec};
    Objective obj{fit_objective, &c};
    double fb = INFINITY;
    // With an FP64 polish to follow, the FP32 phase stops once an iteration
    // changes -l by less than kFp32Ftol relative: below that, FP32 rounding of
    // the block terms hides real progress and line searches only fail.
    constexpr double kFp32Ftol = 1e-7;
    sbv_fit_opts first = oo;
    const bool coarse = oo.fp64_polish && oo.prec == SBV_FP32;
    if (coarse) first.ftol = std::max(oo.ftol, kFp32Ftol);
    first.max_evals = std::max<int32_t>(oo.max_evals - (int32_t)evals, 1);
    sbv_status st = run_minimize(oo.optimizer, x, obj, first, fb, conv, coarse);
    if (st) return st;
    if (c.last != SBV_OK) return c.last;
    evals += obj.evals;
    if (coarse) {
      // finish in FP64 from the FP32 optimum (no checkpoint for the polish)
      sbv_fit_opts po = oo;
      po.prec = SBV_FP64;
      po.checkpoint_path = nullptr;
      po.max_evals = std::max<int32_t>(oo.max_evals - (int32_t)evals, 1);
      FitCtx c2{set, two_nu, SBV_FP64};
      Objective obj2{fit_objective, &c2};
      st = run_minimize(oo.optimizer, x, obj2, po, fb, conv);
      if (st) return st;
      evals += obj2.evals;
    }
    return SBV_OK;
  };
  sbv_status st = one_fit(*o);
  if (st) return st;
  // Outer rounds: rebuild the structure (blocks, order, neighbours) at the
  // fitted ranges, then continue the fit from the current optimum.  Checkpoints
  // belong to the first round only.
  for (int r = 0; r < o->rebuild_rounds; ++r) {
    std::vector<double> beta(d);
    for (int k = 0; k < d; ++k) beta[k] = std::exp(x[k]);
    st = sbv_internal_rebuild(set, beta.data());
    if (st) return st;
    sbv_fit_opts later = *o;
    later.checkpoint_path = nullptr;
    st = one_fit(later);
    if (st) return st;
  }
  double l64 = -INFINITY;
  st = sbv_loglik(&set, 1, x.data(), &two_nu, SBV_FP64, &l64);
  if (st != SBV_OK && st != SBV_E_NOTPD) return st;
  std::memcpy(theta_hat, x.data(), sizeof(double) * (d + 2));
  if (loglik_fp64) *loglik_fp64 = l64;
  if (n_evals) *n_evals = (int32_t)evals;
  if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return conv ? SBV_OK : SBV_E_NOCONV;
}

}  // extern "C"
