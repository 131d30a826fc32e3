// Batched quasi-Newton minimiser of the chi^2 / likelihood cost (host FP64).
//
// The paper minimises its cost with Minuit2's variable-metric method
// (MIGRAD), calling the GPU cost once per function evaluation (Sec. 4.2,
// Table 1).  This minimiser keeps that method's ingredients -- an inverse
// Hessian updated by BFGS, a line search along -V g, the estimated distance
// to the minimum EDM = g^T V g / 2 -- and changes how it talks to the GPU:
//
//   * every fit is a state machine that posts the parameter vectors it needs
//     next (a line-search point, or the 2n points of a Hessian stencil);
//   * one round gathers the posts of all active fits into one batched launch
//     (mu_chi2_batch) that returns each point's cost and analytic gradient;
//   * the start Hessian and a final Newton polish use central differences of
//     the analytic gradient, so the result is the minimum to ~1e-10 of the
//     parameter errors rather than to a loose EDM.
//
// The plain path (batched = 0, analytic_grad = 0) runs the same state machine
// one fit at a time with one launch per cost evaluation and central-difference
// gradients: the single-evaluation GPU path the batched one is compared with.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mu_internal.h"
#include "mu_runtime.h"

using namespace mu;

namespace {

enum Phase { kStart, kHessInit, kIter, kLine, kHessPolish, kPolish, kDone };
constexpr int kRefresh = 50;  // variable-metric steps between Hessian refreshes of an unconverged fit
// Times a fit that stalls with its EDM above the tolerance (steps below the
// step tolerance, a failed line search, or a polish that cannot lower the
// cost) starts again from a fresh differenced Hessian before it gives up.
constexpr int kMaxStalls = 3;

struct Point {
  std::vector<double> p;  // full parameter vector
  bool grad;
  double cost = 0.0;
  std::vector<double> g;  // full gradient (ld) when grad
};

// Cholesky factorisation in place (lower); false when not positive definite.
bool cholesky(std::vector<double> &A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double l = std::sqrt(d);
    A[j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / l;
    }
  }
  return true;
}

// Inverse of a symmetric positive definite matrix from its Cholesky factor.
std::vector<double> spd_inverse(const std::vector<double> &L, int n) {
  std::vector<double> inv(n * n, 0.0), col(n);
  for (int c = 0; c < n; ++c) {
    // solve L y = e_c, then L^T x = y
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * col[k];
      col[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = col[i];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * col[k];
      col[i] = s / L[i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[i * n + c] = col[i];
  }
  return inv;
}

struct Fit {
  int id = 0;  // index of the fit in the caller's arrays
  int ld = 0, n = 0;
  std::vector<int> fi;  // free parameter indices
  std::vector<double> base;  // full vector (fixed entries stay)
  std::vector<double> x, g, V, H, d, xt, hstep;
  double f = 0.0, gd = 0.0, alpha = 1.0, edm = 0.0, last_step = 1e300;
  int phase = kStart;
  int n_iter = 0, n_fcn = 0, n_grad = 0, status = 0, tries = 0, polish_iter = 0;
  int refreshed = -1;  // iteration of the last Hessian refresh
  int stalls = 0;      // restarts after a stall (at most kMaxStalls)
  std::vector<Point> posts;

  std::vector<double> full(const std::vector<double> &xf) const {
    std::vector<double> p = base;
    for (int k = 0; k < n; ++k) p[fi[k]] = xf[k];
    return p;
  }
  void post(const std::vector<double> &xf, bool grad) {
    Point q;
    q.p = full(xf);
    q.grad = grad;
    posts.push_back(std::move(q));
  }
  double sigma(int k) const { return std::sqrt(std::max(2.0 * V[k * n + k], 0.0)); }
  double scale(int k) const { return std::max(std::fabs(x[k]), sigma(k)); }

  void post_hessian() {
    hstep.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
      const double s = (V.empty() ? 0.0 : sigma(k));
      hstep[k] = 1e-5 * std::max({std::fabs(x[k]), s, 1e-3});
      for (int sg = 1; sg >= -1; sg -= 2) {
        std::vector<double> xx = x;
        xx[k] += sg * hstep[k];
        post(xx, true);
      }
    }
  }
  // Hessian from the posted gradient stencil (central differences, symmetrised).
  std::vector<double> take_hessian() {
    std::vector<double> A(n * n);
    for (int k = 0; k < n; ++k) {
      const Point &pp = posts[2 * k], &pm = posts[2 * k + 1];
      for (int i = 0; i < n; ++i) A[i * n + k] = (pp.g[fi[i]] - pm.g[fi[i]]) / (2.0 * hstep[k]);
    }
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < i; ++k) {
        const double s = 0.5 * (A[i * n + k] + A[k * n + i]);
        A[i * n + k] = A[k * n + i] = s;
      }
    return A;
  }
  // V = A^-1. An indefinite A (away from the minimum) is made positive
  // definite by a diagonal shift mu |A_kk|, mu growing tenfold from 1e-3,
  // which keeps its correlations; the diagonal alone is the last resort.
  void set_v_from(const std::vector<double> &A) {
    std::vector<double> L = A;
    if (cholesky(L, n)) {
      V = spd_inverse(L, n);
      return;
    }
    for (double mu = 1e-3; mu <= 1e3; mu *= 10.0) {
      L = A;
      for (int k = 0; k < n; ++k) L[k * n + k] += mu * std::fabs(A[k * n + k]);
      if (cholesky(L, n)) {
        V = spd_inverse(L, n);
        return;
      }
    }
    V.assign(n * n, 0.0);
    for (int k = 0; k < n; ++k) {
      const double h = std::fabs(A[k * n + k]);
      V[k * n + k] = h > 0.0 && std::isfinite(h) ? 1.0 / h : 1e-6 * std::max(x[k] * x[k], 1.0);
    }
  }
  void direction() {
    d.assign(n, 0.0);
    gd = 0.0;
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s -= V[i * n + k] * g[k];
      d[i] = s;
      gd += g[i] * s;
    }
    if (!(gd < 0.0)) {  // not a descent direction: fall back to the diagonal
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k)
          if (i != k) V[i * n + k] = 0.0;
      gd = 0.0;
      for (int i = 0; i < n; ++i) {
        V[i * n + i] = std::fabs(V[i * n + i]) > 0.0 ? std::fabs(V[i * n + i]) : 1e-6;
        d[i] = -V[i * n + i] * g[i];
        gd += g[i] * d[i];
      }
    }
    edm = -0.5 * gd;
  }
  // End of the fit: EDM from the final gradient and metric (after a polish
  // the inverse of the differenced Hessian), and the status it supports.  A
  // fit is converged only when that EDM is below the tolerance, whatever
  // stopped it; a fit that stopped on a small step (or a failed line search)
  // with a larger EDM keeps a status of its own.
  void finish(double tol_edm) {
    edm = 0.0;
    if (!V.empty())
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) edm += 0.5 * g[i] * V[i * n + k] * g[k];
    if (status != 2) {
      if (edm < tol_edm)
        status = 0;
      else if (status == 0)
        status = 4;
    }
    phase = kDone;
  }
  void post_line() {
    xt.assign(n, 0.0);
    for (int k = 0; k < n; ++k) xt[k] = x[k] + alpha * d[k];
    post(xt, true);
  }
};

}  // namespace

namespace mu {

struct FitDriver {
  mu_ctx *ctx;
  int n_fits, ld;
  const mu_data *const *data;
  const mu_theory *const *th;
  int cost_kind;
  mu_fit_opts o;

  // Evaluate posted points; returns MU_OK or an error.  With analytic
  // gradients the points go out as they are; otherwise every gradient point
  // becomes 2n + 1 cost evaluations (central differences).
  mu_status evaluate(std::vector<Fit *> &fits, bool one_launch_per_point) {
    struct Job {
      int fit, point, k, sign;  // k >= 0: finite-difference neighbour of parameter k
    };
    std::vector<Job> jobs;
    std::vector<double> P;
    bool any_grad = false;
    for (size_t f = 0; f < fits.size(); ++f) {
      Fit &F = *fits[f];
      for (size_t q = 0; q < F.posts.size(); ++q) {
        const Point &pt = F.posts[q];
        jobs.push_back({(int)f, (int)q, -1, 0});
        P.insert(P.end(), pt.p.begin(), pt.p.end());
        if (pt.grad && o.analytic_grad) any_grad = true;
        if (pt.grad && !o.analytic_grad) {
          for (int k = 0; k < F.n; ++k)
            for (int sg = 1; sg >= -1; sg -= 2) {
              std::vector<double> pp = pt.p;
              const int i = F.fi[k];
              pp[i] += sg * fd_step(pt.p[i]);
              jobs.push_back({(int)f, (int)q, k, sg});
              P.insert(P.end(), pp.begin(), pp.end());
            }
        }
      }
    }
    const int nj = (int)jobs.size();
    if (nj == 0) return MU_OK;
    std::vector<double> cost(nj), grad(any_grad ? (size_t)nj * ld : 0);
    std::vector<const mu_data *> dv(nj);
    std::vector<const mu_theory *> tv(nj);
    for (int j = 0; j < nj; ++j) {
      dv[j] = fit_data[fits[jobs[j].fit]->id];
      tv[j] = fit_theory[fits[jobs[j].fit]->id];
    }
    mu_status st;
    if (!one_launch_per_point) {
      st = mu_chi2_batch(ctx, nj, dv.data(), tv.data(), (mu_cost)cost_kind, ld, P.data(), MU_MEM_HOST, cost.data(),
                         any_grad ? grad.data() : nullptr);
      if (st != MU_OK) return st;
    } else {
      for (int j = 0; j < nj; ++j) {
        const int np = tv[j]->h.n_par;
        if (any_grad && jobs[j].k < 0 && fits[jobs[j].fit]->posts[jobs[j].point].grad)
          st = mu_chi2_grad(ctx, dv[j], tv[j], (mu_cost)cost_kind, &P[(size_t)j * ld], 1, MU_MEM_HOST, &cost[j],
                            &grad[(size_t)j * ld]);
        else
          st = mu_chi2_eval(ctx, dv[j], tv[j], (mu_cost)cost_kind, &P[(size_t)j * ld], 1, MU_MEM_HOST, &cost[j],
                            nullptr);
        if (st != MU_OK) return st;
        (void)np;
      }
    }
    // scatter the results back
    for (int j = 0; j < nj; ++j) {
      Fit &F = *fits[jobs[j].fit];
      Point &pt = F.posts[jobs[j].point];
      if (jobs[j].k < 0) {
        pt.cost = cost[j];
        F.n_fcn++;
        if (pt.grad) {
          F.n_grad++;
          pt.g.assign(ld, 0.0);
          if (o.analytic_grad)
            for (int i = 0; i < ld; ++i) pt.g[i] = grad[(size_t)j * ld + i];
        }
      } else {
        F.n_fcn++;
        const int i = F.fi[jobs[j].k];
        const double h = fd_step(pt.p[i]);
        // central difference: (f(+h) - f(-h)) / 2h, the pair is adjacent
        if (jobs[j].sign > 0) pt.g[i] = (cost[j] - cost[j + 1]) / (2.0 * h);
      }
    }
    return MU_OK;
  }

  static double fd_step(double v) { return 1e-6 * std::max(std::fabs(v), 1e-2); }

  std::vector<const mu_data *> fit_data;
  std::vector<const mu_theory *> fit_theory;

  // Advance a fit after its posts were evaluated; posts the next request.
  void advance(Fit &F) {
    std::vector<Point> got;
    got.swap(F.posts);
    const int n = F.n;
    auto budget_left = [&]() { return F.n_fcn < o.max_fcn; };
    switch (F.phase) {
      case kStart: {
        F.f = got[0].cost;
        F.g.assign(n, 0.0);
        for (int k = 0; k < n; ++k) F.g[k] = got[0].g[F.fi[k]];
        if (!std::isfinite(F.f)) {
          F.status = 2;
          F.phase = kDone;
          return;
        }
        F.post_hessian();
        F.phase = kHessInit;
        return;
      }
      case kHessInit: {
        F.posts = got;
        std::vector<double> A = F.take_hessian();
        F.posts.clear();
        F.set_v_from(A);
        F.phase = kIter;
        break;
      }
      case kLine: {
        const double ft = got[0].cost;
        if (std::isfinite(ft) && ft <= F.f + 1e-4 * F.alpha * F.gd) {
          std::vector<double> gt(n);
          for (int k = 0; k < n; ++k) gt[k] = got[0].g[F.fi[k]];
          std::vector<double> s(n), y(n);
          double sy = 0.0, ss = 0.0, yy = 0.0;
          for (int k = 0; k < n; ++k) {
            s[k] = F.xt[k] - F.x[k];
            y[k] = gt[k] - F.g[k];
            sy += s[k] * y[k];
            ss += s[k] * s[k];
            yy += y[k] * y[k];
          }
          if (sy > 1e-12 * std::sqrt(ss * yy)) {  // BFGS update of the inverse Hessian
            std::vector<double> Vy(n, 0.0);
            double yVy = 0.0;
            for (int i = 0; i < n; ++i) {
              for (int k = 0; k < n; ++k) Vy[i] += F.V[i * n + k] * y[k];
              yVy += y[i] * Vy[i];
            }
            const double rho = 1.0 / sy;
            for (int i = 0; i < n; ++i)
              for (int k = 0; k < n; ++k)
                F.V[i * n + k] += rho * ((1.0 + rho * yVy) * s[i] * s[k] - Vy[i] * s[k] - s[i] * Vy[k]);
          }
          double step = 0.0;
          for (int k = 0; k < n; ++k) step = std::max(step, std::fabs(s[k]) / std::max(F.scale(k), 1e-300));
          F.last_step = step;
          F.x = F.xt;
          F.f = ft;
          F.g = gt;
          F.n_iter++;
          F.phase = kIter;
          break;
        }
        // backtrack: minimiser of the quadratic through f, f'(0) = gd and f(alpha)
        const double a = F.alpha;
        double an = std::isfinite(ft) ? -F.gd * a * a / (2.0 * (ft - F.f - F.gd * a)) : 0.1 * a;
        an = std::min(std::max(an, 0.1 * a), 0.5 * a);
        F.alpha = an;
        if (++F.tries > 40 && budget_left() && F.stalls < kMaxStalls && F.n_iter < o.max_iter) {
          // no acceptable point along -V g: restart from a differenced Hessian
          F.stalls++;
          F.refreshed = F.n_iter;
          F.last_step = 1e300;
          F.post_hessian();
          F.phase = kHessInit;
          return;
        }
        if (F.tries > 40 || !budget_left()) {
          F.status = budget_left() ? 3 : 1;
          if (o.polish) {
            F.post_hessian();
            F.phase = kHessPolish;
          } else {
            F.finish(o.tol_edm);
          }
          return;
        }
        F.post_line();
        return;
      }
      case kHessPolish: {
        F.posts = got;
        F.H = F.take_hessian();
        F.posts.clear();
        F.set_v_from(F.H);
        F.polish_iter = 0;
        F.phase = kPolish;
        post_newton(F);
        return;
      }
      case kPolish: {
        const double ft = got[0].cost;
        if (std::isfinite(ft) && ft <= F.f + 1e-13 * std::fabs(F.f)) {
          double step = 0.0;
          for (int k = 0; k < n; ++k) step = std::max(step, std::fabs(F.xt[k] - F.x[k]) / std::max(F.scale(k), 1e-300));
          F.x = F.xt;
          F.f = ft;
          for (int k = 0; k < n; ++k) F.g[k] = got[0].g[F.fi[k]];
          if (step > 1e-12 && ++F.polish_iter < 8 && budget_left()) {
            post_newton(F);
            return;
          }
        }
        if (polish_stalled(F)) break;
        F.finish(o.tol_edm);
        return;
      }
      default:
        return;
    }
    // kIter: new direction, convergence check, next line-search point
    if (!budget_left()) {
      F.status = 1;
      F.phase = kDone;
      return;
    }
    F.direction();
    // a fit that has not converged after kRefresh steps gets a fresh Hessian
    // (by differences of the gradient) in place of the variable metric
    if (F.n_iter > 0 && F.n_iter % kRefresh == 0 && F.refreshed != F.n_iter && F.edm >= o.tol_edm &&
        F.n_iter < o.max_iter) {
      F.refreshed = F.n_iter;
      F.post_hessian();
      F.phase = kHessInit;
      return;
    }
    if (F.edm >= o.tol_edm && F.n_iter > 0 && F.last_step < o.tol_step_rel && F.stalls < kMaxStalls &&
        F.n_iter < o.max_iter) {
      // steps below the tolerance while the EDM is not: the variable metric
      // has lost the valley's curvature; restart from a differenced Hessian
      F.stalls++;
      F.refreshed = F.n_iter;
      F.last_step = 1e300;
      F.post_hessian();
      F.phase = kHessInit;
      return;
    }
    if (F.edm < o.tol_edm || (F.n_iter > 0 && F.last_step < o.tol_step_rel) || F.n_iter >= o.max_iter) {
      if (F.n_iter >= o.max_iter && F.edm >= o.tol_edm) F.status = 1;
      if (o.polish) {
        F.post_hessian();
        F.phase = kHessPolish;
      } else {
        F.finish(o.tol_edm);
      }
      return;
    }
    F.alpha = 1.0;
    F.tries = 0;
    F.post_line();
    F.phase = kLine;
  }

  // A polish that ends (no lower point, or an indefinite Hessian) while the
  // EDM from the differenced Hessian is still above the tolerance: back to
  // variable-metric steps with that Hessian's inverse as the metric, at most
  // kMaxStalls times.  Returns true when the fit goes on iterating.
  bool polish_stalled(Fit &F) {
    const int n = F.n;
    F.edm = 0.0;
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) F.edm += 0.5 * F.g[i] * F.V[i * n + k] * F.g[k];
    if (!(F.edm >= o.tol_edm) || F.stalls >= kMaxStalls || F.n_fcn >= o.max_fcn || F.n_iter >= o.max_iter)
      return false;
    F.stalls++;
    F.status = 0;
    F.last_step = 1e300;
    F.phase = kIter;
    return true;
  }

  void post_newton(Fit &F) {
    const int n = F.n;
    std::vector<double> L = F.H;
    F.xt = F.x;
    if (!cholesky(L, n)) {  // no Newton step from an indefinite Hessian
      if (polish_stalled(F)) {
        F.alpha = 1.0;
        F.tries = 0;
        F.direction();
        F.post_line();
        F.phase = kLine;
        return;
      }
      F.finish(o.tol_edm);
      return;
    }
    std::vector<double> Hi = spd_inverse(L, n);
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s -= Hi[i * n + k] * F.g[k];
      F.xt[i] = F.x[i] + s;
    }
    F.post(F.xt, true);
  }
};

}  // namespace mu

extern "C" mu_status mu_fit_batch(mu_ctx *ctx, int32_t n_fits, const mu_data *const *data,
                                  const mu_theory *const *th, mu_cost cost_kind, int32_t ld, const double *start,
                                  const mu_fit_opts *opts, double *params_out, double *cov_out,
                                  mu_fit_result *res) {
  if (!ctx) return MU_E_ARG;
  if (n_fits < 1 || !data || !th || !start || !params_out || !res || ld < 1) {
    set_err(ctx, "mu_fit_batch needs n_fits >= 1, ld >= 1, data, theories, start, params_out and res");
    return MU_E_ARG;
  }
  if (cost_kind != MU_COST_CHI2 && cost_kind != MU_COST_POISSON) {
    set_err(ctx, "unknown cost kind %d", (int)cost_kind);
    return MU_E_ARG;
  }
  for (int f = 0; f < n_fits; ++f) {
    mu_status st = check_pair(ctx, data[f], th[f]);
    if (st != MU_OK) return st;
    if (th[f]->h.n_par > ld) {
      set_err(ctx, "fit %d: theory has %d parameters but ld is %d", f, th[f]->h.n_par, ld);
      return MU_E_ARG;
    }
    for (int k = 0; k < th[f]->h.n_par; ++k)
      if (!std::isfinite(start[(size_t)f * ld + k])) {
        set_err(ctx, "fit %d: start parameter %d is not finite", f, k);
        return MU_E_ARG;
      }
  }
  FitDriver D;
  D.ctx = ctx;
  D.n_fits = n_fits;
  D.ld = ld;
  D.data = data;
  D.th = th;
  D.cost_kind = cost_kind;
  std::memset(&D.o, 0, sizeof D.o);
  if (opts) D.o = *opts;
  if (D.o.max_fcn <= 0) D.o.max_fcn = 100000;
  if (D.o.max_iter <= 0) D.o.max_iter = 1000;
  if (!(D.o.tol_edm > 0.0)) D.o.tol_edm = 1e-8;
  if (!(D.o.tol_step_rel > 0.0)) D.o.tol_step_rel = 1e-7;
  std::vector<Fit> fits(n_fits);
  D.fit_data.assign(data, data + n_fits);
  D.fit_theory.assign(th, th + n_fits);
  for (int f = 0; f < n_fits; ++f) {
    Fit &F = fits[f];
    F.id = f;
    F.ld = ld;
    F.base.assign(start + (size_t)f * ld, start + (size_t)(f + 1) * ld);
    const int np = th[f]->h.n_par;
    for (int k = 0; k < np; ++k)
      if (!(D.o.fixed && D.o.fixed[(size_t)f * ld + k])) F.fi.push_back(k);
    F.n = (int)F.fi.size();
    F.x.resize(F.n);
    for (int k = 0; k < F.n; ++k) F.x[k] = F.base[F.fi[k]];
    if (F.n == 0) {
      F.phase = kDone;
      continue;
    }
    F.post(F.x, true);
  }
  mu_status st = MU_OK;
  if (D.o.batched) {
    // every round: one batched launch with the posts of all active fits
    for (;;) {
      std::vector<Fit *> active;
      for (Fit &F : fits)
        if (F.phase != kDone && !F.posts.empty()) active.push_back(&F);
      if (active.empty()) break;
      if ((st = D.evaluate(active, false)) != MU_OK) break;
      for (Fit *F : active) D.advance(*F);
    }
  } else {
    // plain path: one fit at a time, one launch per evaluated point
    for (Fit &F : fits) {
      while (F.phase != kDone && !F.posts.empty()) {
        std::vector<Fit *> one{&F};
        if ((st = D.evaluate(one, true)) != MU_OK) break;
        D.advance(F);
      }
      if (st != MU_OK) break;
    }
  }
  if (st != MU_OK) return st;
  for (int f = 0; f < n_fits; ++f) {
    Fit &F = fits[f];
    std::vector<double> p = F.full(F.x);
    std::memcpy(params_out + (size_t)f * ld, p.data(), ld * sizeof(double));
    if (cov_out) {
      double *C = cov_out + (size_t)f * ld * ld;
      std::memset(C, 0, (size_t)ld * ld * sizeof(double));
      if (!F.V.empty())
        for (int i = 0; i < F.n; ++i)
          for (int k = 0; k < F.n; ++k) C[(size_t)F.fi[i] * ld + F.fi[k]] = 2.0 * F.V[i * F.n + k];
    }
    res[f].cost = F.f;
    res[f].edm = F.edm;
    res[f].n_iter = F.n_iter;
    res[f].n_fcn = F.n_fcn;
    res[f].n_grad = F.n_grad;
    res[f].status = F.status;
  }
  return MU_OK;
}
