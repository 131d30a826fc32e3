// Parameter errors after the minimum: the Hessian-based covariance (HESSE's
// role) and likelihood-profile errors (MINOS's role).  The paper's fits end
// with Minuit2's minimisation (Sec. 4, Table 1); both costs are -2 ln L up to
// a constant (Eqs. 2-3), so the covariance is 2 H^-1 and a rise of `up` = 1 in
// the profiled cost marks one standard deviation.
//
//   mu_hesse:   H from the Gauss-Newton sum over bins (Jacobian-mode
//               evaluation, then the FP64 MFMA Gram kernel per histogram and
//               the chain rule through the map / function array on the
//               host), or from central differences of the analytic gradient
//               (2n gradient vectors in one launch).
//   mu_profile: the cost minimised over the other free parameters at given
//               values of one parameter, all points as one batched fit.
//   mu_minos:   the two profile crossings of cost_min + up, both sides
//               refined together, one batched fit per round.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mu_internal.h"
#include "mu_runtime.h"

using namespace mu;

namespace {

bool chol(std::vector<double> &A, int n) {
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

std::vector<double> chol_inverse(const std::vector<double> &L, int n) {
  std::vector<double> inv(n * n, 0.0), col(n);
  for (int c = 0; c < n; ++c) {
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

// dR_r / dp for resolved scalar r of map row `row`: a sparse list (k, value).
void ref_jac(const mu_theory *th, int r, int row, std::vector<std::pair<int, double>> &out) {
  out.clear();
  const DevRef &ref = th->h.rref[r];
  if (ref.kind == MU_REF_PAR) {
    out.push_back({th->map[(size_t)row * th->h.n_slots + ref.slot], 1.0});
  } else if (ref.kind == MU_REF_FUN) {
    const int i = th->map[(size_t)row * th->h.n_slots + ref.slot];
    for (int k = 0; k < th->h.n_par; ++k)
      if (th->F[(size_t)i * th->h.n_par + k] != 0.0) out.push_back({k, th->F[(size_t)i * th->h.n_par + k]});
  }
}

// Gauss-Newton Hessian in p of one parameter vector (device work, host result).
mu_status gauss_newton(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *params,
                       std::vector<double> &H) {
  const int n_par = th->h.n_par;
  mu_status st;
  hipError_t e;
  // Jacobian rows: one per fit-range bin
  const size_t jac_bytes = (size_t)d->total * kJacCols * sizeof(double);
  if ((st = ctx->jac.ensure(ctx, jac_bytes, false)) != MU_OK) return st;
  if ((st = ctx->dparams.ensure(ctx, n_par * sizeof(double), false)) != MU_OK) return st;
  // Gram units: contiguous row ranges of one histogram
  constexpr int64_t kRowsPerUnit = 512;
  std::vector<int64_t> units;
  std::vector<int32_t> ufirst(d->n_histo + 1, 0);
  for (int h = 0; h < d->n_histo; ++h) {
    ufirst[h] = (int32_t)(units.size() / 3);
    const int64_t r0 = d->hh[h].off, r1 = r0 + d->hh[h].n;
    for (int64_t r = r0; r < r1; r += kRowsPerUnit) {
      units.push_back(h);
      units.push_back(r);
      units.push_back(std::min(r + kRowsPerUnit, r1));
    }
  }
  const int n_units = (int)(units.size() / 3);
  ufirst[d->n_histo] = n_units;
  const size_t part_bytes = (size_t)n_units * 16 * 64 * sizeof(double);
  const size_t hr_bytes = (size_t)d->n_histo * kJacCols * kJacCols * sizeof(double);
  const size_t meta_bytes = units.size() * sizeof(int64_t) + ufirst.size() * sizeof(int32_t);
  if ((st = ctx->gram.ensure(ctx, part_bytes + hr_bytes + meta_bytes + 256, false)) != MU_OK) return st;
  char *g = static_cast<char *>(ctx->gram.ptr);
  double *part = reinterpret_cast<double *>(g);
  double *HR = reinterpret_cast<double *>(g + part_bytes);
  int64_t *d_units = reinterpret_cast<int64_t *>(g + part_bytes + hr_bytes);
  int32_t *d_ufirst = reinterpret_cast<int32_t *>(g + part_bytes + hr_bytes + units.size() * sizeof(int64_t));
  e = hipMemcpyAsync(ctx->dparams.ptr, params, n_par * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_units, units.data(), units.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_ufirst, ufirst.data(), ufirst.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(hesse inputs)");
  // the evaluation kernel in Jacobian mode: one vector, the split launch
  const int shape = ctx->specialize ? th->shape : kShapeGeneric;
  int anchor = ctx->anchor_every;
  const int64_t W = ctx->pick_split(shape, kModeCost, cost_kind, d->f64, d->total, &anchor);
  LaunchArgs a;
  std::memset(&a, 0, sizeof a);
  a.tmpl.th = th->d_th;
  a.tmpl.histos = d->d_hh;
  a.tmpl.counts = d->counts;
  a.tmpl.p = static_cast<const double *>(ctx->dparams.ptr);
  a.tmpl.model_out = static_cast<double *>(ctx->jac.ptr);
  a.tmpl.n_histo = d->n_histo;
  a.tmpl.shape = shape;
  a.p_stride = n_par;
  a.n_units = (int32_t)((d->total + W - 1) / W);
  a.cost_kind = cost_kind;
  a.anchor_every = anchor;
  a.counts_in_table = !d->f64 && d->max_count < kInvTab;
  a.inv_src = ctx->d_inv;
  a.n_vec = 1;
  a.split_w = W;
  a.total = d->total;
  e = th->rtc_fn ? launch_rtc(th->rtc_fn, a, kModeJac, d->f64, ctx->stream) : launch_jac(a, d->f64, shape, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "Jacobian launch");
  e = launch_gram(static_cast<const double *>(ctx->jac.ptr), d_units, n_units, part, d_ufirst, d->n_histo, HR,
                  ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "Gram launch");
  std::vector<double> hr((size_t)d->n_histo * kJacCols * kJacCols);
  e = hipMemcpyAsync(hr.data(), HR, hr.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "Gram read-back");
  // chain rule: H_p = sum_h D_h^T HR_h D_h with D_h[r][k] = dR_r/dp_k
  H.assign((size_t)n_par * n_par, 0.0);
  std::vector<std::pair<int, double>> jr, js;
  for (int h = 0; h < d->n_histo; ++h) {
    const double *B = hr.data() + (size_t)h * kJacCols * kJacCols;
    const int row = d->hh[h].map_row;
    for (int r = 0; r < kRS; ++r) {
      ref_jac(th, r, row, jr);
      if (jr.empty()) continue;
      for (int s = 0; s < kRS; ++s) {
        const double b = B[r * kJacCols + s];
        if (b == 0.0) continue;
        ref_jac(th, s, row, js);
        for (const auto &x : jr)
          for (const auto &y : js) H[(size_t)x.first * n_par + y.first] += x.second * b * y.second;
      }
    }
  }
  return MU_OK;
}

// Hessian by central differences of the analytic gradient: the 2n points in
// one gradient launch; columns of fixed parameters stay zero.
mu_status diff_hessian(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *params,
                       const std::vector<int> &free, std::vector<double> &H) {
  const int n_par = th->h.n_par, nf = (int)free.size();
  std::vector<double> P((size_t)2 * nf * n_par), c(2 * nf), g((size_t)2 * nf * n_par), hs(nf);
  for (int q = 0; q < nf; ++q) {
    const int k = free[q];
    hs[q] = 1e-5 * std::max(std::fabs(params[k]), 1e-3);
    for (int sg = 0; sg < 2; ++sg) {
      double *row = &P[(size_t)(2 * q + sg) * n_par];
      std::memcpy(row, params, n_par * sizeof(double));
      row[k] += sg == 0 ? hs[q] : -hs[q];
    }
  }
  mu_status st = eval_uniform(ctx, d, th, cost_kind, P.data(), 2 * nf, MU_MEM_HOST, c.data(), nullptr, g.data(),
                              nullptr, kModeGrad);
  if (st != MU_OK) return st;
  H.assign((size_t)n_par * n_par, 0.0);
  for (int q = 0; q < nf; ++q)
    for (int i = 0; i < nf; ++i) {
      const int k = free[q], m = free[i];
      H[(size_t)m * n_par + k] = (g[(size_t)(2 * q) * n_par + m] - g[(size_t)(2 * q + 1) * n_par + m]) / (2.0 * hs[q]);
    }
  for (int i = 0; i < n_par; ++i)
    for (int k = 0; k < i; ++k) {
      const double s = 0.5 * (H[(size_t)i * n_par + k] + H[(size_t)k * n_par + i]);
      H[(size_t)i * n_par + k] = H[(size_t)k * n_par + i] = s;
    }
  return MU_OK;
}

}  // namespace

extern "C" mu_status mu_hesse(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                              int32_t method, const double *params, const uint8_t *fixed, double *hess, double *cov,
                              int32_t *pos_def) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (!params || !hess || (cost_kind != MU_COST_CHI2 && cost_kind != MU_COST_POISSON) ||
      (method != MU_HESSE_GAUSS_NEWTON && method != MU_HESSE_DIFF)) {
    set_err(ctx, "mu_hesse needs parameters, a Hessian output, a cost kind and a method");
    return MU_E_ARG;
  }
  const int n_par = th->h.n_par;
  for (int k = 0; k < n_par; ++k)
    if (!std::isfinite(params[k])) {
      set_err(ctx, "parameter %d is not finite", k);
      return MU_E_ARG;
    }
  (void)hipSetDevice(ctx->device);
  std::vector<int> free;
  for (int k = 0; k < n_par; ++k)
    if (!(fixed && fixed[k])) free.push_back(k);
  std::vector<double> H;
  mu_data *d = const_cast<mu_data *>(data);
  st = method == MU_HESSE_GAUSS_NEWTON ? gauss_newton(ctx, d, th, cost_kind, params, H)
                                       : diff_hessian(ctx, d, th, cost_kind, params, free, H);
  if (st != MU_OK) return st;
  // fixed parameters: zero rows and columns
  for (int k = 0; k < n_par; ++k)
    if (fixed && fixed[k])
      for (int i = 0; i < n_par; ++i) H[(size_t)k * n_par + i] = H[(size_t)i * n_par + k] = 0.0;
  const int nf = (int)free.size();
  std::vector<double> L((size_t)nf * nf);
  for (int i = 0; i < nf; ++i)
    for (int k = 0; k < nf; ++k) L[(size_t)i * nf + k] = H[(size_t)free[i] * n_par + free[k]];
  const bool pd = nf > 0 && chol(L, nf);
  std::memcpy(hess, H.data(), H.size() * sizeof(double));
  if (pos_def) *pos_def = pd ? 1 : 0;
  if (cov) {
    std::fill(cov, cov + (size_t)n_par * n_par, pd ? 0.0 : NAN);
    if (pd) {
      const std::vector<double> inv = chol_inverse(L, nf);
      for (int i = 0; i < nf; ++i)
        for (int k = 0; k < nf; ++k) cov[(size_t)free[i] * n_par + free[k]] = 2.0 * inv[(size_t)i * nf + k];
    }
  }
  return MU_OK;
}

extern "C" mu_status mu_profile(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                                const double *p_min, const uint8_t *fixed, int32_t k, int32_t n_points,
                                const double *values, double *prof_cost, double *prof_params,
                                int32_t *status) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  const int n_par = th->h.n_par;
  if (!p_min || !values || !prof_cost || n_points < 1 || k < 0 || k >= n_par) {
    set_err(ctx, "mu_profile needs p_min, values, outputs, n_points >= 1 and 0 <= k < n_par");
    return MU_E_ARG;
  }
  // start each point at the minimum moved along the parameter's correlations
  // (the Gauss-Newton covariance), so the constrained fits start close
  std::vector<uint8_t> fx((size_t)n_points * n_par, 0);
  std::vector<double> start((size_t)n_points * n_par), out((size_t)n_points * n_par), hess((size_t)n_par * n_par),
      cov((size_t)n_par * n_par);
  for (int q = 0; q < n_points; ++q)
    for (int i = 0; i < n_par; ++i) fx[(size_t)q * n_par + i] = (fixed && fixed[i]) || i == k;
  int32_t pd = 0;
  st = mu_hesse(ctx, data, th, cost_kind, MU_HESSE_GAUSS_NEWTON, p_min, fixed, hess.data(), cov.data(), &pd);
  if (st != MU_OK) return st;
  const double ckk = cov[(size_t)k * n_par + k];
  for (int q = 0; q < n_points; ++q) {
    double *s = &start[(size_t)q * n_par];
    for (int i = 0; i < n_par; ++i) {
      double shift = 0.0;
      if (pd && ckk > 0.0 && !fx[(size_t)q * n_par + i]) shift = cov[(size_t)i * n_par + k] / ckk * (values[q] - p_min[k]);
      s[i] = p_min[i] + shift;
    }
    s[k] = values[q];
  }
  std::vector<const mu_data *> dv(n_points, data);
  std::vector<const mu_theory *> tv(n_points, th);
  mu_fit_opts o;
  std::memset(&o, 0, sizeof o);
  o.analytic_grad = 1;
  o.batched = 1;
  o.polish = 1;
  o.fixed = fx.data();
  std::vector<mu_fit_result> res(n_points);
  st = mu_fit_batch(ctx, n_points, dv.data(), tv.data(), cost_kind, n_par, start.data(), &o, out.data(), nullptr,
                    res.data());
  if (st != MU_OK) return st;
  for (int q = 0; q < n_points; ++q) {
    prof_cost[q] = res[q].cost;
    if (status) status[q] = res[q].status;
  }
  if (prof_params) std::memcpy(prof_params, out.data(), out.size() * sizeof(double));
  return MU_OK;
}

extern "C" mu_status mu_minos(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                              const double *p_min, const uint8_t *fixed, int32_t k, double up, double *err_lo,
                              double *err_hi, int32_t *n_rounds) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  const int n_par = th->h.n_par;
  if (!p_min || !err_lo || !err_hi || k < 0 || k >= n_par || (fixed && fixed[k]) || !(up > 0.0)) {
    set_err(ctx, "mu_minos needs p_min, outputs, a free parameter k and up > 0");
    return MU_E_ARG;
  }
  std::vector<double> hess((size_t)n_par * n_par), cov((size_t)n_par * n_par);
  int32_t pd = 0;
  st = mu_hesse(ctx, data, th, cost_kind, MU_HESSE_GAUSS_NEWTON, p_min, fixed, hess.data(), cov.data(), &pd);
  if (st != MU_OK) return st;
  double f0 = 0.0;
  st = eval_uniform(ctx, const_cast<mu_data *>(data), th, cost_kind, p_min, 1, MU_MEM_HOST, &f0, nullptr, nullptr,
                    nullptr, kModeCost);
  if (st != MU_OK) return st;
  const double sig = pd ? std::sqrt(cov[(size_t)k * n_par + k] * up) : 1e-3 * std::max(std::fabs(p_min[k]), 1.0);
  // per side: a bracket [a, b] of offsets (excess(a) < 0 <= excess(b)) and a
  // current trial; regula falsi on the profile excess, both sides in one fit
  // call per round (excess(0) = -up at the minimum)
  double a[2] = {0.0, 0.0}, fa[2] = {-up, -up}, b[2] = {-sig, sig}, fb[2] = {NAN, NAN}, x[2] = {-sig, sig};
  bool done[2] = {false, false}, bracketed[2] = {false, false};
  int rounds = 0;
  for (; rounds < 60 && !(done[0] && done[1]); ++rounds) {
    double vals[2], pc[2];
    int32_t pst[2];
    int nv = 0, side[2];
    for (int s = 0; s < 2; ++s)
      if (!done[s]) {
        side[nv] = s;
        vals[nv++] = p_min[k] + x[s];
      }
    st = mu_profile(ctx, data, th, cost_kind, p_min, fixed, k, nv, vals, pc, nullptr, pst);
    if (st != MU_OK) return st;
    for (int q = 0; q < nv; ++q) {
      const int s = side[q];
      const double fx = pc[q] - f0 - up;
      if (!bracketed[s]) {
        if (fx >= 0.0) {
          b[s] = x[s];
          fb[s] = fx;
          bracketed[s] = true;
        } else {  // not far enough yet: keep the point, double the offset
          a[s] = x[s];
          fa[s] = fx;
          x[s] *= 2.0;
          continue;
        }
      } else if (fx < 0.0) {
        a[s] = x[s];
        fa[s] = fx;
      } else {
        b[s] = x[s];
        fb[s] = fx;
      }
      if (std::fabs(fx) <= 1e-9 * up || std::fabs(b[s] - a[s]) <= 1e-12 * sig) {
        done[s] = true;
        continue;
      }
      // the profile is close to a parabola near the crossing: interpolate in
      // the squared offset, kept inside the bracket
      const double qa = a[s] * a[s], qb = b[s] * b[s];
      double qx = qa + (qb - qa) * (0.0 - fa[s]) / (fb[s] - fa[s]);
      double nx = (s == 0 ? -1.0 : 1.0) * std::sqrt(std::max(qx, 0.0));
      const double lo = std::min(a[s], b[s]), hi = std::max(a[s], b[s]);
      if (!(nx > lo && nx < hi)) nx = 0.5 * (a[s] + b[s]);
      x[s] = nx;
    }
  }
  if (!(done[0] && done[1])) {
    set_err(ctx, "mu_minos: a crossing was not found within %d rounds", rounds);
    return MU_E_STATE;
  }
  *err_lo = std::fabs(fa[0]) < std::fabs(fb[0]) ? a[0] : b[0];
  *err_hi = std::fabs(fa[1]) < std::fabs(fb[1]) ? a[1] : b[1];
  if (n_rounds) *n_rounds = rounds;
  return MU_OK;
}
