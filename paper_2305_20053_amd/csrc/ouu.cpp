// Outer OUU solve (paper Sec. 2.1, eq. (ouu) / (CVaR_ouu); Sec. 4.2 solves it
// with a bound-constrained limited-memory BFGS over the box Z_ad).
//
// Bound-constrained limited-memory BFGS on the host, every objective and
// gradient from saa_objective_grad (PDE or MR-DINO form on the device):
//  * the variables at a bound whose gradient points out of the box are held
//    there for the iteration (active set); the quasi-Newton direction is the
//    two-loop recursion over the free variables only, with the stored pairs
//    restricted to them;
//  * the step is searched along the projection of the ray onto the box,
//    backtracking (safeguarded quadratic interpolation) to the Armijo
//    condition measured with the projected step;
//  * a failed search drops the stored pairs and retries from steepest descent;
//  * stop when the projected gradient |P(x - g) - x|_inf <= pgtol, or when an
//    accepted step lowers J by at most ftol max(|J|, 1).
// With joint_t the variable is (z, t) and every evaluation is J_hat(z, t)
// with t_mode = 1 (t free, unbounded); otherwise t is minimised out inside
// each evaluation (t_mode = 0).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/saa.h"

namespace {

struct Eval {
  saa_ctx* ctx;
  int form;
  const void* model;
  saa_options opt;
  int dz;
  bool joint;
  int count = 0, fallbacks = 0;
  double t_last = 0.0;
  // x: z (and t when joint) -> f, g; returns a status code
  int operator()(const std::vector<double>& x, double& f, std::vector<double>& g) {
    saa_options o = opt;
    if (joint) {
      o.t_mode = 1;
      o.t_in = x[dz];
    }
    saa_report rep;
    const int st = saa_objective_grad(ctx, x.data(), form, model, &o, &f, g.data(), &rep);
    ++count;
    if (st == SAA_W_FALLBACK) ++fallbacks;
    if (st != SAA_OK && st != SAA_W_FALLBACK) return st;
    if (joint) g[dz] = rep.dJ_dt;
    t_last = rep.t_star;
    return SAA_OK;
  }
};

double dot(const std::vector<double>& a, const std::vector<double>& b, const std::vector<char>& fr) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i)
    if (fr[i]) s += a[i] * b[i];
  return s;
}

}  // namespace

extern "C" {

int saa_ouu_options_default(saa_ouu_options* oo) {
  if (!oo) return SAA_E_INVALID;
  oo->max_iter = 200;
  oo->max_eval = 1000;
  oo->memory = 10;
  oo->joint_t = 0;
  oo->pgtol = 1e-6;
  oo->ftol = 1e-12;
  return SAA_OK;
}

int saa_ouu_solve(saa_ctx* ctx, int form, const void* model, const saa_options* opt, const saa_ouu_options* oo_in,
                  const double* lb, const double* ub, double* z, saa_ouu_report* rep) {
  if (!ctx || !opt || !z || !rep) return SAA_E_INVALID;
  saa_ouu_options oo;
  saa_ouu_options_default(&oo);
  if (oo_in) oo = *oo_in;
  if (oo.max_iter < 0 || oo.max_eval < 1 || oo.memory < 1 || oo.memory > 100 || !(oo.pgtol >= 0.0) ||
      !(oo.ftol >= 0.0) || (oo.joint_t != 0 && oo.joint_t != 1))
    return SAA_E_INVALID;
  if (oo.joint_t && opt->t_mode != 0) return SAA_E_INVALID;
  int64_t du_ = 0;
  int dz = 0, nkl_ = 0;
  int rc = saa_ctx_dims(ctx, &du_, &dz, &nkl_);
  if (rc) return rc;
  const bool joint = oo.joint_t == 1;
  const int nv = dz + (joint ? 1 : 0);
  std::vector<double> lo(nv, -INFINITY), hi(nv, INFINITY);
  for (int k = 0; k < dz; ++k) {
    if (lb) lo[k] = lb[k];
    if (ub) hi[k] = ub[k];
    if (std::isnan(lo[k]) || std::isnan(hi[k]) || lo[k] > hi[k] || !std::isfinite(z[k])) return SAA_E_INVALID;
  }
  const auto t0 = std::chrono::steady_clock::now();
  *rep = saa_ouu_report{};
  Eval ev{ctx, form, model, *opt, dz, joint};
  auto proj = [&](std::vector<double>& x) {
    for (int i = 0; i < nv; ++i) x[i] = std::min(hi[i], std::max(lo[i], x[i]));
  };
  std::vector<double> x(nv), g(nv), xn(nv), gn(nv), d(nv);
  for (int k = 0; k < dz; ++k) x[k] = z[k];
  proj(x);
  double f = 0.0;
  if (joint) {   // start t at the minimiser of J_hat(z0, .)
    saa_report r0;
    double f0;
    saa_options o = *opt;
    o.t_mode = 0;
    rc = saa_objective_grad(ctx, x.data(), form, model, &o, &f0, g.data(), &r0);
    ++ev.count;
    if (rc != SAA_OK && rc != SAA_W_FALLBACK) return rc;
    x[dz] = r0.t_star;
  }
  if ((rc = ev(x, f, g))) return rc;

  auto pg_norm = [&](const std::vector<double>& xx, const std::vector<double>& gg) {
    double m = 0.0;
    for (int i = 0; i < nv; ++i) m = std::max(m, std::fabs(std::min(hi[i], std::max(lo[i], xx[i] - gg[i])) - xx[i]));
    return m;
  };
  std::vector<std::vector<double>> S, Y;   // oldest first
  int status = SAA_OUU_MAXITER, it = 0, err = SAA_OK;
  std::vector<char> fr(nv);
  for (it = 0; it < oo.max_iter; ++it) {
    if (pg_norm(x, g) <= oo.pgtol) {
      status = SAA_OUU_PGTOL;
      break;
    }
    // active set: at a bound with the gradient pointing outwards
    for (int i = 0; i < nv; ++i)
      fr[i] = !((x[i] <= lo[i] && g[i] > 0.0) || (x[i] >= hi[i] && g[i] < 0.0));
    // two-loop recursion over the free variables
    std::vector<double> q(nv, 0.0);
    for (int i = 0; i < nv; ++i) q[i] = fr[i] ? g[i] : 0.0;
    const int m = (int)S.size();
    std::vector<double> al(m, 0.0), rho(m, 0.0);
    double gamma = 0.0;
    for (int j = m - 1; j >= 0; --j) {
      const double sy = dot(S[j], Y[j], fr);
      if (!(sy > 0.0)) continue;
      rho[j] = 1.0 / sy;
      if (gamma == 0.0) gamma = sy / dot(Y[j], Y[j], fr);
      al[j] = rho[j] * dot(S[j], q, fr);
      for (int i = 0; i < nv; ++i)
        if (fr[i]) q[i] -= al[j] * Y[j][i];
    }
    if (gamma == 0.0) {   // no usable pair: a steepest-descent step of unit max-norm
      double gm = 0.0;
      for (int i = 0; i < nv; ++i)
        if (fr[i]) gm = std::max(gm, std::fabs(g[i]));
      gamma = gm > 0.0 ? 1.0 / gm : 1.0;
    }
    for (int i = 0; i < nv; ++i) q[i] *= gamma;
    for (int j = 0; j < m; ++j) {
      if (rho[j] == 0.0) continue;
      const double b = rho[j] * dot(Y[j], q, fr);
      for (int i = 0; i < nv; ++i)
        if (fr[i]) q[i] += S[j][i] * (al[j] - b);
    }
    double gd = 0.0;
    for (int i = 0; i < nv; ++i) {
      d[i] = fr[i] ? -q[i] : 0.0;
      gd += g[i] * d[i];
    }
    if (!(gd < 0.0)) {   // not a descent direction: drop the memory, steepest descent
      S.clear();
      Y.clear();
      double gm = 0.0;
      for (int i = 0; i < nv; ++i)
        if (fr[i]) gm = std::max(gm, std::fabs(g[i]));
      for (int i = 0; i < nv; ++i) d[i] = fr[i] ? -g[i] / (gm > 0.0 ? gm : 1.0) : 0.0;
    }
    // projected backtracking line search (Armijo with the projected step)
    double a = 1.0, fn = 0.0;
    bool accepted = false;
    for (int ls = 0; ls < 40; ++ls) {
      if (ev.count >= oo.max_eval) break;
      for (int i = 0; i < nv; ++i) xn[i] = x[i] + a * d[i];
      proj(xn);
      double slope = 0.0;   // g . (xn - x)
      for (int i = 0; i < nv; ++i) slope += g[i] * (xn[i] - x[i]);
      if (!(slope < 0.0)) break;   // the projected step no longer descends
      if ((err = ev(xn, fn, gn))) break;
      if (std::isfinite(fn) && fn <= f + 1e-4 * slope) {
        accepted = true;
        break;
      }
      // quadratic model along the projected path, safeguarded to [0.1 a, 0.5 a]
      double an = 0.5 * a;
      const double curv = std::isfinite(fn) ? fn - f - slope : INFINITY;
      if (curv > 0.0 && std::isfinite(curv)) an = std::min(0.5 * a, std::max(0.1 * a, -0.5 * slope * a / curv));
      else an = 0.1 * a;
      a = an;
    }
    if (err) break;
    if (!accepted && !S.empty() && ev.count < oo.max_eval) {   // retry once from steepest descent
      S.clear();
      Y.clear();
      --it;
      continue;
    }
    if (!accepted) {
      status = ev.count >= oo.max_eval ? SAA_OUU_MAXEVAL : SAA_OUU_LINESEARCH;
      break;
    }
    std::vector<double> s(nv), y(nv);
    double sy = 0.0, yy = 0.0;
    for (int i = 0; i < nv; ++i) {
      s[i] = xn[i] - x[i];
      y[i] = gn[i] - g[i];
      sy += s[i] * y[i];
      yy += y[i] * y[i];
    }
    if (sy > 2.2e-16 * yy) {   // keep only pairs with positive curvature
      S.push_back(s);
      Y.push_back(y);
      if ((int)S.size() > oo.memory) {
        S.erase(S.begin());
        Y.erase(Y.begin());
      }
    }
    const double drop = f - fn;
    x.swap(xn);
    g.swap(gn);
    f = fn;
    if (drop <= oo.ftol * std::max(std::fabs(f), 1.0)) {
      status = SAA_OUU_FTOL;
      ++it;
      break;
    }
    if (ev.count >= oo.max_eval) {
      status = SAA_OUU_MAXEVAL;
      ++it;
      break;
    }
  }
  for (int k = 0; k < dz; ++k) z[k] = x[k];
  rep->J = f;
  rep->pg_norm = pg_norm(x, g);
  rep->t = joint ? x[dz] : ev.t_last;
  rep->iterations = it;
  rep->evaluations = ev.count;
  rep->status = status;
  int na = 0;
  for (int k = 0; k < dz; ++k) na += (x[k] <= lo[k] && g[k] > 0.0) || (x[k] >= hi[k] && g[k] < 0.0);
  rep->n_active = na;
  rep->n_fallback = ev.fallbacks;
  rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return err;
}

}  // extern "C"
