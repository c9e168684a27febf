// C ABI of the SAA engine: argument validation, context and workspace
// management, and the launch sequence of each entry point.  All numerical
// work runs in the HIP kernels of pde.hip / cvar.hip.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <array>
#include <new>
#include <vector>

#include "../../include/saa.h"
#include "pde.h"
#include "runtime.h"

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
namespace saa_launch {
void sine_table(double* S, int K1, int n, hipStream_t st);
void source_matrix(double* FT, int n, int s, double sigma, hipStream_t st);
void field(const double* xi, const double* S, const double* amp, double* em, int K1, int n, int64_t N,
           hipStream_t st);
template <typename TS>
void hierarchy(const PdeGeo& g, const double* em, double* kap, int64_t kstride, int64_t chunk,
               const MgBufs<TS>& b, int64_t N, hipStream_t st);
template <typename TW, typename TS>
void state(const PdeGeo& g, const double* FT, const double* Z, int64_t z_stride, const double* em, TW* u, TW* f,
           const MgBufs<TS>& b, const SolveParams& sp, double* q, int* newton, int* lin, int* flag, int64_t N,
           hipStream_t st);
template <typename TW, typename TS>
void adjoint(const PdeGeo& g, const double* FT, const double* em, const TW* u, TW* bvec, TW* lam,
             const MgBufs<TS>& b, const SolveParams& sp, const double* q, const double* tstar, int act,
             double act_w, double* gout, int* lin, int* flag, int* did, int64_t N, hipStream_t st);
template <typename TW, typename TS>
void linearized(const PdeGeo& g, const double* FT, const double* em, const TW* u, TW* bvec, TW* x,
                const MgBufs<TS>& b, const SolveParams& sp, double* dudz, int* lin, int* flag, int64_t N,
                hipStream_t st);
template <typename TW>
void interior_copy(const TW* u, double* out, int n, int64_t N, hipStream_t st);
template <typename TW, typename TS>
void adjoint_jac(const PdeGeo& g, const double* FT, const double* em, const TW* u, TW* bvec, TW* x,
                 const MgBufs<TS>& b, const SolveParams& sp, const double* MPhiT, int r_u, double* JY, int* lin,
                 int* flag, int64_t N, hipStream_t st);
void cvar(const double* q, const double* g, int64_t N, int dz, double beta, double eps, double alpha,
          const double* z, int t_mode, double t_in, int phase, double* tstar, double* out, const int* newton,
          const int* lin, const int* flag, const int* lin_adj, const int* did, void* stats, void* work,
          hipStream_t st);
size_t cvar_work_bytes();
void risk(const double* q, const double* g, int64_t N, int dz, int kind, double eps, double kappa, double tau,
          double alpha, const double* z, int phase, double* tstar, double* out, const int* newton, const int* lin,
          const int* flag, const int* lin_adj, const int* did, void* stats, void* work, hipStream_t st);
}  // namespace saa_launch

#include "ctx.h"
#include "model.h"

using namespace saa_rt;

namespace saa_rt {

// Tracking target: (M ut) at the interior nodes (node layout, 0 on the
// boundary) and ut^T M ut over all nodes, for the P1 mass of the
// triangulation with diagonals (i,j)-(i+1,j+1) (element matrices
// area / 12 [[2,1,1],[1,2,1],[1,1,2]]).
double target_value(int target, double u_target, double x, double y);
void target_mass(int n, int target, double u_target, std::vector<double>& mt, double& ctt) {
  const int np = n + 1;
  std::vector<double> ut((size_t)np * np);
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i <= n; ++i) ut[(size_t)j * np + i] = target_value(target, u_target, (double)i / n, (double)j / n);
  const double h2 = 1.0 / ((double)n * n);
  mt.assign((size_t)np * np, 0.0);
  for (int j = 1; j < n; ++j)
    for (int i = 1; i < n; ++i) {
      const size_t q = (size_t)j * np + i;
      mt[q] = (h2 / 12.0) *
              (6.0 * ut[q] + ut[q + 1] + ut[q - 1] + ut[q + np] + ut[q - np] + ut[q + np + 1] + ut[q - np - 1]);
    }
  double s = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const double a = ut[(size_t)j * np + i], b = ut[(size_t)j * np + i + 1], d = ut[(size_t)(j + 1) * np + i + 1],
                   e = ut[(size_t)(j + 1) * np + i];
      s += (a * a + b * b + d * d + (a + b + d) * (a + b + d)) + (a * a + d * d + e * e + (a + d + e) * (a + d + e));
    }
  ctt = s * (0.5 * h2 / 12.0);
}

// Target state at (x, y) (Sec. 4.2).
double target_value(int target, double u_target, double x, double y) {
  switch (target) {
    case SAA_TARGET_SIN: return std::sin(2.0 * M_PI * x) * std::sin(2.0 * M_PI * y);
    case SAA_TARGET_QUAD: return 4.0 * y * (1.0 - y);
    default: return u_target;
  }
}

}  // namespace saa_rt

namespace {

template <typename TS>
int alloc_mg(saa_ctx* c, MgStore<TS>& m) {
  if (m.allocated) return SAA_OK;
  const size_t ls = (size_t)c->N_max * c->geo.lstride * sizeof(TS);
  const size_t ns = (size_t)c->N_max * c->nodes * sizeof(TS);
  DevBuf* lv[] = {&m.WE, &m.WN, &m.KD, &m.D, &m.X, &m.B, &m.T};
  for (DevBuf* b : lv) {
    int rc = b->alloc_zero(ls, c->st);
    if (rc) return rc;
  }
  DevBuf* fv[] = {&m.cx, &m.cr, &m.cp, &m.cq};
  for (DevBuf* b : fv) {
    int rc = b->alloc_zero(ns, c->st);
    if (rc) return rc;
  }
  m.allocated = true;
  return SAA_OK;
}

template <typename TS>
int build_mg(saa_ctx* c, MgStore<TS>& m) {
  int rc = alloc_mg(c, m);
  if (rc) return rc;
  if (c->N == 0) return SAA_OK;
  if (!c->kap.p) {
    rc = c->kap.alloc((size_t)c->kchunk * c->kstride * sizeof(double));
    if (rc) return rc;
  }
  saa_launch::hierarchy<TS>(c->geo, (const double*)c->em.p, (double*)c->kap.p, c->kstride, c->kchunk, m.view(),
                            c->N, c->st);
  m.built = true;
  return check_hip(hipGetLastError());
}

SolveParams solve_params(const saa_options* o, bool fp32_state) {
  SolveParams sp;
  sp.newton_tol = o->newton_tol > 0 ? o->newton_tol : (fp32_state ? 1e-5 : 1e-13);
  sp.lin_rtol = o->lin_rtol > 0 ? o->lin_rtol : (fp32_state ? 1e-5 : 1e-6);
  // adjoint / linearised solves feed gradients and Jacobians only: 1e-11 is
  // two orders below the 1e-9 gradient target
  sp.adj_tol = fp32_state ? sp.newton_tol : std::fmax(sp.newton_tol, 1e-11);
  sp.max_newton = o->max_newton > 0 ? o->max_newton : 30;
  sp.max_lin = o->max_lin > 0 ? o->max_lin : 200;
  sp.max_dc = o->max_dc > 0 ? o->max_dc : 10;
  sp.nu = 1;
  return sp;
}

// The risk reduction of `opt` over (q, g): CVaR (t* search, eq. (CVaR_saa_ouu))
// or one of the expectation-type measures.  phase & 1: t (t*, the mean of q,
// tau or 0) -> tstar; phase & 2: J, dJ/dt, grad -> out.
void reduce(saa_ctx* c, const double* q, const double* g, const saa_options* opt, int phase, const int* newton,
            const int* lin, const int* flag, const int* lin_adj, const int* did, void* stats) {
  if (opt->risk == SAA_RISK_CVAR)
    saa_launch::cvar(q, g, c->N, c->dz, opt->beta, opt->eps, opt->alpha, (double*)c->zdev.p, opt->t_mode,
                     opt->t_in, phase, c->tstar(), c->out(), newton, lin, flag, lin_adj, did, stats, c->cwork.p,
                     c->st);
  else
    saa_launch::risk(q, g, c->N, c->dz, opt->risk, opt->eps, opt->risk_kappa, opt->risk_tau, opt->alpha,
                     (double*)c->zdev.p, phase, c->tstar(), c->out(), newton, lin, flag, lin_adj, did, stats,
                     c->cwork.p, c->st);
}

// Adjoint activity of the risk measure (see saa_k_adjoint).
int adjoint_act(const saa_options* opt) {
  if (opt->all_adjoints) return 1;
  switch (opt->risk) {
    case SAA_RISK_CVAR: return 0;
    case SAA_RISK_POF: return 2;
    case SAA_RISK_BPOE: return 3;
    default: return 1;
  }
}

// Width / threshold that goes with adjoint_act.
double adjoint_act_w(const saa_options* opt) {
  return opt->risk == SAA_RISK_BPOE ? opt->risk_tau : opt->eps;
}

int validate_options(const saa_options* o) {
  if (!o) return SAA_E_INVALID;
  if (!is_fin(o->beta) || o->beta < 0.0 || o->beta >= 1.0) return SAA_E_INVALID;
  if (!is_fin(o->eps) || o->eps <= 0.0) return SAA_E_INVALID;
  if (!is_fin(o->alpha) || o->alpha < 0.0) return SAA_E_INVALID;
  if (o->t_mode != 0 && o->t_mode != 1) return SAA_E_INVALID;
  if (o->t_mode == 1 && !is_fin(o->t_in)) return SAA_E_INVALID;
  if (o->prec < SAA_FP64 || o->prec > SAA_FP8) return SAA_E_INVALID;
  if (!is_fin(o->newton_tol) || !is_fin(o->lin_rtol)) return SAA_E_INVALID;
  if (o->risk < SAA_RISK_CVAR || o->risk > SAA_RISK_BPOE) return SAA_E_INVALID;
  if (o->risk != SAA_RISK_CVAR && o->t_mode != 0) return SAA_E_INVALID;
  if (!is_fin(o->risk_kappa) || o->risk_kappa < 0.0 || !is_fin(o->risk_tau)) return SAA_E_INVALID;
  if (o->jac_mode < SAA_JAC_AUTO || o->jac_mode > SAA_JAC_ADJOINT) return SAA_E_INVALID;
  return SAA_OK;
}

// Launch the state solve for the requested PDE precision.
int run_state(saa_ctx* c, int prec, const double* Z, int64_t z_stride, const SolveParams& sp) {
  int rc;
  if (!c->u.p) {  // PDE-form node vectors are allocated at first use
    const size_t tw = (size_t)c->N_max * c->nodes * sizeof(double);
    if ((rc = c->u.alloc_zero(tw, c->st)) || (rc = c->f.alloc_zero(tw, c->st)) ||
        (rc = c->lam.alloc_zero(tw, c->st)))
      return rc;
  }
  switch (prec) {
    case SAA_FP64:
      if (!c->mg64.built && (rc = build_mg(c, c->mg64))) return rc;
      saa_launch::state<double, double>(c->geo, (double*)c->FT.p, Z, z_stride, (double*)c->em.p, (double*)c->u.p,
                                        (double*)c->f.p, c->mg64.view(), sp, (double*)c->q.p, (int*)c->newton.p,
                                        (int*)c->lin.p, (int*)c->flag.p, c->N, c->st);
      break;
    case SAA_FP32_DC64:
      if (!c->mg32.built && (rc = build_mg(c, c->mg32))) return rc;
      saa_launch::state<double, float>(c->geo, (double*)c->FT.p, Z, z_stride, (double*)c->em.p, (double*)c->u.p,
                                       (double*)c->f.p, c->mg32.view(), sp, (double*)c->q.p, (int*)c->newton.p,
                                       (int*)c->lin.p, (int*)c->flag.p, c->N, c->st);
      break;
    case SAA_FP32:
      if (!c->mg32.built && (rc = build_mg(c, c->mg32))) return rc;
      saa_launch::state<float, float>(c->geo, (double*)c->FT.p, Z, z_stride, (double*)c->em.p, (float*)c->u.p,
                                      (float*)c->f.p, c->mg32.view(), sp, (double*)c->q.p, (int*)c->newton.p,
                                      (int*)c->lin.p, (int*)c->flag.p, c->N, c->st);
      break;
    default:
      return SAA_E_INVALID;
  }
  return check_hip(hipGetLastError());
}

int run_adjoint(saa_ctx* c, int prec, const SolveParams& sp, int act, double act_w, double* gout) {
  switch (prec) {
    case SAA_FP64:
      saa_launch::adjoint<double, double>(c->geo, (double*)c->FT.p, (double*)c->em.p, (double*)c->u.p,
                                          (double*)c->f.p, (double*)c->lam.p, c->mg64.view(), sp, (double*)c->q.p,
                                          c->tstar(), act, act_w, gout, (int*)c->lin_adj.p, (int*)c->flag.p,
                                          (int*)c->did.p, c->N, c->st);
      break;
    case SAA_FP32_DC64:
      saa_launch::adjoint<double, float>(c->geo, (double*)c->FT.p, (double*)c->em.p, (double*)c->u.p,
                                         (double*)c->f.p, (double*)c->lam.p, c->mg32.view(), sp, (double*)c->q.p,
                                         c->tstar(), act, act_w, gout, (int*)c->lin_adj.p, (int*)c->flag.p,
                                         (int*)c->did.p, c->N, c->st);
      break;
    case SAA_FP32:
      saa_launch::adjoint<float, float>(c->geo, (double*)c->FT.p, (double*)c->em.p, (float*)c->u.p,
                                        (float*)c->f.p, (float*)c->lam.p, c->mg32.view(), sp, (double*)c->q.p,
                                        c->tstar(), act, act_w, gout, (int*)c->lin_adj.p, (int*)c->flag.p,
                                        (int*)c->did.p, c->N, c->st);
      break;
    default:
      return SAA_E_INVALID;
  }
  return check_hip(hipGetLastError());
}

// Bring the result block to the host (one copy) and wait for the stream.
int fetch_results(saa_ctx* c) {
  int rc = check_hip(hipMemcpyAsync(c->hres.p, c->res.p, RES_BYTES, hipMemcpyDeviceToHost, c->st));
  if (!rc) rc = check_hip(hipStreamSynchronize(c->st));
  return rc;
}

// Report from the host copy of the result block (fetch_results first).
int fill_report(saa_ctx* c, saa_report* rep, double seconds, const PhaseTimer* tm) {
  CvarStats s;
  std::memcpy(&s, (const char*)c->hres.p + RES_STATS, sizeof(s));
  const double* h = (const double*)c->hres.p;
  const double t = h[RES_T], dJdt = h[1];
  if (rep) {
    rep->t_star = t;
    rep->dJ_dt = dJdt;
    rep->err_estimate = -1.0;
    rep->seconds = seconds;
    rep->newton_max = s.newton_max;
    rep->n_unconverged = s.n_unconverged;
    rep->n_adjoints = s.n_adjoints;
    rep->fallback_used = 0;
    rep->lin_total = s.lin_state + s.lin_adjoint;
    rep->newton_total = s.newton_total;
    rep->ms_state = rep->ms_adjoint = rep->ms_reduce = 0.0;
    rep->graph = 0;
    rep->pad = 0;
    if (tm) tm->ms(&rep->ms_state, &rep->ms_adjoint, &rep->ms_reduce);
  }
  return s.n_unconverged > 0 ? SAA_E_NOCONV : SAA_OK;
}

// Common validation of an objective / per-sample call.
int validate_call(saa_ctx* c, const double* z, int form, const void* model, const saa_options* opt) {
  int rc = validate_options(opt);
  if (rc) return rc;
  if (c->N < 1) return SAA_E_INVALID;
  for (int k = 0; k < c->dz; ++k)
    if (!is_fin(z[k])) return SAA_E_INVALID;
  if (form == SAA_FORM_PDE) {
    if (model != nullptr) return SAA_E_INVALID;
    if (opt->prec != SAA_FP64 && opt->prec != SAA_FP32 && opt->prec != SAA_FP32_DC64) return SAA_E_INVALID;
  } else if (form == SAA_FORM_MRDINO) {
    if (model == nullptr) return SAA_E_INVALID;
    if (opt->prec != SAA_FP32 && opt->prec != SAA_BF16 && opt->prec != SAA_FP8) return SAA_E_INVALID;
    const mrdino_model* m = (const mrdino_model*)model;
    if (m->dims.d_z != c->dz || m->dims.r_m > c->K1 * c->K1) return SAA_E_MODEL;
  } else {
    return SAA_E_INVALID;
  }
  return SAA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace saa_rt {

// Reduced control Jacobians of the states of the last saa_solve_states call
// by adjoints (see saa_k_adjoint_jac): JY (device, N d_Z x r_u).
int adjoint_jacobians(saa_ctx* c, const saa_options* opt, const double* MPhiT, int r_u, double* JY) {
  const SolveParams sp = solve_params(opt, opt->prec == SAA_FP32);
  switch (opt->prec) {
    case SAA_FP64:
      saa_launch::adjoint_jac<double, double>(c->geo, (double*)c->FT.p, (double*)c->em.p, (double*)c->u.p,
                                              (double*)c->f.p, (double*)c->lam.p, c->mg64.view(), sp, MPhiT, r_u, JY,
                                              (int*)c->lin_adj.p, (int*)c->flag.p, c->N, c->st);
      break;
    case SAA_FP32_DC64:
      saa_launch::adjoint_jac<double, float>(c->geo, (double*)c->FT.p, (double*)c->em.p, (double*)c->u.p,
                                             (double*)c->f.p, (double*)c->lam.p, c->mg32.view(), sp, MPhiT, r_u, JY,
                                             (int*)c->lin_adj.p, (int*)c->flag.p, c->N, c->st);
      break;
    case SAA_FP32:
      saa_launch::adjoint_jac<float, float>(c->geo, (double*)c->FT.p, (double*)c->em.p, (float*)c->u.p,
                                            (float*)c->f.p, (float*)c->lam.p, c->mg32.view(), sp, MPhiT, r_u, JY,
                                            (int*)c->lin_adj.p, (int*)c->flag.p, c->N, c->st);
      break;
    default:
      return SAA_E_INVALID;
  }
  return check_hip(hipGetLastError());
}

}  // namespace saa_rt

extern "C" {

int saa_abi_version(void) { return SAA_ABI_VERSION; }

const char* saa_status_str(int status) {
  switch (status) {
    case SAA_OK: return "ok";
    case SAA_W_FALLBACK: return "ok (surrogate replaced by the PDE form)";
    case SAA_E_INVALID: return "invalid argument";
    case SAA_E_NOCONV: return "a Newton or CG iteration did not converge";
    case SAA_E_DEVICE: return "HIP runtime error";
    case SAA_E_OOM: return "device memory allocation failed";
    case SAA_E_MODEL: return "model does not match the problem";
    case SAA_E_IO: return "file could not be read or written, or is corrupt";
    default: return "unknown status";
  }
}

int saa_options_default(saa_options* o) {
  if (!o) return SAA_E_INVALID;
  std::memset(o, 0, sizeof(*o));
  o->beta = 0.95;
  o->eps = 1e-4;
  o->alpha = 1e-3;
  o->t_mode = 0;
  o->t_in = 0.0;
  o->prec = SAA_FP32_DC64;
  o->newton_tol = 0.0;
  o->lin_rtol = 0.0;
  o->max_newton = 0;
  o->max_lin = 0;
  o->max_dc = 0;
  o->all_adjoints = 0;
  o->fallback_tol = 1e-2;
  return SAA_OK;
}

int saa_ctx_create(const saa_problem* p, int64_t N_max, void* hip_stream, saa_ctx** out) {
  if (!p || !out) return SAA_E_INVALID;
  *out = nullptr;
  if (p->dim != 2) return SAA_E_INVALID;
  if (p->n < 4 || p->n > 4096 || (p->n & (p->n - 1))) return SAA_E_INVALID;
  if (p->n_src_per_dim < 1 || p->n_src_per_dim > 8) return SAA_E_INVALID;
  if (!is_fin(p->src_sigma) || p->src_sigma <= 0) return SAA_E_INVALID;
  if (p->kl_per_dim < 1 || p->kl_per_dim > 64) return SAA_E_INVALID;
  if (!is_fin(p->kl_shift) || p->kl_shift < 0 || !is_fin(p->kl_exp) || p->kl_exp <= 0) return SAA_E_INVALID;
  if (!is_fin(p->kl_amp) || !is_fin(p->reaction) || p->reaction < 0 || !is_fin(p->u_target))
    return SAA_E_INVALID;
  if (p->target != SAA_TARGET_CONST && p->target != SAA_TARGET_SIN && p->target != SAA_TARGET_QUAD)
    return SAA_E_INVALID;
  if (N_max < 1 || N_max > (int64_t)1 << 24) return SAA_E_INVALID;
  // the field synthesis keeps a K1 x (n+1) table and the K1 x K1 coefficients in 64 KB of LDS
  if ((int64_t)p->kl_per_dim * (p->n + 1) + (int64_t)p->kl_per_dim * p->kl_per_dim > 8192) return SAA_E_INVALID;

  saa_ctx* c = new (std::nothrow) saa_ctx();
  if (!c) return SAA_E_OOM;
  c->prob = *p;
  c->N_max = N_max;
  c->st = (hipStream_t)hip_stream;
  c->K1 = p->kl_per_dim;
  c->dz = p->n_src_per_dim * p->n_src_per_dim;
  c->nodes = (int64_t)(p->n + 1) * (p->n + 1);
  c->d_u = (int64_t)(p->n - 1) * (p->n - 1);
  PdeGeo& g = c->geo;
  g.L = 0;
  int64_t off = 0;
  for (int n = p->n; n >= 2; n >>= 1) {
    g.n[g.L] = n;
    g.off[g.L] = off;
    off += (int64_t)(n + 1) * (n + 1);
    ++g.L;
  }
  g.lstride = off;
  g.nodes = c->nodes;
  g.dz = c->dz;
  g.h2 = 1.0 / ((double)p->n * p->n);
  g.r = p->reaction;
  int64_t ks = 0;
  for (int l = 0; l < g.L; ++l) ks += 2 * (int64_t)g.n[l] * g.n[l];
  c->kstride = ks;
  c->kchunk = N_max < 256 ? N_max : 256;

  int rc = SAA_OK;
  const size_t tw = (size_t)N_max * c->nodes * sizeof(double);
  if (!rc) rc = c->FT.alloc((size_t)c->dz * c->nodes * sizeof(double));
  if (!rc) rc = c->S.alloc((size_t)c->K1 * (p->n + 1) * sizeof(double));
  if (!rc) rc = c->amp.alloc((size_t)c->K1 * c->K1 * sizeof(double));
  if (!rc) rc = c->em.alloc(tw);
  if (!rc) rc = c->xi.alloc((size_t)N_max * c->K1 * c->K1 * sizeof(double));
  if (!rc) rc = c->q.alloc((size_t)N_max * sizeof(double));
  if (!rc) rc = c->g.alloc((size_t)N_max * c->dz * sizeof(double));
  if (!rc) rc = c->newton.alloc_zero((size_t)N_max * sizeof(int), c->st);
  if (!rc) rc = c->lin.alloc_zero((size_t)N_max * sizeof(int), c->st);
  if (!rc) rc = c->lin_adj.alloc_zero((size_t)N_max * sizeof(int), c->st);
  if (!rc) rc = c->flag.alloc_zero((size_t)N_max * sizeof(int), c->st);
  if (!rc) rc = c->did.alloc_zero((size_t)N_max * sizeof(int), c->st);
  if (!rc) rc = c->zdev.alloc(SAA_MAX_DZ * sizeof(double));
  if (!rc) rc = c->res.alloc_zero(RES_BYTES, c->st);
  if (!rc) rc = c->hres.alloc(RES_BYTES);
  if (!rc) rc = c->cwork.alloc(saa_launch::cvar_work_bytes());
  if (!rc) rc = c->timer.create();
  if (!rc) rc = c->order.alloc(sizeof(int) * (size_t)c->K1 * c->K1);
  if (!rc) rc = c->mt.alloc(sizeof(double) * (size_t)c->nodes);
  if (rc) {
    delete c;
    return rc;
  }
  {  // KL modes by increasing j^2 + k^2, ties by increasing (j, k): index (j-1) K1 + (k-1)
    std::vector<std::array<int, 3>> modes;
    for (int j = 1; j <= c->K1; ++j)
      for (int k = 1; k <= c->K1; ++k) modes.push_back({j * j + k * k, j, k});
    std::sort(modes.begin(), modes.end());
    std::vector<int> ord;
    for (const auto& md : modes) ord.push_back((md[1] - 1) * c->K1 + (md[2] - 1));
    rc = check_hip(hipMemcpyAsync(c->order.p, ord.data(), sizeof(int) * ord.size(), hipMemcpyHostToDevice, c->st));
    if (!rc) rc = check_hip(hipStreamSynchronize(c->st));
  }
  if (!rc) {
    saa_rt::target_mass(p->n, p->target, p->u_target, c->mt_host, c->ctt);
    g.mt = (const double*)c->mt.p;
    g.ctt = c->ctt;
    rc = check_hip(hipMemcpyAsync(c->mt.p, c->mt_host.data(), sizeof(double) * c->mt_host.size(),
                                  hipMemcpyHostToDevice, c->st));
    if (!rc) rc = check_hip(hipStreamSynchronize(c->st));
  }
  // shared operators: sine table, KL amplitudes, lumped source matrix
  {
    double* a = new double[(size_t)c->K1 * c->K1];
    for (int j = 1; j <= c->K1; ++j)
      for (int k = 1; k <= c->K1; ++k)
        a[(j - 1) * c->K1 + (k - 1)] =
            p->kl_amp * std::pow(M_PI * M_PI * (double)(j * j + k * k) + p->kl_shift, -p->kl_exp);
    rc = check_hip(hipMemcpyAsync(c->amp.p, a, sizeof(double) * c->K1 * c->K1, hipMemcpyHostToDevice, c->st));
    if (!rc) rc = check_hip(hipStreamSynchronize(c->st));
    delete[] a;
  }
  if (!rc) {
    saa_launch::sine_table((double*)c->S.p, c->K1, p->n, c->st);
    saa_launch::source_matrix((double*)c->FT.p, p->n, p->n_src_per_dim, p->src_sigma, c->st);
    rc = check_hip(hipGetLastError());
  }
  if (!rc) rc = check_hip(hipStreamSynchronize(c->st));
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return SAA_OK;
}

void saa_ctx_destroy(saa_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  delete c;
}

int saa_ctx_dims(const saa_ctx* c, int64_t* d_u, int* d_z, int* n_kl) {
  if (!c) return SAA_E_INVALID;
  if (d_u) *d_u = c->d_u;
  if (d_z) *d_z = c->dz;
  if (n_kl) *n_kl = c->K1 * c->K1;
  return SAA_OK;
}

int saa_set_samples(saa_ctx* c, int64_t N, const double* xi_dev) {
  if (!c || !xi_dev || N < 1 || N > c->N_max) return SAA_E_INVALID;
  int rc = check_hip(hipMemcpyAsync(c->xi.p, xi_dev, sizeof(double) * N * c->K1 * c->K1,
                                    hipMemcpyDeviceToDevice, c->st));
  if (rc) return rc;
  c->N = N;
  c->enc_rm = -1;
  c->sg.reset();   // its encode-dependent inputs changed
  saa_launch::field((const double*)c->xi.p, (const double*)c->S.p, (const double*)c->amp.p, (double*)c->em.p,
                    c->K1, c->prob.n, N, c->st);
  rc = check_hip(hipGetLastError());
  if (rc) return rc;
  c->mg64.built = false;
  c->mg32.built = false;
  if (c->mg64.allocated && (rc = build_mg(c, c->mg64))) return rc;
  if (c->mg32.allocated && (rc = build_mg(c, c->mg32))) return rc;
  return check_hip(hipStreamSynchronize(c->st));
}

// Device work of one MR-DINO evaluation on c->st: control bias, fused network
// kernel (q and dq/dz of every sample), CVaR reduction.
static int surrogate_work(saa_ctx* c, mrdino_model* m, const saa_options* opt) {
  int rc = saa_model_eval(m, c, (const double*)c->zdev.p, opt->prec, (double*)c->q.p, (double*)c->g.p);
  if (rc) return rc;
  reduce(c, (double*)c->q.p, (double*)c->g.p, opt, 3, nullptr, nullptr, nullptr, nullptr, nullptr, c->stats());
  return check_hip(hipGetLastError());
}

// Capture surrogate_work into c->sg (kernel nodes only: z is uploaded and the
// results are copied outside the graph).  The capture runs on a stream of the
// context, since the caller's may be the legacy stream; a failure leaves the
// context evaluating eagerly.
static int capture_surrogate(saa_ctx* c, mrdino_model* m, const saa_options* opt,
                             const SurrogateGraph::Key& key) {
  SurrogateGraph& sg = c->sg;
  sg.reset();
  if (!sg.cap && hipStreamCreateWithFlags(&sg.cap, hipStreamNonBlocking) != hipSuccess) {
    sg.cap = nullptr;
    sg.disabled = true;
    (void)hipGetLastError();
    return SAA_OK;
  }
  hipStream_t user = c->st;
  c->st = sg.cap;
  hipGraph_t graph = nullptr;
  int rc = SAA_OK;
  hipError_t e = hipStreamBeginCapture(sg.cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = surrogate_work(c, m, opt);
    e = hipStreamEndCapture(sg.cap, &graph);
  }
  c->st = user;
  if (e == hipSuccess && graph && !rc) e = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (rc || e != hipSuccess || !sg.exec) {
    sg.exec = nullptr;
    sg.disabled = true;
    (void)hipGetLastError();
    return rc;
  }
  sg.key = key;
  return SAA_OK;
}

static int objective_grad_impl(saa_ctx* c, const double* z, int form, const void* model, const saa_options* opt,
                       double* J, double* grad_z, saa_report* rep) {
  if (!c || !z || !J || !grad_z) return SAA_E_INVALID;
  int rc = validate_call(c, z, form, model, opt);
  if (rc) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  if ((rc = check_hip(hipMemcpyAsync(c->zdev.p, z, sizeof(double) * c->dz, hipMemcpyHostToDevice, c->st))))
    return rc;
  PhaseTimer& tm = c->timer;
  tm.on = opt->timing != 0;
  tm.mark(c->st, 0);
  int graph_used = 0;
  if (form == SAA_FORM_PDE) {
    const SolveParams sp = solve_params(opt, opt->prec == SAA_FP32);
    if ((rc = run_state(c, opt->prec, (const double*)c->zdev.p, 0, sp))) return rc;
    tm.mark(c->st, 1);
    reduce(c, (double*)c->q.p, (double*)c->g.p, opt, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    tm.mark(c->st, 2);
    if ((rc = run_adjoint(c, opt->prec, sp, adjoint_act(opt), adjoint_act_w(opt), (double*)c->g.p))) return rc;
    tm.mark(c->st, 3);
    reduce(c, (double*)c->q.p, (double*)c->g.p, opt, 2, (int*)c->newton.p, (int*)c->lin.p, (int*)c->flag.p,
           (int*)c->lin_adj.p, (int*)c->did.p, c->stats());
  } else {
    // surrogate: q and dq/dz of every sample in one fused launch, then the
    // reduction.  The second evaluation with the same arguments captures this
    // device work in a hipGraph; later ones replay it (untimed calls only).
    mrdino_model* m = (mrdino_model*)model;
    SurrogateGraph& sg = c->sg;
    const SurrogateGraph::Key key{m->serial, opt->prec,      opt->t_mode, opt->beta,       opt->eps,
                                  opt->alpha, opt->t_in,     c->N,        opt->risk,       opt->risk_kappa,
                                  opt->risk_tau};
    const bool enc_ready = opt->prec == SAA_FP32 || c->enc_rm == m->dims.r_m;
    if (!tm.on && !sg.disabled && !(sg.exec && sg.key == key) && sg.seen == key && enc_ready &&
        (rc = capture_surrogate(c, m, opt, key)))
      return rc;
    if (!tm.on && sg.exec && sg.key == key) {
      if ((rc = check_hip(hipGraphLaunch(sg.exec, c->st)))) return rc;
      graph_used = 1;
    } else {
      if ((rc = saa_model_eval(m, c, (const double*)c->zdev.p, opt->prec, (double*)c->q.p, (double*)c->g.p)))
        return rc;
      tm.mark(c->st, 1);
      tm.mark(c->st, 2);
      tm.mark(c->st, 3);
      reduce(c, (double*)c->q.p, (double*)c->g.p, opt, 3, nullptr, nullptr, nullptr, nullptr, nullptr, c->stats());
      sg.seen = key;
    }
  }
  tm.mark(c->st, 4);
  if ((rc = check_hip(hipGetLastError()))) return rc;
  if ((rc = fetch_results(c))) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  const double* host = (const double*)c->hres.p;
  *J = host[0];
  for (int k = 0; k < c->dz; ++k) grad_z[k] = host[2 + k];
  rc = fill_report(c, rep, secs, &tm);
  if (rep) rep->graph = graph_used;
  return rc;
}

int saa_objective_grad(saa_ctx* c, const double* z, int form, const void* model, const saa_options* opt,
                       double* J, double* grad_z, saa_report* rep) {
  saa_report own{};
  saa_report* r = rep ? rep : &own;
  int rc = objective_grad_impl(c, z, form, model, opt, J, grad_z, r);
  if (rc < 0 || form != SAA_FORM_MRDINO || !(opt->fallback_tol >= 0.0) || !c->holdout) return rc;
  // Error estimate (surrogate vs PDE form on the held-out samples) and fallback.
  saa_ctx* h = c->holdout;
  saa_options o = *opt;
  o.fallback_tol = -1.0;
  o.timing = 0;
  double Js = 0, Jp = 0, gs[SAA_MAX_DZ], gp[SAA_MAX_DZ];
  saa_report hr{};
  if ((rc = objective_grad_impl(h, z, SAA_FORM_MRDINO, model, &o, &Js, gs, &hr)) < 0) return rc;
  o.prec = SAA_FP32_DC64;
  if ((rc = objective_grad_impl(h, z, SAA_FORM_PDE, nullptr, &o, &Jp, gp, &hr)) < 0) return rc;
  double dg = 0.0, ng = 0.0;
  for (int k = 0; k < c->dz; ++k) {
    dg += (gs[k] - gp[k]) * (gs[k] - gp[k]);
    ng += gp[k] * gp[k];
  }
  const double e_J = std::fabs(Js - Jp) / std::fmax(std::fabs(Jp), 1e-300);
  const double e_g = std::sqrt(dg / std::fmax(ng, 1e-300));
  const double err = std::fmax(e_J, e_g);
  const double t_est = r->seconds;
  r->err_estimate = err;
  if (err <= opt->fallback_tol) return SAA_OK;
  // fall back to the PDE form on the main samples
  if ((rc = objective_grad_impl(c, z, SAA_FORM_PDE, nullptr, &o, J, grad_z, r)) < 0) return rc;
  r->err_estimate = err;
  r->fallback_used = 1;
  r->seconds += t_est;
  return rc == SAA_OK ? SAA_W_FALLBACK : rc;
}

int saa_attach_holdout(saa_ctx* c, saa_ctx* holdout) {
  if (!c || holdout == c) return SAA_E_INVALID;
  if (holdout) {
    const saa_problem& a = c->prob;
    const saa_problem& b = holdout->prob;
    if (a.dim != b.dim || a.n != b.n || a.n_src_per_dim != b.n_src_per_dim || a.src_sigma != b.src_sigma ||
        a.kl_per_dim != b.kl_per_dim || a.kl_shift != b.kl_shift || a.kl_exp != b.kl_exp || a.kl_amp != b.kl_amp ||
        a.reaction != b.reaction || a.u_target != b.u_target || a.target != b.target || holdout->N < 1)
      return SAA_E_INVALID;
  }
  c->holdout = holdout;
  return SAA_OK;
}

int saa_per_sample(saa_ctx* c, const double* z, int form, const void* model, const saa_options* opt,
                   double* q_dev, double* g_dev, saa_report* rep) {
  if (!c || !z || !q_dev || !g_dev) return SAA_E_INVALID;
  int rc = validate_call(c, z, form, model, opt);
  if (rc) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  if ((rc = check_hip(hipMemcpyAsync(c->zdev.p, z, sizeof(double) * c->dz, hipMemcpyHostToDevice, c->st))))
    return rc;
  if (form == SAA_FORM_PDE) {
    const SolveParams sp = solve_params(opt, opt->prec == SAA_FP32);
    if ((rc = run_state(c, opt->prec, (const double*)c->zdev.p, 0, sp))) return rc;
    if ((rc = run_adjoint(c, opt->prec, sp, 1, 0.0, g_dev))) return rc;
    if ((rc = check_hip(hipMemcpyAsync(q_dev, c->q.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->st))))
      return rc;
    reduce(c, (double*)c->q.p, g_dev, opt, 3, (int*)c->newton.p, (int*)c->lin.p, (int*)c->flag.p,
           (int*)c->lin_adj.p, (int*)c->did.p, c->stats());
  } else {
    if ((rc = saa_model_eval((mrdino_model*)model, c, (const double*)c->zdev.p, opt->prec, q_dev, g_dev)))
      return rc;
    reduce(c, q_dev, g_dev, opt, 3, nullptr, nullptr, nullptr, nullptr, nullptr, c->stats());
  }
  if ((rc = check_hip(hipGetLastError()))) return rc;
  if ((rc = fetch_results(c))) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return fill_report(c, rep, secs, nullptr);
}

int saa_solve_states(saa_ctx* c, const double* Z_dev, const saa_options* opt, double* u_dev, double* q_dev,
                     double* dudz_dev, saa_report* rep) {
  if (!c || !Z_dev || !u_dev) return SAA_E_INVALID;
  int rc = validate_options(opt);
  if (rc) return rc;
  if (c->N < 1) return SAA_E_INVALID;
  if (opt->prec != SAA_FP64 && opt->prec != SAA_FP32 && opt->prec != SAA_FP32_DC64) return SAA_E_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  const SolveParams sp = solve_params(opt, opt->prec == SAA_FP32);
  if ((rc = run_state(c, opt->prec, Z_dev, c->dz, sp))) return rc;
  const int n = c->prob.n;
  if (opt->prec == SAA_FP32) saa_launch::interior_copy<float>((float*)c->u.p, u_dev, n, c->N, c->st);
  else saa_launch::interior_copy<double>((double*)c->u.p, u_dev, n, c->N, c->st);
  if (q_dev &&
      (rc = check_hip(hipMemcpyAsync(q_dev, c->q.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->st))))
    return rc;
  if ((rc = check_hip(hipMemsetAsync(c->lin_adj.p, 0, sizeof(int) * c->N, c->st)))) return rc;
  if (dudz_dev) {
    switch (opt->prec) {
      case SAA_FP64:
        saa_launch::linearized<double, double>(c->geo, (double*)c->FT.p, (double*)c->em.p, (double*)c->u.p,
                                               (double*)c->f.p, (double*)c->lam.p, c->mg64.view(), sp, dudz_dev,
                                               (int*)c->lin_adj.p, (int*)c->flag.p, c->N, c->st);
        break;
      case SAA_FP32_DC64:
        saa_launch::linearized<double, float>(c->geo, (double*)c->FT.p, (double*)c->em.p, (double*)c->u.p,
                                              (double*)c->f.p, (double*)c->lam.p, c->mg32.view(), sp, dudz_dev,
                                              (int*)c->lin_adj.p, (int*)c->flag.p, c->N, c->st);
        break;
      default:
        saa_launch::linearized<float, float>(c->geo, (double*)c->FT.p, (double*)c->em.p, (float*)c->u.p,
                                             (float*)c->f.p, (float*)c->lam.p, c->mg32.view(), sp, dudz_dev,
                                             (int*)c->lin_adj.p, (int*)c->flag.p, c->N, c->st);
    }
  }
  // stats only (phase 0)
  saa_launch::cvar((double*)c->q.p, (double*)c->g.p, c->N, c->dz, 0.0, 1.0, 0.0, (double*)c->zdev.p, 1, 0.0, 0,
                   c->tstar(), c->out(), (int*)c->newton.p, (int*)c->lin.p, (int*)c->flag.p,
                   (int*)c->lin_adj.p, nullptr, c->stats(), c->cwork.p, c->st);
  if ((rc = check_hip(hipGetLastError()))) return rc;
  if ((rc = fetch_results(c))) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  rc = fill_report(c, rep, secs, nullptr);
  if (rep) rep->t_star = rep->dJ_dt = 0.0;   // no CVaR reduction here
  return rc;
}

int saa_sample_status(saa_ctx* c, int* flags, int* newton_iters, int* lin_iters, int* adj_lin_iters) {
  if (!c || c->N < 1) return SAA_E_INVALID;
  const size_t b = sizeof(int) * (size_t)c->N;
  int rc = SAA_OK;
  if (flags && !rc) rc = check_hip(hipMemcpyAsync(flags, c->flag.p, b, hipMemcpyDeviceToHost, c->st));
  if (newton_iters && !rc) rc = check_hip(hipMemcpyAsync(newton_iters, c->newton.p, b, hipMemcpyDeviceToHost, c->st));
  if (lin_iters && !rc) rc = check_hip(hipMemcpyAsync(lin_iters, c->lin.p, b, hipMemcpyDeviceToHost, c->st));
  if (adj_lin_iters && !rc) rc = check_hip(hipMemcpyAsync(adj_lin_iters, c->lin_adj.p, b, hipMemcpyDeviceToHost, c->st));
  if (!rc) rc = check_hip(hipStreamSynchronize(c->st));
  return rc;
}

}  // extern "C"
