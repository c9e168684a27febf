/*
 * saa.h -- C ABI of the MI355X SAA smoothed-CVaR engine.
 *
 * The library evaluates, for a fixed set of N random-field samples m_i and a
 * control z, the sample-average smoothed-CVaR objective
 *
 *   J(z) = min_t  t + 1/(N (1-beta)) sum_i s_eps(q_i(z) - t) + alpha/2 |z|^2
 *
 * (paper Sec. 2.2, eq. (CVaR_saa_ouu), with the C^2 smoothed plus function of
 * Sec. 2.1) and its gradient grad J = sum_i w_i dq_i/dz + alpha z, where
 * w_i = s_eps'(q_i - t*) / (N (1-beta)) (chain rule of eq.
 * (ouu_risk_gradient)).  q_i = int (u_i - u_target)^2 dx is the tracking QoI of
 * the state u_i of the semilinear elliptic equation of Sec. 4.2,
 *
 *   -div(exp(m_i) grad u) + r u^3 = sum_k z_k f_k,   u = 0 on the boundary,
 *
 * discretised by P1 finite elements on a uniform n x n triangulated grid.
 * dq_i/dz comes from one adjoint solve per sample (Sec. 2.3,
 * eq. (ouu_qoi_gradient)).
 *
 * Conventions for every entry point:
 *  - Every call returns an int status (SAA_OK = 0, > 0 success with warning,
 *    < 0 error).  No C++ exception crosses this boundary.
 *  - Arguments are validated before any device work; invalid arguments return
 *    SAA_E_INVALID and leave outputs untouched.
 *  - "device" pointers are HIP device allocations owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller.  The library never
 *    keeps a caller pointer past the call, except that saa_set_samples copies
 *    the samples into the context.
 *  - All device work is enqueued on the HIP stream given at context creation;
 *    calls that return host values synchronise that stream before returning.
 *  - A context is not thread-safe: calls on one context must be serialised.
 *
 * Grid conventions (2D): nodes x_p = (i h, j h), 0 <= i, j <= n, h = 1/n, flat
 * node index p = j (n+1) + i.  The d_U = (n-1)^2 unknowns are the interior
 * nodes, listed in increasing flat index ("interior order").
 */
#ifndef SAA_H
#define SAA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SAA_ABI_VERSION 3

/* Status codes. */
enum {
  SAA_OK = 0,
  SAA_W_FALLBACK = 1,  /* success; the surrogate was replaced by the PDE form */
  SAA_E_INVALID = -1,  /* bad argument (null pointer, out-of-range value, NaN) */
  SAA_E_NOCONV = -2,   /* a Newton or CG iteration did not converge; outputs
                          are written, report->n_unconverged says how many */
  SAA_E_DEVICE = -3,   /* a HIP runtime call failed */
  SAA_E_OOM = -4,      /* device allocation failed */
  SAA_E_MODEL = -5,    /* model does not match the context's problem */
  SAA_E_IO = -6        /* file could not be read or written, or is corrupt */
};

/* Forms of the objective. */
enum { SAA_FORM_PDE = 0, SAA_FORM_MRDINO = 1 };

/* Arithmetic precision.
 * PDE form:
 *  SAA_FP64      : FP64 everywhere (FP64 multigrid-preconditioned CG).
 *  SAA_FP32      : FP32 everywhere except the final CVaR reduction (FP64).
 *  SAA_FP32_DC64 : FP32 multigrid-preconditioned CG inside FP64 Newton /
 *                  defect correction: residuals, state, adjoint, QoI and
 *                  gradient in FP64.
 * MR-DINO form (the CVaR reduction is FP64 in every case):
 *  SAA_FP32      : FP32 network evaluation (reference kernel).
 *  SAA_BF16      : BF16 operands, FP32 accumulation (MFMA).
 *  SAA_FP8       : FP8 E4M3 operands with power-of-two scales per weight
 *                  operand and per sample, FP32 accumulation (MFMA); a few
 *                  percent less accurate in dq/dz than BF16. */
enum { SAA_FP64 = 0, SAA_FP32 = 1, SAA_FP32_DC64 = 2, SAA_BF16 = 3, SAA_FP8 = 4 };

/* Problem definition (Sec. 4.2).  Sources f_k(x) = (sigma sqrt(2 pi))^-1
 * exp(-|x - x_k|^2 / (2 sigma^2)) sit on the interior lattice
 * x_k = ((a+1)/(s+1), (b+1)/(s+1)), k = s b + a, s = n_src_per_dim.
 * The log-coefficient is m(x) = sum_{j,k=1..K1} a_jk xi_jk sin(j pi x) sin(k pi y)
 * with a_jk = kl_amp (pi^2 (j^2 + k^2) + kl_shift)^(-kl_exp).
 *
 * dim = 3: the same equation on the unit cube with trilinear (Q1) elements
 * on n^3 cells (n even, 4 <= n <= 96, halving to a coarsest grid of at most
 * 7 cells: 48, 32, 40, 56 ... are accepted, 36 is not), sources on the
 * s x s x s lattice ((a+1)/(s+1), (b+1)/(s+1), (c+1)/(s+1)), k = a + s b +
 * s^2 c, d_Z = s^3 (s in 1..4), field sum_{j,k,l} a_jkl xi_jkl sin sin sin
 * with a_jkl = kl_amp (pi^2 (j^2 + k^2 + l^2) + kl_shift)^(-kl_exp) (K1 in
 * 1..16, xi laid out (N, K1, K1, K1) with j the x-frequency), kappa per
 * element the mean of exp(m) over its 8 vertices, lumped reaction and
 * source, consistent Q1 mass in the QoI; the sinusoidal target is
 * sin(2 pi x) sin(2 pi y) sin(2 pi z).  Both forms are available; the
 * training data use forward control Jacobians only (jac_mode ADJOINT
 * returns SAA_E_INVALID), projected in chunks of samples; N_max up to
 * min(2^20, floor((2^32 - 1) / (256 (n + 1)))), so that every launch grid
 * (N (n + 1) workgroups of 256 threads for the field) fits 2^32 - 1
 * work-items: 172960 at n = 96, 986895 at n = 16. */
typedef struct saa_problem {
  int dim;             /* 2, or 3 (see above) */
  int n;               /* cells per side; 2D: 2^k or 3 * 2^k, 4 <= n <= 4096 */
  int n_src_per_dim;   /* s: d_Z = s^2 controls (1..8); 3D: s^3 (1..4) */
  double src_sigma;    /* source width sigma > 0 */
  int kl_per_dim;      /* K1 in 1..64 */
  double kl_shift;     /* >= 0 */
  double kl_exp;       /* > 0 */
  double kl_amp;       /* any finite value */
  double reaction;     /* r >= 0 */
  double u_target;     /* target state when target = SAA_TARGET_CONST */
  int target;          /* target state (Sec. 4.2): SAA_TARGET_CONST (u_target
                          everywhere), SAA_TARGET_SIN (sin(2 pi x) sin(2 pi y)),
                          SAA_TARGET_QUAD (4 y (1 - y)); interpolated at the
                          nodes, boundary nodes included */
  int pad_;
} saa_problem;

enum { SAA_TARGET_CONST = 0, SAA_TARGET_SIN = 1, SAA_TARGET_QUAD = 2 };

/* Options of one objective evaluation.  Fill with saa_options_default() and
 * override fields as needed. */
typedef struct saa_options {
  double beta;         /* CVaR level, 0 <= beta < 1 */
  double eps;          /* smoothing width of s_eps, > 0 */
  double alpha;        /* control cost weight, >= 0 */
  int t_mode;          /* 0: t minimised out (J(z) = min_t J_hat(z,t));
                          1: J_hat(z, t_in) and dJ_hat/dt are returned */
  double t_in;
  int prec;            /* SAA_FP64 | SAA_FP32 | SAA_FP32_DC64 (PDE form) */
  double newton_tol;   /* stop Newton / defect correction when the update, or
                          the error predicted after it from the contraction of
                          the last two updates, is <= newton_tol * |iterate|
                          (2-norms); <= 0: default (1e-13 with FP64 state,
                          1e-5 with FP32 state).  An iteration also stops once
                          its updates stop contracting below 1e-4 relative
                          (rounding floor).  Inner PCG tolerances adapt to the
                          predicted error, never tighter than lin_rtol.
                          Adjoint and linearised solves use
                          max(newton_tol, 1e-11) with FP64 state. */
  double lin_rtol;     /* relative residual of each inner PCG solve; <= 0:
                          default 1e-6 (1e-5 with FP32 state) */
  int max_newton;      /* <= 0: default 30 */
  int max_lin;         /* max PCG iterations per inner solve; <= 0: 200 */
  int max_dc;          /* max adjoint defect-correction passes; <= 0: 10 */
  int all_adjoints;    /* 0: solve adjoints only for samples whose CVaR weight
                          w_i is non-zero (the others contribute exactly 0 to
                          grad J); 1: solve all */
  double fallback_tol; /* MR-DINO form: relative error above which the PDE form
                          is used instead; < 0 disables */
  int timing;          /* 1: time each phase with HIP events on the context's
                          stream and fill the ms_* fields of the report */
  int risk;            /* risk measure rho (Sec. 2.1; SAA estimators Sec. 2.2):
                          SAA_RISK_CVAR: smoothed CVaR_beta by eq. (CVaR_saa_ouu)
                            (default);
                          SAA_RISK_MEAN: E[Q] (risk neutral);
                          SAA_RISK_MEAN_VAR: E[Q] + risk_kappa Var[Q] (the SAA
                            variance with 1/N), first two moments;
                          SAA_RISK_POF: smoothed probability of failure
                            P[Q > risk_tau] ~ E[s_eps'(Q - risk_tau)] (the
                            derivative of the same C^2 smoothing, a C^1 step
                            of width eps);
                          SAA_RISK_BPOE: smoothed buffered probability of
                            exceedance of risk_tau, min over a >= 0 of
                            E[s_eps(a (Q - risk_tau) + 1)] (Mafusalov and
                            Uryasev); a* = infinity (value 0) when no sample
                            exceeds risk_tau.
                          The non-CVaR measures need t_mode = 0; beta is
                          ignored; the report's t_star is the mean of q
                          (MEAN_VAR), risk_tau (POF), a* (BPOE) or 0 (MEAN),
                          dJ_dt 0. */
  int jac_mode;        /* control Jacobians of mrdino_data_create (Sec. 3.4):
                          SAA_JAC_AUTO (adjoint when d_Z >= r_u, else
                          forward), SAA_JAC_FORWARD (d_Z linearised solves per
                          sample), SAA_JAC_ADJOINT (r_u solves with right-hand
                          sides M phi_k per sample, giving the reduced
                          Jacobian Phi^T M du/dz directly) */
  double risk_kappa;   /* MEAN_VAR weight, >= 0 */
  double risk_tau;     /* POF threshold, finite */
} saa_options;

enum { SAA_RISK_CVAR = 0, SAA_RISK_MEAN = 1, SAA_RISK_MEAN_VAR = 2, SAA_RISK_POF = 3, SAA_RISK_BPOE = 4 };
enum { SAA_JAC_AUTO = 0, SAA_JAC_FORWARD = 1, SAA_JAC_ADJOINT = 2 };

typedef struct saa_report {
  double t_star;       /* the t used (minimiser, or t_in) */
  double dJ_dt;        /* 1 - sum_i w_i */
  double err_estimate; /* surrogate error estimate, or 0 */
  double seconds;      /* wall time of the call (device-synchronised) */
  int newton_max;      /* max Newton iterations over samples */
  int n_unconverged;   /* samples whose Newton or adjoint did not converge */
  int n_adjoints;      /* adjoint solves performed */
  int fallback_used;   /* 1 if the PDE form replaced the surrogate */
  int64_t lin_total;   /* total inner PCG iterations over all samples */
  int64_t newton_total;/* total Newton iterations over all samples */
  double ms_state;     /* with opt->timing: device time of the state solve (or
                          surrogate evaluation) kernel, milliseconds */
  double ms_adjoint;   /* ... of the adjoint solves */
  double ms_reduce;    /* ... of the CVaR reductions */
  int graph;           /* MR-DINO form: 1 if the device work ran as one replay of
                          the context's captured hipGraph (see saa_objective_grad) */
  int pad;
} saa_report;

typedef struct saa_ctx saa_ctx;

/* Library ABI version (SAA_ABI_VERSION). */
int saa_abi_version(void);

/* Text for a status code; never NULL. */
const char* saa_status_str(int status);

/* Defaults: beta 0.95, eps 1e-4, alpha 1e-3, t_mode 0, prec SAA_FP32_DC64,
 * tolerances <= 0 (i.e. per-precision defaults), all_adjoints 0,
 * fallback_tol 1e-2.  Returns SAA_E_INVALID for NULL. */
int saa_options_default(saa_options* opt);

/* Create a context for `prob` that can hold up to N_max samples.  The
 * context owns all workspaces (sized for N_max) and the shared operators
 * (source matrix, sine tables).  `hip_stream` is a hipStream_t (NULL = the
 * default stream).  On success *out receives the context; the caller frees it
 * with saa_ctx_destroy.  Device memory in 2D is about 1.3 MB per sample at
 * n = 128 and 1.8 GB per sample at n = 4096 (FP32-DC64; the solver
 * workspaces of a precision are allocated at its first use), plus d_Z x
 * (n+1)^2 doubles of source matrix and at most 4 GiB of set-up scratch for
 * saa_set_samples; SAA_E_OOM when an allocation fails, SAA_E_INVALID for a
 * problem outside the ranges above or N_max outside 1 .. 4194303 in 2D (one
 * 1024-thread workgroup per sample must fit a grid of 2^32 - 1 work-items;
 * the 3D bound is stated above), checked before any device work.
 * Debugging aid: with the environment variable SAA_POISON_WORKSPACE set (and
 * not "0") when the context is created, every saa_objective_grad and
 * saa_per_sample call first fills the context's per-call buffers (q, dq/dz,
 * results, reduction workspace, state, right-hand side, adjoint and
 * per-sample counters) with NaN bytes; results must not change.  It adds
 * one fill per buffer per call and is off by default. */
int saa_ctx_create(const saa_problem* prob, int64_t N_max, void* hip_stream, saa_ctx** out);

/* Free a context and everything it owns (NULL is ignored). */
void saa_ctx_destroy(saa_ctx* ctx);

/* Number of unknowns d_U, controls d_Z and KL coefficients per sample of the
 * context's problem; any pointer may be NULL. */
int saa_ctx_dims(const saa_ctx* ctx, int64_t* d_u, int* d_z, int* n_kl);

/* Install the fixed sample set (Sec. 2.2: fixed samples make the SAA problem
 * deterministic).  xi_dev: device, N x K1^2 float64, row-major, sample-major,
 * within a sample j (x-frequency) slow and k fast.  Builds on the device the
 * nodal fields exp(m_i) and the multigrid operator hierarchy of every sample.
 * 1 <= N <= N_max.  Not part of an objective evaluation's timing. */
int saa_set_samples(saa_ctx* ctx, int64_t N, const double* xi_dev);

/* SAA objective and gradient at control z (host, d_Z float64).  form selects
 * the PDE form (model must be NULL) or the MR-DINO surrogate.  J (host, 1) and
 * grad_z (host, d_Z) receive the results; report may be NULL.  Returns
 * SAA_E_NOCONV if some sample did not converge (results still written).
 * MR-DINO form: the second untimed evaluation with the same model, precision,
 * beta, eps, alpha, t_mode, t_in and sample count captures its device work
 * (control bias, fused network kernel, CVaR reduction) in a hipGraph owned by
 * the context; later such calls replay it (report->graph = 1).  z is uploaded
 * and the results are read outside the graph; parameter updates of the same
 * model (mrdino_set_params, mrdino_set_qoi) are in place and stay valid;
 * saa_set_samples drops the graph. */
int saa_objective_grad(saa_ctx* ctx, const double* z, int form, const void* model,
                       const saa_options* opt, double* J, double* grad_z,
                       saa_report* report);

/* Attach (holdout != NULL) or detach (NULL) a context of held-out samples of
 * the same problem.  With a holdout attached, saa_objective_grad in the MR-DINO
 * form with opt->fallback_tol >= 0 also evaluates the surrogate and the PDE
 * form (FP32_DC64) on the held-out samples at the same z, sets
 * report->err_estimate = max(|J_s - J_p| / |J_p|, |grad_s - grad_p| / |grad_p|)
 * and, when it exceeds fallback_tol, returns the PDE form on the main samples
 * with status SAA_W_FALLBACK and report->fallback_used = 1.  Without a holdout
 * err_estimate is -1.  The caller keeps ownership; the holdout must stay alive
 * while attached. */
int saa_attach_holdout(saa_ctx* ctx, saa_ctx* holdout);

/* Per-sample QoI and gradient at control z (host, d_Z): q_dev (device, N
 * float64) and g_dev (device, N x d_Z float64, row-major) receive q_i and
 * dq_i/dz for every sample (all adjoints are solved).  report may be NULL. */
int saa_per_sample(saa_ctx* ctx, const double* z, int form, const void* model,
                   const saa_options* opt, double* q_dev, double* g_dev,
                   saa_report* report);

/* PDE states at per-sample controls (training data, Sec. 3.4).
 * Z_dev: device, N x d_Z float64 (control of sample i in row i).
 * u_dev (device, N x d_U float64, interior order) receives the states; q_dev
 * (device, N, may be NULL) the QoIs; dudz_dev (device, N x d_Z x d_U float64,
 * may be NULL) the control Jacobians du_i/dz = A(u_i)^{-1} F by d_Z
 * linearised solves with the state's operator (eq. (projected_sensitivity),
 * d_Z < r_U case).  Uses opt->prec, tolerances and iteration limits. */
int saa_solve_states(saa_ctx* ctx, const double* Z_dev, const saa_options* opt,
                     double* u_dev, double* q_dev, double* dudz_dev, saa_report* report);

/* ------------------------------------------------------------------------
 * MR-DINO surrogate (Sec. 3.3, eq. (rbnet)): u_w = Phi phi_w(m_r, z) + b.
 * phi_w is a dense network on x = [m_r; z]: `depth` hidden layers of `width`
 * units with GELU (erf form), then a linear layer to r_u reduced state
 * coordinates.  m_r are the r_m leading whitened KL coordinates of the sample
 * (modes ordered by increasing j^2 + k^2 [+ l^2], ties by increasing (j, k[, l])).  For the
 * quadratic tracking QoI the reduced evaluation of Sec. 3.3 gives
 * q = |phi + c|^2 + c0 (c, c0 from the POD basis, see mrdino_set_qoi), and
 * dq/dz is obtained by reverse-mode differentiation of the network
 * (eq. (neural_operator_gradient)).
 * ------------------------------------------------------------------------ */
typedef struct mrdino_dims {
  int r_m;     /* input KL coordinates (1..128 at width 256, 1..256 at width 512) */
  int d_z;     /* controls (1..32 at width 256, 1..64 at width 512); must equal the context's d_Z */
  int r_u;     /* reduced state coordinates (1..width) */
  int width;   /* hidden width: 256 or 512 */
  int depth;   /* hidden layers (4) */
} mrdino_dims;

typedef struct mrdino_model mrdino_model;

/* Number of parameters of a network with these dimensions.  Packed order:
 * W_0 (width x (r_m + d_z), row-major), b_0 (width), W_1 (width x width), b_1,
 * ..., W_depth (r_u x width), b_depth. */
int mrdino_num_params(const mrdino_dims* dims, int64_t* n);

/* Create a model (parameters zero) whose device work runs on `hip_stream`.
 * Returns SAA_E_INVALID for unsupported dimensions. */
int mrdino_create(const mrdino_dims* dims, void* hip_stream, mrdino_model** out);

/* Free a model (NULL is ignored). */
void mrdino_free(mrdino_model* model);

/* Save a model (dimensions, FP32 parameters, c, c0 and, once trained, the
 * optimiser state) to a file, and load one into a new model whose device work
 * runs on `hip_stream`.  Format: the bytes "SAADINO1", uint32 version 2, int32
 * r_m d_z r_u width depth, int64 n_params, float64 c0, float64 c[r_u], float32
 * params[n_params], int32 has_train and, when it is 1, int64 Adam step, int64
 * completed epochs, uint64 minibatch-stream state, float32 m[n_params],
 * float32 v[n_params]; then the 64-bit FNV-1a hash of all preceding bytes, in
 * native byte order.  Version 1 files (no has_train field) also load.  Loading
 * validates the whole file before any device work: a missing, truncated,
 * altered or unsupported file returns SAA_E_IO and *out stays NULL.  A loaded
 * model with optimiser state continues training exactly where the saved one
 * stopped (mrdino_train_cfg.resume = 1). */
int mrdino_save(const mrdino_model* model, const char* path);
/* Dimensions of a model (e.g. one returned by mrdino_load). */
int mrdino_get_dims(const mrdino_model* model, mrdino_dims* dims);
int mrdino_load(const char* path, void* hip_stream, mrdino_model** out);

/* Set / get the FP32 parameters (host, n = mrdino_num_params, packed order
 * above).  Setting rebuilds the device operands (BF16 MFMA copies). */
int mrdino_set_params(mrdino_model* model, const float* params, int64_t n);
int mrdino_get_params(const mrdino_model* model, float* params, int64_t n);

/* Reduced QoI terms: c (host, r_u) and c0, so that q = |phi + c|^2 + c0.  For
 * an M-orthonormal POD basis Phi and mean state b: c = Phi^T (M (b - u_t))_I
 * and c0 = |b - u_t|_M^2 - |c|^2. */
int mrdino_set_qoi(mrdino_model* model, const double* c, double c0);

/* Network outputs for the samples installed in ctx at the control z (host,
 * d_Z float64): x_i = [m_r(xi_i); z] (Sec. 3.3, eq. (rbnet)).  `want` is a
 * bitmask of the outputs to write (device pointers; the others may be NULL):
 *   MRDINO_WANT_Q       q_dev      N float64: q_i = |phi_i + c|^2 + c0
 *   MRDINO_WANT_DQDZ    dqdz_dev   N x d_Z float64: dq_i/dz (reverse mode)
 *   MRDINO_WANT_PHI     phi_dev    N x r_u float32: reduced state phi_i
 *   MRDINO_WANT_DPHIDZ  dphidz_dev N x d_Z x r_u float32: entry (i, k, j) =
 *                       d phi_ij / d z_k (forward mode, eq. (rbnet) derivative)
 * q and dq/dz come from the fused evaluation kernel in `prec` (SAA_FP32,
 * SAA_BF16 or SAA_FP8); phi and dphi/dz always in float32, through the training forward
 * in batches (its workspace stays allocated in the model).  Runs on the
 * model's stream after synchronising the context's; returns once the outputs
 * are written. */
enum { MRDINO_WANT_Q = 1, MRDINO_WANT_DQDZ = 2, MRDINO_WANT_PHI = 4, MRDINO_WANT_DPHIDZ = 8 };
int mrdino_eval(mrdino_model* model, saa_ctx* ctx, const double* z, int want, int prec, double* q_dev,
                double* dqdz_dev, float* phi_dev, float* dphidz_dev);

/* ------------------------------------------------------------------------
 * MR-DINO construction (Sec. 3.3-3.4): training data from the PDE form,
 * weighted POD, derivative-informed training.
 * ------------------------------------------------------------------------ */
typedef struct mrdino_data mrdino_data;

/* Training data for the samples installed in ctx at per-sample controls
 * Z_dev (device, N x d_Z float64; the auxiliary control law of Sec. 3.1):
 *  1. states u_i by the PDE form (opt->prec, tolerances) and, in forward
 *     mode (opt->jac_mode), control Jacobians du_i/dz by d_Z linearised
 *     solves per sample (Sec. 3.4);
 *  2. weighted POD (Sec. 3.3) from the first n_pod states: mean b, Gram
 *     G = D^T M D of the centred snapshots, G V = V Lambda (host
 *     eigensolver), Phi = D V_r Lambda_r^{-1/2} (M-orthonormal; each column of
 *     V signed so its largest-magnitude entry is positive);
 *  3. reduced data y_i = Phi^T M (u_i - b) and J_i = Phi^T M du_i/dz
 *     (eq. (reduced_basis_derivative_equivalence)), in adjoint mode by r_u
 *     solves A(u_i) lambda_k = M phi_k and J_i[k, :] = F^T lambda_k;
 *     inputs x_i = [m_r; z_i];
 *  4. reduced-QoI terms c, c0 (see mrdino_set_qoi).
 * 2 <= N, 1 <= r_u <= n_pod <= min(N, 8192), 1 <= r_m <= K1^2.  With a
 * non-NULL `basis` (held-out data) steps 2 and 4 are skipped: its mean, POD
 * basis and QoI terms are reused (n_pod is ignored; r_u and the problem must
 * match).  Device memory during construction: about 8 (d_Z + 2) N d_U bytes
 * in forward mode, 16 N d_U + 8 r_u d_U in adjoint mode.
 * Returns SAA_E_INVALID also when the Gram matrix has rank below r_u. */
int mrdino_data_create(saa_ctx* ctx, const double* Z_dev, int r_m, int r_u, int n_pod, const saa_options* opt,
                       const mrdino_data* basis, mrdino_data** out, saa_report* report);

/* Free training data (NULL is ignored). */
void mrdino_data_free(mrdino_data* data);

/* Sizes and reduced-QoI terms: N, c (host, r_u), c0, Gram eigenvalues (host,
 * n_pod, decreasing); any pointer may be NULL. */
int mrdino_data_info(const mrdino_data* data, int64_t* N, double* c, double* c0, double* lam);

/* Reduced-QoI terms c (host, r_u) and c0 of the tracking functional for
 * another target state (target: SAA_TARGET_*, u_target for the constant one)
 * with the same POD basis: one trained surrogate serves several objectives
 * (Sec. 4.2 reuses one network across targets and beta).  Pass them to
 * mrdino_set_qoi.  SAA_E_INVALID for a bad target or NULL pointers. */
int mrdino_data_qoi(const mrdino_data* data, int target, double u_target, double* c, double* c0);

/* Copy a data array to host memory: which = 0 inputs X (float, N x (r_m+d_Z)),
 * 1 Y (float, N x r_u), 2 J (float, (N d_Z) x r_u, row i d_Z + k holds
 * d/dz_k of sample i), 3 Phi^T (double, r_u x d_U), 4 mean state b (double,
 * d_U).  n is the element count of the array. */
int mrdino_data_get(const mrdino_data* data, int which, void* host, int64_t n);

/* Batch-mean training loss L = 1/B sum_b |phi_b - y_b|^2 + |dphi_b/dz - J_b|_F^2
 * (dino = 1; dino = 0 drops the Jacobian term: the L2-only MR-NO loss) of the
 * data rows idx (host, B indices), and its gradient (host, n_params floats,
 * packed order; may be NULL) by the hand-written reverse pass through the
 * forward-mode Jacobian recurrence (Sec. 3.4,
 * eq. (reduced_basis_derivative_equivalence)).  prec: SAA_BF16 (products with
 * BF16 operands and FP32 accumulation, the training precision) or SAA_FP32
 * (FP32 operands); elementwise work and the loss sums are FP32 / FP64 either
 * way.  Other precisions return SAA_E_INVALID. */
int mrdino_loss_grad(mrdino_model* model, mrdino_data* data, const int* idx, int B, int dino, int prec,
                     double* loss, float* grad);

typedef struct mrdino_train_cfg {
  int batch;          /* minibatch size */
  int epochs;
  int lr_drop_epoch;  /* from this epoch on lr_late is used (<= 0: never) */
  double lr, lr_late; /* Adam step sizes */
  double beta1, beta2, adam_eps;
  int dino;           /* 1: DINO loss (MR-DINO); 0: L2-only loss (MR-NO) */
  uint64_t seed;      /* minibatch order: splitmix64 stream, Fisher-Yates per epoch */
  int prec;           /* SAA_BF16 (BF16 operands, FP32 accumulation and master weights) or SAA_FP32 */
  int resume;         /* 0: new optimisation (Adam moments zero, epoch clock 0, stream from seed);
                         1: continue the model's optimiser state (e.g. from mrdino_load) */
} mrdino_train_cfg;

/* Train the model's FP32 parameters with Adam (the optimiser of Sec. 4.2.1) on
 * the data; every epoch visits floor(N / batch) minibatches of a fresh
 * permutation.  The optimiser state (Adam moments and step, completed epochs,
 * which drive lr_drop_epoch, and the minibatch stream) lives in the model:
 * cfg.resume = 1 continues it, so k epochs then m more give bitwise the same
 * parameters as k + m epochs in one call.  On return the device operands are
 * repacked and the model's reduced-QoI terms are set from the data.  The
 * output layer is trained in scaled units, phi = sigma phi', against the
 * targets y / sigma and J / sigma (the DINO loss divided by sigma^2: the same
 * minimiser), sigma = the RMS of the data's reduced states rounded to a power
 * of two, so that the conversion of the stored parameters (always in the
 * data's units) is exact; a fresh output layer scaled by sigma starts at the
 * scale of the targets.  epoch_loss (host, epochs, may be NULL) receives the
 * mean loss of each epoch in the data's units;
 * seconds (may be NULL) the device time of the loop.  Invalid settings return
 * SAA_E_INVALID before any device work; a failed launch SAA_E_DEVICE. */
int mrdino_train(mrdino_model* model, mrdino_data* data, const mrdino_train_cfg* cfg, double* epoch_loss,
                 double* seconds);

/* Relative reduced-space errors of the model on a data set:
 * err_state = sqrt(sum_i |phi_i - y_i|^2 / sum_i |y_i|^2),
 * err_jac = sqrt(sum_i |dphi_i/dz - J_i|_F^2 / sum_i |J_i|_F^2). */
int mrdino_data_errors(mrdino_model* model, mrdino_data* data, double* err_state, double* err_jac);

/* Host symmetric eigensolver used for the POD Gram matrix (Householder
 * tridiagonalisation, implicit QL with Wilkinson shifts).  A: n x n row-major
 * (symmetrised), w: eigenvalues in decreasing order, V: n x n row-major with
 * the eigenvectors as columns.  Needs no GPU. */
int saa_sym_eig(int n, const double* A, double* w, double* V);

/* The same on the GPU (parallel cyclic Jacobi, one kernel per round of n/2
 * disjoint rotations), used by mrdino_data_create for the POD.  A_dev:
 * device, n x n row-major (symmetrised, not modified); w: host, n, decreasing;
 * V_dev: device, n x n row-major, eigenvectors as columns; hip_stream: the
 * stream (NULL = default); sweeps (may be NULL) receives the Jacobi sweeps
 * run.  Synchronises the stream.  SAA_E_NOCONV after 60 sweeps. */
int saa_sym_eig_gpu(int n, const double* A_dev, double* w, double* V_dev, void* hip_stream, int* sweeps);

/* ------------------------------------------------------------------------
 * Outer OUU solve (Sec. 2.1, eq. (ouu); eq. (CVaR_ouu) for the joint form;
 * Sec. 4.2 minimises over a box Z_ad with a bound-constrained limited-memory
 * BFGS).  The solver runs on the host; every objective / gradient is one
 * saa_objective_grad call (PDE or MR-DINO form, options `opt`).  Variables
 * at a bound whose gradient points out of the box are held for the
 * iteration; the direction is the L-BFGS two-loop recursion over the free
 * variables; the step is backtracked along the projected ray to the Armijo
 * condition.
 * ------------------------------------------------------------------------ */
typedef struct saa_ouu_options {
  int max_iter;        /* outer iterations (default 200) */
  int max_eval;        /* objective evaluations, line searches included (1000) */
  int memory;          /* stored (s, y) pairs, 1..100 (10) */
  int joint_t;         /* 0: t minimised out inside every evaluation (opt->t_mode
                          must be 0); 1: (z, t) is the variable, t unbounded,
                          each evaluation is J_hat(z, t) with t_mode = 1 */
  double pgtol;        /* stop when |P(x - grad) - x|_inf <= pgtol (1e-6) */
  double ftol;         /* stop when an accepted step lowers J by at most
                          ftol max(|J|, 1) (1e-12) */
} saa_ouu_options;

enum { SAA_OUU_PGTOL = 0, SAA_OUU_FTOL = 1, SAA_OUU_MAXITER = 2, SAA_OUU_MAXEVAL = 3, SAA_OUU_LINESEARCH = 4 };

typedef struct saa_ouu_report {
  double J;            /* objective at the returned z */
  double pg_norm;      /* projected-gradient infinity norm there */
  double t;            /* the t of the returned point (t* or the joint t) */
  double seconds;      /* wall time of the solve */
  int iterations;      /* accepted steps */
  int evaluations;     /* saa_objective_grad calls */
  int status;          /* SAA_OUU_*: why the iteration stopped */
  int n_active;        /* components of z held at a bound at the end */
  int n_fallback;      /* evaluations that fell back to the PDE form */
  int pad;
} saa_ouu_report;

/* Defaults above.  SAA_E_INVALID for NULL. */
int saa_ouu_options_default(saa_ouu_options* oo);

/* Minimise J over z in the box [lb, ub] (host arrays of d_Z, either may be
 * NULL for no bound; entries may be +-inf) from the start z (host, d_Z; it
 * is projected onto the box first).  On return z holds the last accepted
 * iterate and *report describes it.  oo may be NULL (defaults).  Returns
 * SAA_OK whatever the stopping reason (see report->status); SAA_E_INVALID
 * for bad arguments (lb > ub, NaN bounds, non-finite z, bad options) before
 * any device work; a failing evaluation's status (e.g. SAA_E_NOCONV) ends the
 * solve with z at the last accepted iterate. */
int saa_ouu_solve(saa_ctx* ctx, int form, const void* model, const saa_options* opt, const saa_ouu_options* oo,
                  const double* lb, const double* ub, double* z, saa_ouu_report* report);

/* Largest sample count of saa_risk_reduce (its per-workgroup counters are 32-bit). */
#define SAA_REDUCE_MAX_N 2147483647LL

/* The risk reduction alone (Sec. 2.1-2.2, eq. (CVaR_saa_ouu) and the chain
 * rule of eq. (ouu_risk_gradient)) on per-sample values the caller already
 * holds: q_dev (N float64) and g_dev (N x d_Z float64, row-major dq_i/dz),
 * z_dev (d_Z float64), all device memory.  opt selects the risk measure and
 * its parameters (beta, eps, alpha, t_mode / t_in, risk, risk_kappa,
 * risk_tau; the solver fields are ignored).  Results go to device memory:
 * out_dev[0] = J, out_dev[1] = dJ/dt, out_dev[2 .. 2 + d_Z) = grad J; t_dev[0]
 * = t* (CVaR), the mean of q (mean + kappa Var), tau (probability of
 * failure), a* (buffered probability of exceedance) or 0 (mean).  Work is
 * enqueued on `hip_stream` (a hipStream_t, NULL = default); the library
 * allocates a workspace of about 2.3 MB for the call and synchronises the
 * stream before releasing it.  SAA_E_INVALID (before any device work) for
 * null pointers, N outside 1 .. SAA_REDUCE_MAX_N, d_Z outside 1 ..
 * SAA_MAX_DZ (64) or invalid options; SAA_E_OOM, SAA_E_DEVICE on failure.
 * Results are bitwise those of the reduction inside saa_objective_grad. */
int saa_risk_reduce(const double* q_dev, const double* g_dev, int64_t N, int d_z, const double* z_dev,
                    const saa_options* opt, double* out_dev, double* t_dev, void* hip_stream);

/* saa_risk_reduce for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, but the workspace is a static
 * device array of SAA_REDUCE_SCRATCH_BYTES (about 2.3 MB) that each GPU the
 * library runs on holds until the process ends.  Nothing is allocated or
 * freed and the stream is not synchronised: results are ready when the work
 * enqueued on `hip_stream` completes.  Every call on one GPU shares that
 * GPU's workspace (the kernels re-initialise what they read), so calls that
 * overlap on one GPU (several streams or threads) race and must be
 * serialised by the caller.  Sizes beyond N = SAA_REDUCE_MAX_N or d_Z = 64
 * return SAA_E_INVALID before any device work; SAA_E_DEVICE if the
 * workspace's device address cannot be obtained or a launch fails. */
#define SAA_REDUCE_SCRATCH_BYTES 2283552
int saa_risk_reduce_noalloc(const double* q_dev, const double* g_dev, int64_t N, int d_z, const double* z_dev,
                            const saa_options* opt, double* out_dev, double* t_dev, void* hip_stream);

/* Autotuning cache.  Launch shapes are chosen by timing the candidates at the
 * first use for a given size and recorded per device (architecture and
 * compute-unit count) in a text file of "key value" lines that later
 * processes reuse: $SAA_TUNE_CACHE ("off" keeps choices in memory only), else
 * $HOME/.cache/saa_tune.txt.  Keys (the device tag is added internally):
 *   mlp/w<width>/p<1 BF16 | 2 FP8>/N<N rounded up to a power of two>:
 *     tile shape of the fused surrogate kernel, 0..2 at width 256 (8 waves x
 *     64 samples, 8 x 32, 4 x 64), 0..1 at width 512 (8 x 32, 16 x 32); every
 *     shape gives bitwise the same results;
 *   state3/p<prec>/n<n>/N<N>, adjoint3/p<prec>/n<n>/N<N>: threads per sample
 *     of the 3D kernels (256, 512, 1024).
 * saa_tune_get returns SAA_E_INVALID when the key has no recorded choice;
 * saa_tune_set records one (it takes effect for contexts without an installed
 * choice; see saa_ctx_launch3).  Keys may not contain spaces. */
int saa_tune_get(const char* key, int* value);
int saa_tune_set(const char* key, int value);

/* Per-sample status of the last saa_objective_grad, saa_per_sample or
 * saa_solve_states call on this context.  Host arrays of N entries each (any
 * may be NULL): flags (bit 1: Newton not converged, 2: an inner PCG hit
 * max_lin or broke down, 4: adjoint / linearised defect correction not
 * converged, 8: non-finite update), Newton iterations, PCG iterations of the
 * state solve, PCG iterations of the adjoint / linearised solves.  N is the
 * number of installed samples.  Synchronises the context's stream. */
int saa_sample_status(saa_ctx* ctx, int* flags, int* newton_iters, int* lin_iters, int* adj_lin_iters);

/* PDE-form objective and gradient of `count` 2D contexts (1..4, any grid
 * sizes, all on one stream, distinct) at their controls z[k] (host, d_Z of
 * context k): one state launch and one adjoint launch serve all of them
 * (the samples of context k take a contiguous range of the launch's
 * workgroups), with each context's CVaR reduction in between.  J[k],
 * grad_z[k] (host) and reports[k] (may be NULL) are the results of
 * saa_objective_grad on each context alone, bit for bit.  opt applies to
 * all (PDE precisions only; timing must be 0).  SAA_E_INVALID for a 3D
 * context, a repeated context, contexts on different streams or a bad
 * argument; otherwise the worst status of the contexts. */
int saa_objective_grad_multi(int count, saa_ctx* const* ctx, const double* const* z, const saa_options* opt,
                             double* J, double* const* grad_z, saa_report* reports);

/* Threads per sample of the 3D state and adjoint kernels for the PDE
 * precision prec (SAA_FP64, SAA_FP32 or SAA_FP32_DC64).  The kernels exist
 * for 256, 512 and 1024 threads; while a size is 0 the next call of that
 * precision times the three on the context's stream (HIP events; the
 * launches recompute all their outputs, so results do not depend on the
 * extra runs) and records the fastest.  set = 0: *bs_state and *bs_adjoint
 * receive the recorded sizes (0 = not chosen yet); set = 1: they are
 * installed (256, 512, 1024, or 0 to time again).  SAA_E_INVALID for a 2D
 * context, NULL pointers, another prec or another size. */
int saa_ctx_launch3(saa_ctx* ctx, int prec, int* bs_state, int* bs_adjoint, int set);

#ifdef __cplusplus
}
#endif

#endif /* SAA_H */
