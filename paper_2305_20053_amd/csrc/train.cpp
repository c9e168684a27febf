// MR-DINO construction (paper Sec. 3.3-3.4, Sec. 4.2.1): training data from
// the GPU PDE path, mass-weighted POD, reduced projections, and the
// derivative-informed training loop.  Every numerical step runs in the
// kernels of train.hip / pde.hip / mlp.hip, except the eigendecomposition of
// the small n_pod x n_pod Gram matrix (host, linalg.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "ctx.h"
#include "mlp.h"
#include "model.h"

extern "C" int saa_sym_eig(int n, const double* A, double* w, double* V);
extern "C" int saa_sym_eig_gpu(int n, const double* A_dev, double* w, double* V_dev, void* hip_stream, int* sweeps);

#include <rocblas/rocblas.h>

namespace saa_launch {
int gemm_mfma(bool bf16, bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda, const float* B,
              int ldb, float beta, float* C, int ldc, float* ws, int64_t ws_floats, hipStream_t st);
int dgemm(rocblas_handle h, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st);
rocblas_handle blas_create();
void blas_destroy(rocblas_handle h);
void mass_rows(const double* U, int64_t ldu, const double* ubar, double* out, int64_t ldo, int n, int64_t rows,
               hipStream_t st);
void mass_rows3(const double* V, int64_t ldv, const double* vbar, double* out, int64_t ldo, int n, int64_t rows,
                hipStream_t st);
void colmean(const double* X, int64_t rows, int cols, int64_t ldx, double* out, hipStream_t st);
void train_inputs(const double* xi, int nkl, const int* order, int r_m, const double* Z, int d_z, int64_t N, float* X,
                  hipStream_t st);
void gather_rows(const float* src, int64_t width, const int* idx, int B, float* dst, hipStream_t st);
void bias_gelu(float* A, const float* bias, float* H, int64_t rows, int cols, int act, hipStream_t st);
void tangent0(const float* W0, int ldw, int r_m, int d_z, const float* A, int B, int W, float* JA, float* JH,
              hipStream_t st);
void tangent_scale(const float* JA, const float* A, int B, int d_z, int W, float* JH, hipStream_t st);
int residual(const float* P, const float* Y, int64_t n, float scale, float y_scale, float* G, double* part,
             hipStream_t st);
void scale(float* x, int64_t n, float f, hipStream_t st);
void layer_back(float* gH, float* gJH, const float* A, const float* JA, int B, int d_z, int W, int dino,
                hipStream_t st);
void colsum(const float* X, int64_t rows, int cols, float* out, int accumulate, hipStream_t st);
void w0z_grad(const float* gJA, int B, int d_z, int W, int r_m, int ldw, float* dW0, hipStream_t st);
void adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps, float c1,
          float c2, hipStream_t st);
void sum_parts(const double* part, int n, double* out, int accumulate, hipStream_t st);
void d2f(const double* x, float* y, int64_t n, hipStream_t st);
void center_rows(const double* U, const double* ubar, double* out, int64_t cols, int64_t rows, hipStream_t st);
int sumsq(const float* x, int64_t n, double* part, hipStream_t st);
}  // namespace saa_launch


using namespace saa_rt;

struct mrdino_data {
  int dim = 2, n = 0, r_m = 0, d_z = 0, r_u = 0, n_pod = 0;
  int64_t N = 0, d_u = 0;
  DevBuf X, Y, JY;          // FP32 training arrays: N x (r_m + d_z), N x r_u, (N d_z) x r_u
  DevBuf PhiT, ubar;        // FP64 r_u x d_U (M-orthonormal rows), d_U
  std::vector<double> lam;  // Gram eigenvalues, decreasing
  std::vector<double> c;    // reduced QoI terms
  double c0 = 0.0;
  hipStream_t st = nullptr;
  rocblas_handle blas = nullptr;   // FP64 POD products (library GEMM), owned
  double y_scale = 0.0;            // training output scale (0: not yet computed)
  ~mrdino_data() { saa_launch::blas_destroy(blas); }
};

namespace {

// Training workspace of one batch size (per model).
struct TrainWs {
  int B = 0;
  DevBuf Xb, Yb, JYb, idx;
  DevBuf A[MLP_MAX_DEPTH], H[MLP_MAX_DEPTH], JA[MLP_MAX_DEPTH], JH[MLP_MAX_DEPTH];
  DevBuf P, JP, gP, gJP, gH[2], gJH[2];
  DevBuf grad, m, v, parts, loss;
  DevBuf gws;               // partial products of k-split GEMMs
  int64_t gws_floats = 0;
};

struct TrainState {
  TrainWs ws;
  int64_t step = 0;    // Adam steps taken
  int64_t epoch = 0;   // epochs completed (the learning-rate schedule's clock)
  uint64_t rng = 0;    // minibatch-order stream
  bool started = false;
};

TrainState* train_state(mrdino_model* m) {
  if (!m->train) m->train = new (std::nothrow) TrainState();
  return (TrainState*)m->train;
}


int alloc_ws(mrdino_model* mdl, int B) {
  TrainState* ts = train_state(mdl);
  if (!ts) return SAA_E_OOM;
  TrainWs& w = ts->ws;
  if (w.B >= B) return SAA_OK;
  const mrdino_dims& d = mdl->dims;
  const int W = d.width, in = d.r_m + d.d_z;
  const size_t f = sizeof(float);
  const size_t bw = (size_t)B * W * f, tw = (size_t)B * d.d_z * W * f;
  int rc = SAA_OK;
  hipStream_t st = mdl->st;
  if (!rc) rc = w.Xb.alloc_zero((size_t)B * in * f, st);
  if (!rc) rc = w.Yb.alloc_zero((size_t)B * d.r_u * f, st);
  if (!rc) rc = w.JYb.alloc_zero((size_t)B * d.d_z * d.r_u * f, st);
  if (!rc) rc = w.idx.alloc_zero((size_t)B * sizeof(int), st);
  for (int l = 0; l < d.depth && !rc; ++l) {
    rc = w.A[l].alloc_zero(bw, st);
    if (!rc) rc = w.H[l].alloc_zero(bw, st);
    if (!rc) rc = w.JA[l].alloc_zero(tw, st);
    if (!rc) rc = w.JH[l].alloc_zero(tw, st);
  }
  if (!rc) rc = w.P.alloc_zero((size_t)B * d.r_u * f, st);
  if (!rc) rc = w.JP.alloc_zero((size_t)B * d.d_z * d.r_u * f, st);
  if (!rc) rc = w.gP.alloc_zero((size_t)B * d.r_u * f, st);
  if (!rc) rc = w.gJP.alloc_zero((size_t)B * d.d_z * d.r_u * f, st);
  for (int k = 0; k < 2 && !rc; ++k) {
    rc = w.gH[k].alloc_zero(bw, st);
    if (!rc) rc = w.gJH[k].alloc_zero(tw, st);
  }
  if (!rc) rc = w.grad.alloc_zero(f * mdl->n_params, st);
  if (!rc && !w.m.p) rc = w.m.alloc_zero(f * mdl->n_params, st);
  if (!rc && !w.v.p) rc = w.v.alloc_zero(f * mdl->n_params, st);
  if (!rc) rc = w.parts.alloc_zero(sizeof(double) * (((size_t)B * d.d_z * d.r_u + 1023) / 1024 + 16), st);
  if (!rc) rc = w.loss.alloc_zero(sizeof(double) * 4, st);
  // up to 16 k slices of the largest weight-gradient product
  const int64_t wmax = std::max<int64_t>((int64_t)W * std::max(W, in), (int64_t)d.r_u * W);
  if (!rc && w.gws_floats < 16 * wmax) {
    rc = w.gws.alloc(sizeof(float) * 16 * wmax);
    w.gws_floats = rc ? 0 : 16 * wmax;
  }
  if (!rc) w.B = B;
  return rc;
}

float* F(DevBuf& b) { return (float*)b.p; }

// One training product C = alpha op(A) op(B) + beta C on the MFMA kernels,
// operands in BF16 (bf) or FP32, FP32 accumulation.
struct Mm {
  TrainWs& w;
  bool bf;
  hipStream_t st;
  int rc = SAA_OK;
  void operator()(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float beta,
                  float* C, int ldc) {
    const int e = saa_launch::gemm_mfma(bf, ta, tb, M, N, K, 1.0f, A, lda, B, ldb, beta, C, ldc, (float*)w.gws.p,
                                        w.gws_floats, st);
    if (!rc) rc = e;
  }
};

// Forward (and, with dino, forward-mode tangents) of the batch in ws.Xb:
// a_l = H_{l-1} W_l^T, h_l = GELU(a_l + b_l); tangents J_l = GELU'(a_l) (J_{l-1} W_l^T),
// J_0 = GELU'(a_0) W_0[:, r_m:]^T; phi = H W^T + b, dphi/dz = J W^T.
int forward(mrdino_model* mdl, TrainWs& w, int B, int dino, bool bf) {
  const mrdino_dims& d = mdl->dims;
  const int W = d.width, in = d.r_m + d.d_z, dz = d.d_z;
  const float* P = (const float*)mdl->master.p;
  hipStream_t st = mdl->st;
  Mm mm{w, bf, st};
  const float* hin = F(w.Xb);
  int kin = in;
  for (int l = 0; l < d.depth; ++l) {
    mm(false, true, B, W, kin, hin, kin, P + mdl->off_w[l], kin, 0.0f, F(w.A[l]), W);
    saa_launch::bias_gelu(F(w.A[l]), P + mdl->off_b[l], F(w.H[l]), B, W, 1, st);
    hin = F(w.H[l]);
    kin = W;
  }
  mm(false, true, B, d.r_u, W, hin, W, P + mdl->off_w[d.depth], W, 0.0f, F(w.P), d.r_u);
  saa_launch::bias_gelu(F(w.P), P + mdl->off_b[d.depth], nullptr, B, d.r_u, 0, st);
  if (!dino) return mm.rc;
  saa_launch::tangent0(P + mdl->off_w[0], in, d.r_m, dz, F(w.A[0]), B, W, F(w.JA[0]), F(w.JH[0]), st);
  for (int l = 1; l < d.depth; ++l) {
    mm(false, true, B * dz, W, W, F(w.JH[l - 1]), W, P + mdl->off_w[l], W, 0.0f, F(w.JA[l]), W);
    saa_launch::tangent_scale(F(w.JA[l]), F(w.A[l]), B, dz, W, F(w.JH[l]), st);
  }
  mm(false, true, B * dz, d.r_u, W, F(w.JH[d.depth - 1]), W, P + mdl->off_w[d.depth], W, 0.0f, F(w.JP), d.r_u);
  return mm.rc;
}

// Loss (ws.loss[0] = state part, [1] = Jacobian part, unnormalised sums) and,
// with want_grad, the gradient of L = (1/B) sum (|e|^2 + |E_J|_F^2) into ws.grad.
int loss_grad(mrdino_model* mdl, TrainWs& w, int B, int dino, bool want_grad, bool bf, float y_scale = 1.0f) {
  const mrdino_dims& d = mdl->dims;
  const int W = d.width, in = d.r_m + d.d_z, dz = d.d_z;
  const float* P = (const float*)mdl->master.p;
  hipStream_t st = mdl->st;
  double* loss = (double*)w.loss.p;
  int rc = forward(mdl, w, B, dino, bf);
  if (rc) return rc;
  const float sc = 2.0f / (float)B;
  int nb = saa_launch::residual(F(w.P), F(w.Yb), (int64_t)B * d.r_u, sc, y_scale, F(w.gP), (double*)w.parts.p, st);
  saa_launch::sum_parts((double*)w.parts.p, nb, loss + 0, 0, st);
  if (dino) {
    nb = saa_launch::residual(F(w.JP), F(w.JYb), (int64_t)B * dz * d.r_u, sc, y_scale, F(w.gJP),
                              (double*)w.parts.p, st);
    saa_launch::sum_parts((double*)w.parts.p, nb, loss + 1, 0, st);
  } else {
    saa_launch::sum_parts((double*)w.parts.p, 0, loss + 1, 0, st);   // zero
  }
  if (!want_grad) return check_hip(hipGetLastError());
  Mm mm{w, bf, st};
  float* G = F(w.grad);
  const int L = d.depth;
  // output layer: dW = gP^T H (+ gJP^T JH), db = column sums of gP
  mm(true, false, d.r_u, W, B, F(w.gP), d.r_u, F(w.H[L - 1]), W, 0.0f, G + mdl->off_w[L], W);
  if (dino) mm(true, false, d.r_u, W, B * dz, F(w.gJP), d.r_u, F(w.JH[L - 1]), W, 1.0f, G + mdl->off_w[L], W);
  saa_launch::colsum(F(w.gP), B, d.r_u, G + mdl->off_b[L], 0, st);
  int cur = 0;
  mm(false, false, B, W, d.r_u, F(w.gP), d.r_u, P + mdl->off_w[L], W, 0.0f, F(w.gH[cur]), W);
  if (dino) mm(false, false, B * dz, W, d.r_u, F(w.gJP), d.r_u, P + mdl->off_w[L], W, 0.0f, F(w.gJH[cur]), W);
  for (int l = L - 1; l >= 0; --l) {
    saa_launch::layer_back(F(w.gH[cur]), F(w.gJH[cur]), F(w.A[l]), F(w.JA[l]), B, dz, W, dino, st);
    const int kin = (l == 0) ? in : W;
    const float* hprev = (l == 0) ? F(w.Xb) : F(w.H[l - 1]);
    mm(true, false, W, kin, B, F(w.gH[cur]), W, hprev, kin, 0.0f, G + mdl->off_w[l], kin);
    if (dino) {
      if (l >= 1)
        mm(true, false, W, W, B * dz, F(w.gJH[cur]), W, F(w.JH[l - 1]), W, 1.0f, G + mdl->off_w[l], W);
      else
        saa_launch::w0z_grad(F(w.gJH[cur]), B, dz, W, d.r_m, in, G + mdl->off_w[0], st);
    }
    saa_launch::colsum(F(w.gH[cur]), B, W, G + mdl->off_b[l], 0, st);
    if (l >= 1) {
      const int nxt = cur ^ 1;
      mm(false, false, B, W, W, F(w.gH[cur]), W, P + mdl->off_w[l], W, 0.0f, F(w.gH[nxt]), W);
      if (dino) mm(false, false, B * dz, W, W, F(w.gJH[cur]), W, P + mdl->off_w[l], W, 0.0f, F(w.gJH[nxt]), W);
      cur = nxt;
    }
  }
  return mm.rc ? mm.rc : check_hip(hipGetLastError());
}

// Gather the minibatch rows idx_dev[0..B) (device indices) of the data set.
void load_batch(mrdino_model* mdl, mrdino_data* D, TrainWs& w, const int* idx_dev, int B) {
  const mrdino_dims& d = mdl->dims;
  saa_launch::gather_rows(F(D->X), d.r_m + d.d_z, idx_dev, B, F(w.Xb), mdl->st);
  saa_launch::gather_rows(F(D->Y), d.r_u, idx_dev, B, F(w.Yb), mdl->st);
  saa_launch::gather_rows(F(D->JY), (int64_t)d.d_z * d.r_u, idx_dev, B, F(w.JYb), mdl->st);
}

// 2^round(log2(rms)) of the reduced training states (1 if they vanish).
int output_scale(mrdino_data* D, hipStream_t st, double* sigma) {
  if (D->y_scale > 0.0) {
    *sigma = D->y_scale;
    return SAA_OK;
  }
  const int64_t n = D->N * D->r_u;
  DevBuf parts, acc;
  int rc = parts.alloc(sizeof(double) * ((n + 1023) / 1024 + 1));
  if (!rc) rc = acc.alloc(sizeof(double));
  if (rc) return rc;
  const int nb = saa_launch::sumsq((const float*)D->Y.p, n, (double*)parts.p, st);
  saa_launch::sum_parts((double*)parts.p, nb, (double*)acc.p, 0, st);
  double ss = 0.0;
  if ((rc = check_hip(hipMemcpyAsync(&ss, acc.p, sizeof(double), hipMemcpyDeviceToHost, st))) ||
      (rc = check_hip(hipStreamSynchronize(st))))
    return rc;
  const double rms = std::sqrt(ss / (double)n);
  D->y_scale = (rms > 0.0 && std::isfinite(rms)) ? std::ldexp(1.0, (int)std::lround(std::log2(rms))) : 1.0;
  *sigma = D->y_scale;
  return SAA_OK;
}

bool compatible(const mrdino_model* m, const mrdino_data* D) {
  return m->dims.r_m == D->r_m && m->dims.d_z == D->d_z && m->dims.r_u == D->r_u;
}

// splitmix64 (Steele, Lea, Flood 2014): the minibatch order generator.
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

void saa_model_free_train(mrdino_model* m) {
  delete (TrainState*)m->train;
  m->train = nullptr;
}

int saa_model_get_train_state(const mrdino_model* m, TrainCheckpoint& ck) {
  const TrainState* ts = (const TrainState*)m->train;
  ck.present = ts && ts->started && ts->ws.m.p && ts->ws.v.p;
  if (!ck.present) return SAA_OK;
  ck.step = ts->step;
  ck.epoch = ts->epoch;
  ck.rng = ts->rng;
  ck.m.resize(m->n_params);
  ck.v.resize(m->n_params);
  int rc = check_hip(hipMemcpyAsync(ck.m.data(), ts->ws.m.p, sizeof(float) * m->n_params, hipMemcpyDeviceToHost, m->st));
  if (!rc)
    rc = check_hip(hipMemcpyAsync(ck.v.data(), ts->ws.v.p, sizeof(float) * m->n_params, hipMemcpyDeviceToHost, m->st));
  if (!rc) rc = check_hip(hipStreamSynchronize(m->st));
  return rc;
}

int saa_model_set_train_state(mrdino_model* m, const TrainCheckpoint& ck) {
  if (!ck.present) return SAA_OK;
  if ((int64_t)ck.m.size() != m->n_params || (int64_t)ck.v.size() != m->n_params) return SAA_E_INVALID;
  TrainState* ts = train_state(m);
  if (!ts) return SAA_E_OOM;
  TrainWs& w = ts->ws;
  int rc = SAA_OK;
  if (!w.m.p) rc = w.m.alloc(sizeof(float) * m->n_params);
  if (!rc && !w.v.p) rc = w.v.alloc(sizeof(float) * m->n_params);
  if (!rc)
    rc = check_hip(hipMemcpyAsync(w.m.p, ck.m.data(), sizeof(float) * m->n_params, hipMemcpyHostToDevice, m->st));
  if (!rc)
    rc = check_hip(hipMemcpyAsync(w.v.p, ck.v.data(), sizeof(float) * m->n_params, hipMemcpyHostToDevice, m->st));
  if (!rc) rc = check_hip(hipStreamSynchronize(m->st));
  if (rc) return rc;
  ts->step = ck.step;
  ts->epoch = ck.epoch;
  ts->rng = ck.rng;
  ts->started = true;
  return SAA_OK;
}

// Consistent mass on interior rows (P1 on the square, Q1 on the cube):
// out[s] = M_II (U[s] - ubar), rows of the interior grid.
static void mass_rows_dim(int dim, const double* U, int64_t ldu, const double* ubar, double* out, int64_t ldo, int n,
                          int64_t rows, hipStream_t st) {
  if (dim == 3) saa_launch::mass_rows3(U, ldu, ubar, out, ldo, n, rows, st);
  else saa_launch::mass_rows(U, ldu, ubar, out, ldo, n, rows, st);
}

// Reduced QoI terms of the tracking functional for a target with interior
// mass vector mt (node layout) and ut^T M ut = ctt (Sec. 3.3):
//   c = Phi^T (M ubar - (M ut)_I),  c0 = ubar^T M ubar - 2 ubar . (M ut)_I + ctt - |c|^2,
// so that |u - ut|_M^2 = |phi + c|^2 + c0 for u = ubar + Phi phi (Phi M-orthonormal).
static int qoi_terms(const mrdino_data* D, const std::vector<double>& mt, double ctt, std::vector<double>& c_out,
                     double& c0_out) {
  const int64_t du = D->d_u;
  const int r_u = D->r_u;
  hipStream_t st = D->st;
  saa_rt::DevBuf Mub, vdev, cdev;
  int rc;
  if ((rc = Mub.alloc(sizeof(double) * du)) || (rc = vdev.alloc(sizeof(double) * du)) ||
      (rc = cdev.alloc(sizeof(double) * r_u)))
    return rc;
  mass_rows_dim(D->dim, (double*)D->ubar.p, du, nullptr, (double*)Mub.p, du, D->n, 1, st);
  std::vector<double> ub(du), mub(du);
  if ((rc = check_hip(hipMemcpyAsync(ub.data(), D->ubar.p, sizeof(double) * du, hipMemcpyDeviceToHost, st))) ||
      (rc = check_hip(hipMemcpyAsync(mub.data(), Mub.p, sizeof(double) * du, hipMemcpyDeviceToHost, st))) ||
      (rc = check_hip(hipStreamSynchronize(st))))
    return rc;
  // (M u_t) at the interior nodes, interior order
  const int nn = D->n;
  std::vector<double> v(du);
  double quad = 0.0, cross = 0.0;
  for (int64_t p = 0; p < du; ++p) {
    const int64_t i = p % (nn - 1) + 1, j = (p / (nn - 1)) % (nn - 1) + 1, k = p / ((int64_t)(nn - 1) * (nn - 1)) + 1;
    const int64_t node = D->dim == 3 ? i + (nn + 1) * (j + (int64_t)(nn + 1) * k) : j * (nn + 1) + i;
    const double m = mt[(size_t)node];
    v[p] = mub[p] - m;
    quad += ub[p] * mub[p];
    cross += ub[p] * m;
  }
  if ((rc = check_hip(hipMemcpyAsync(vdev.p, v.data(), sizeof(double) * du, hipMemcpyHostToDevice, st)))) return rc;
  if ((rc = saa_launch::dgemm(D->blas, false, false, r_u, 1, (int)du, 1.0, (double*)D->PhiT.p, (int)du,
                              (double*)vdev.p, 1, 0.0, (double*)cdev.p, 1, st)))
    return rc;
  c_out.assign(r_u, 0.0);
  if ((rc = check_hip(hipMemcpyAsync(c_out.data(), cdev.p, sizeof(double) * r_u, hipMemcpyDeviceToHost, st))) ||
      (rc = check_hip(hipStreamSynchronize(st))))
    return rc;
  double cc = 0.0;
  for (double x : c_out) cc += x * x;
  c0_out = quad - 2.0 * cross + ctt - cc;
  return check_hip(hipGetLastError());
}

extern "C" {

int mrdino_data_create(saa_ctx* c, const double* Z_dev, int r_m, int r_u, int n_pod, const saa_options* opt,
                       const mrdino_data* basis, mrdino_data** out, saa_report* rep) {
  if (!c || !Z_dev || !opt || !out) return SAA_E_INVALID;
  *out = nullptr;
  const int64_t N = c->N, du = c->d_u;
  const int dz = c->dz;
  if (basis) {
    if (basis->d_u != du || basis->r_u != r_u || basis->d_z != dz || basis->n != c->prob.n ||
        basis->dim != (c->d3 ? 3 : 2))
      return SAA_E_INVALID;
    n_pod = basis->n_pod;
    if (N < 1 || r_m < 1 || r_m > c->n_kl) return SAA_E_INVALID;
  } else if (N < 2 || r_m < 1 || r_m > c->n_kl || r_u < 1 || n_pod < r_u || n_pod > N || n_pod > 8192) {
    return SAA_E_INVALID;
  }
  hipStream_t st = c->st;
  mrdino_data* D = new (std::nothrow) mrdino_data();
  if (!D) return SAA_E_OOM;
  D->dim = c->d3 ? 3 : 2;
  D->n = c->prob.n;
  D->r_m = r_m;
  D->d_z = dz;
  D->r_u = r_u;
  D->n_pod = n_pod;
  D->N = N;
  D->d_u = du;
  D->st = st;
  auto fail = [&](int rc) {
    delete D;
    return rc;
  };
  if (!(D->blas = saa_launch::blas_create())) return fail(SAA_E_DEVICE);
  DevBuf U, dUdz, Dm, MD, G, Vs, MPhiT, Yd, JYd;
  // control Jacobians: d_Z forward solves, or r_u adjoint solves (Sec. 3.4);
  // on the cube only forward solves, projected chunk by chunk (a full
  // N x d_Z x d_U array would not fit)
  if (c->d3 && opt->jac_mode == SAA_JAC_ADJOINT) return fail(SAA_E_INVALID);
  const bool adj = !c->d3 && (opt->jac_mode == SAA_JAC_ADJOINT || (opt->jac_mode == SAA_JAC_AUTO && dz >= r_u));
  int rc = U.alloc(sizeof(double) * N * du);
  if (!rc && !adj && !c->d3) rc = dUdz.alloc(sizeof(double) * N * dz * du);
  if (rc) return fail(rc);
  // 1. states (and, on the square, forward-mode control Jacobians) of the training samples
  rc = saa_solve_states(c, Z_dev, opt, (double*)U.p, nullptr, (adj || c->d3) ? nullptr : (double*)dUdz.p, rep);
  if (rc) return fail(rc);
  if (basis) {  // held-out data: reuse the training basis and QoI terms
    if ((rc = D->ubar.alloc(sizeof(double) * du)) || (rc = D->PhiT.alloc(sizeof(double) * r_u * du)) ||
        (rc = MPhiT.alloc(sizeof(double) * r_u * du)))
      return fail(rc);
    if ((rc = check_hip(hipMemcpyAsync(D->ubar.p, basis->ubar.p, sizeof(double) * du, hipMemcpyDeviceToDevice, st))) ||
        (rc = check_hip(hipMemcpyAsync(D->PhiT.p, basis->PhiT.p, sizeof(double) * r_u * du, hipMemcpyDeviceToDevice,
                                       st))))
      return fail(rc);
    D->lam = basis->lam;
    mass_rows_dim(D->dim, (double*)D->PhiT.p, du, nullptr, (double*)MPhiT.p, du, D->n, r_u, st);
  } else {
  // 2. weighted POD from the first n_pod states (Sec. 3.3; the paper uses 512)
  if ((rc = D->ubar.alloc(sizeof(double) * du)) || (rc = Dm.alloc(sizeof(double) * n_pod * du)) ||
      (rc = MD.alloc(sizeof(double) * n_pod * du)) || (rc = G.alloc(sizeof(double) * n_pod * n_pod)))
    return fail(rc);
  saa_launch::colmean((double*)U.p, n_pod, (int)du, du, (double*)D->ubar.p, st);
  saa_launch::center_rows((double*)U.p, (double*)D->ubar.p, (double*)Dm.p, du, n_pod, st);
  mass_rows_dim(D->dim, (double*)Dm.p, du, nullptr, (double*)MD.p, du, D->n, n_pod, st);
  if ((rc = saa_launch::dgemm(D->blas, false, true, n_pod, n_pod, (int)du, 1.0, (double*)Dm.p, (int)du,
                              (double*)MD.p, (int)du, 0.0, (double*)G.p, n_pod, st)))
    return fail(rc);
  std::vector<double> V((size_t)n_pod * n_pod);
  D->lam.assign(n_pod, 0.0);
  {  // eigenpairs of the Gram matrix on the GPU (parallel Jacobi)
    DevBuf Vd;
    if ((rc = Vd.alloc(sizeof(double) * V.size())) ||
        (rc = saa_sym_eig_gpu(n_pod, (const double*)G.p, D->lam.data(), (double*)Vd.p, st, nullptr)) ||
        (rc = check_hip(hipMemcpyAsync(V.data(), Vd.p, sizeof(double) * V.size(), hipMemcpyDeviceToHost, st))) ||
        (rc = check_hip(hipStreamSynchronize(st))))
      return fail(rc);
  }
  if (!(D->lam[r_u - 1] > 1e-14 * D->lam[0])) return fail(SAA_E_INVALID);   // rank below r_u
  std::vector<double> vs((size_t)n_pod * r_u);
  for (int col = 0; col < r_u; ++col) {
    int piv = 0;
    for (int r = 1; r < n_pod; ++r)
      if (std::fabs(V[(size_t)r * n_pod + col]) > std::fabs(V[(size_t)piv * n_pod + col])) piv = r;
    const double sgn = V[(size_t)piv * n_pod + col] < 0.0 ? -1.0 : 1.0;
    const double sc = sgn / std::sqrt(D->lam[col]);
    for (int r = 0; r < n_pod; ++r) vs[(size_t)r * r_u + col] = sc * V[(size_t)r * n_pod + col];
  }
  if ((rc = Vs.alloc(sizeof(double) * vs.size())) || (rc = D->PhiT.alloc(sizeof(double) * r_u * du)) ||
      (rc = MPhiT.alloc(sizeof(double) * r_u * du)))
    return fail(rc);
  if ((rc = check_hip(hipMemcpyAsync(Vs.p, vs.data(), sizeof(double) * vs.size(), hipMemcpyHostToDevice, st))))
    return fail(rc);
  // Phi^T = (V_r Lambda_r^{-1/2})^T D  (rows M-orthonormal)
  if ((rc = saa_launch::dgemm(D->blas, true, false, r_u, (int)du, n_pod, 1.0, (double*)Vs.p, r_u, (double*)Dm.p,
                              (int)du, 0.0, (double*)D->PhiT.p, (int)du, st)))
    return fail(rc);
  mass_rows_dim(D->dim, (double*)D->PhiT.p, du, nullptr, (double*)MPhiT.p, du, D->n, r_u, st);
  Dm.release();
  MD.release();
  }
  // 3. reduced data: y = Phi^T M (u - ubar), J_r = Phi^T M du/dz (eq. (projected_sensitivity))
  if ((rc = Yd.alloc(sizeof(double) * N * r_u)) || (rc = JYd.alloc(sizeof(double) * N * dz * r_u))) return fail(rc);
  saa_launch::center_rows((double*)U.p, (double*)D->ubar.p, (double*)U.p, du, N, st);
  if ((rc = saa_launch::dgemm(D->blas, false, true, (int)N, r_u, (int)du, 1.0, (double*)U.p, (int)du,
                              (double*)MPhiT.p, (int)du, 0.0, (double*)Yd.p, r_u, st)))
    return fail(rc);
  if (adj) {   // J_r = (A^{-1} M Phi)^T F, from the states still held by the context
    if ((rc = saa_rt::adjoint_jacobians(c, opt, (const double*)MPhiT.p, r_u, (double*)JYd.p))) return fail(rc);
  } else if (c->d3) {   // du/dz of a chunk of samples, then J_r = (M Phi)^T du/dz for the chunk
    // one workgroup per sample: chunks of at least a CU round (256 samples)
    // keep every CU busy; 16 GiB of du/dz per chunk (about 320 samples at 48^3)
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(N, ((int64_t)16 << 30) / (8 * dz * du)));
    if ((rc = dUdz.alloc(sizeof(double) * chunk * dz * du))) return fail(rc);
    for (int64_t s0 = 0; s0 < N && !rc; s0 += chunk) {
      const int64_t ns = std::min<int64_t>(chunk, N - s0);
      rc = saa_rt::jacobians3(c, opt, s0, ns, (double*)dUdz.p, du);
      if (!rc)
        rc = saa_launch::dgemm(D->blas, false, true, (int)(ns * dz), r_u, (int)du, 1.0, (double*)dUdz.p, (int)du,
                               (double*)MPhiT.p, (int)du, 0.0, (double*)JYd.p + s0 * dz * r_u, r_u, st);
    }
    if (rc) return fail(rc);
  } else {
    if ((rc = saa_launch::dgemm(D->blas, false, true, (int)(N * dz), r_u, (int)du, 1.0, (double*)dUdz.p, (int)du,
                                (double*)MPhiT.p, (int)du, 0.0, (double*)JYd.p, r_u, st)))
      return fail(rc);
  }
  if ((rc = D->X.alloc(sizeof(float) * N * (r_m + dz))) || (rc = D->Y.alloc(sizeof(float) * N * r_u)) ||
      (rc = D->JY.alloc(sizeof(float) * N * dz * r_u)))
    return fail(rc);
  saa_launch::d2f((double*)Yd.p, (float*)D->Y.p, N * r_u, st);
  saa_launch::d2f((double*)JYd.p, (float*)D->JY.p, N * dz * r_u, st);
  saa_launch::train_inputs((const double*)c->xi.p, (int)c->n_kl, (const int*)c->order.p, r_m, Z_dev, dz, N,
                           (float*)D->X.p, st);
  // 4. reduced QoI terms c, c0 for the context's target (Sec. 3.3)
  if ((rc = qoi_terms(D, c->mt_host, c->ctt, D->c, D->c0))) return fail(rc);
  if ((rc = check_hip(hipGetLastError()))) return fail(rc);
  *out = D;
  return SAA_OK;
}

void mrdino_data_free(mrdino_data* D) {
  if (!D) return;
  (void)hipStreamSynchronize(D->st);
  delete D;
}

int mrdino_data_qoi(const mrdino_data* D, int target, double u_target, double* c, double* c0) {
  if (!D || !c || !c0 || !std::isfinite(u_target)) return SAA_E_INVALID;
  if (target != SAA_TARGET_CONST && target != SAA_TARGET_SIN && target != SAA_TARGET_QUAD) return SAA_E_INVALID;
  std::vector<double> mt, cv;
  double ctt = 0.0, c0v = 0.0;
  if (D->dim == 3) saa_rt::target_mass3(D->n, target, u_target, mt, ctt);
  else saa_rt::target_mass(D->n, target, u_target, mt, ctt);
  const int rc = qoi_terms(D, mt, ctt, cv, c0v);
  if (rc) return rc;
  for (int k = 0; k < D->r_u; ++k) c[k] = cv[k];
  *c0 = c0v;
  return SAA_OK;
}

int mrdino_data_info(const mrdino_data* D, int64_t* N, double* c, double* c0, double* lam) {
  if (!D) return SAA_E_INVALID;
  if (N) *N = D->N;
  if (c) std::memcpy(c, D->c.data(), sizeof(double) * D->r_u);
  if (c0) *c0 = D->c0;
  if (lam) std::memcpy(lam, D->lam.data(), sizeof(double) * D->n_pod);
  return SAA_OK;
}

int mrdino_data_get(const mrdino_data* D, int which, void* host, int64_t n) {
  if (!D || !host) return SAA_E_INVALID;
  const DevBuf* b = nullptr;
  size_t bytes = 0;
  switch (which) {
    case 0: b = &D->X; bytes = sizeof(float) * D->N * (D->r_m + D->d_z); break;
    case 1: b = &D->Y; bytes = sizeof(float) * D->N * D->r_u; break;
    case 2: b = &D->JY; bytes = sizeof(float) * D->N * D->d_z * D->r_u; break;
    case 3: b = &D->PhiT; bytes = sizeof(double) * D->r_u * D->d_u; break;
    case 4: b = &D->ubar; bytes = sizeof(double) * D->d_u; break;
    default: return SAA_E_INVALID;
  }
  if ((size_t)n * ((which >= 3) ? sizeof(double) : sizeof(float)) != bytes) return SAA_E_INVALID;
  int rc = check_hip(hipMemcpyAsync(host, b->p, bytes, hipMemcpyDeviceToHost, D->st));
  if (!rc) rc = check_hip(hipStreamSynchronize(D->st));
  return rc;
}

int mrdino_loss_grad(mrdino_model* m, mrdino_data* D, const int* idx, int B, int dino, int prec, double* loss,
                     float* grad) {
  if (!m || !D || !idx || B < 1 || !loss || !compatible(m, D)) return SAA_E_INVALID;
  if (prec != SAA_BF16 && prec != SAA_FP32) return SAA_E_INVALID;
  for (int b = 0; b < B; ++b)
    if (idx[b] < 0 || idx[b] >= D->N) return SAA_E_INVALID;
  int rc = alloc_ws(m, B);
  if (rc) return rc;
  TrainWs& w = train_state(m)->ws;
  if ((rc = check_hip(hipMemcpyAsync(w.idx.p, idx, sizeof(int) * B, hipMemcpyHostToDevice, m->st)))) return rc;
  load_batch(m, D, w, (const int*)w.idx.p, B);
  if ((rc = loss_grad(m, w, B, dino, grad != nullptr, prec == SAA_BF16))) return rc;
  double l[2];
  if ((rc = check_hip(hipMemcpyAsync(l, w.loss.p, sizeof(l), hipMemcpyDeviceToHost, m->st)))) return rc;
  if (grad && (rc = check_hip(hipMemcpyAsync(grad, w.grad.p, sizeof(float) * m->n_params, hipMemcpyDeviceToHost,
                                             m->st))))
    return rc;
  if ((rc = check_hip(hipStreamSynchronize(m->st)))) return rc;
  *loss = (l[0] + l[1]) / B;
  return check_hip(hipGetLastError());
}

int mrdino_eval(mrdino_model* m, saa_ctx* c, const double* z, int want, int prec, double* q_dev, double* dqdz_dev,
                float* phi_dev, float* dphidz_dev) {
  if (!m || !c || !z || want < 1 || want > 15 || c->N < 1) return SAA_E_INVALID;
  if (((want & MRDINO_WANT_Q) && !q_dev) || ((want & MRDINO_WANT_DQDZ) && !dqdz_dev) ||
      ((want & MRDINO_WANT_PHI) && !phi_dev) || ((want & MRDINO_WANT_DPHIDZ) && !dphidz_dev))
    return SAA_E_INVALID;
  const mrdino_dims& d = m->dims;
  if (d.d_z != c->dz || d.r_m > c->n_kl) return SAA_E_MODEL;
  for (int k = 0; k < d.d_z; ++k)
    if (!std::isfinite(z[k])) return SAA_E_INVALID;
  int rc = SAA_OK;
  if (want & (MRDINO_WANT_Q | MRDINO_WANT_DQDZ)) {
    if (prec != SAA_FP32 && prec != SAA_BF16 && prec != SAA_FP8) return SAA_E_INVALID;
    if ((rc = check_hip(hipMemcpyAsync(c->zdev.p, z, sizeof(double) * d.d_z, hipMemcpyHostToDevice, c->st))))
      return rc;
    double* q = (want & MRDINO_WANT_Q) ? q_dev : (double*)c->q.p;
    double* g = (want & MRDINO_WANT_DQDZ) ? dqdz_dev : (double*)c->g.p;
    if ((rc = saa_model_eval(m, c, (const double*)c->zdev.p, prec, q, g))) return rc;
  }
  if ((rc = check_hip(hipStreamSynchronize(c->st)))) return rc;
  if (want & (MRDINO_WANT_PHI | MRDINO_WANT_DPHIDZ)) {
    const int dino = (want & MRDINO_WANT_DPHIDZ) ? 1 : 0;
    const int B = (int)std::min<int64_t>(c->N, 512);
    if ((rc = alloc_ws(m, B))) return rc;
    TrainWs& w = train_state(m)->ws;
    DevBuf Zb;
    std::vector<double> zrep((size_t)B * d.d_z);
    for (int b = 0; b < B; ++b) std::copy(z, z + d.d_z, zrep.begin() + (size_t)b * d.d_z);
    if ((rc = Zb.alloc(sizeof(double) * zrep.size()))) return rc;
    if ((rc = check_hip(hipMemcpyAsync(Zb.p, zrep.data(), sizeof(double) * zrep.size(), hipMemcpyHostToDevice,
                                       m->st))))
      return rc;
    const int nkl = (int)c->n_kl;
    for (int64_t b0 = 0; b0 < c->N && !rc; b0 += B) {
      const int nb = (int)std::min<int64_t>(B, c->N - b0);
      saa_launch::train_inputs((const double*)c->xi.p + b0 * nkl, nkl, (const int*)c->order.p, d.r_m,
                               (const double*)Zb.p, d.d_z, nb, F(w.Xb), m->st);
      if ((rc = forward(m, w, nb, dino, false))) break;
      if (want & MRDINO_WANT_PHI)
        rc = check_hip(hipMemcpyAsync(phi_dev + b0 * d.r_u, w.P.p, sizeof(float) * nb * d.r_u,
                                      hipMemcpyDeviceToDevice, m->st));
      if (!rc && dino)
        rc = check_hip(hipMemcpyAsync(dphidz_dev + b0 * d.d_z * d.r_u, w.JP.p,
                                      sizeof(float) * (size_t)nb * d.d_z * d.r_u, hipMemcpyDeviceToDevice, m->st));
    }
    if (!rc) rc = check_hip(hipStreamSynchronize(m->st));
  }
  if (!rc) rc = check_hip(hipGetLastError());
  return rc;
}

int mrdino_train(mrdino_model* m, mrdino_data* D, const mrdino_train_cfg* cfg, double* epoch_loss, double* seconds) {
  if (!m || !D || !cfg || !compatible(m, D)) return SAA_E_INVALID;
  const int B = cfg->batch;
  if (B < 1 || B > D->N || cfg->epochs < 0 || !(cfg->lr > 0) || !(cfg->lr_late > 0) || !(cfg->beta1 >= 0) ||
      !(cfg->beta1 < 1) || !(cfg->beta2 >= 0) || !(cfg->beta2 < 1) || !(cfg->adam_eps > 0) ||
      (cfg->prec != SAA_BF16 && cfg->prec != SAA_FP32))
    return SAA_E_INVALID;
  const bool bf = cfg->prec == SAA_BF16;
  int rc = alloc_ws(m, B);
  if (rc) return rc;
  TrainState* ts = train_state(m);
  TrainWs& w = ts->ws;
  hipStream_t st = m->st;
  if (!cfg->resume || !ts->started) {   // a new optimisation: fresh moments, schedule and minibatch stream
    if ((rc = check_hip(hipMemsetAsync(w.m.p, 0, sizeof(float) * m->n_params, st))) ||
        (rc = check_hip(hipMemsetAsync(w.v.p, 0, sizeof(float) * m->n_params, st))))
      return rc;
    ts->step = 0;
    ts->epoch = 0;
    ts->rng = cfg->seed;
    ts->started = true;
  }
  // Output scale: the reduced states of this workload vary by a few 1e-3
  // while a fresh network outputs O(1); the output layer is trained as
  // phi = sigma phi' with targets y / sigma, J / sigma (the DINO loss divided
  // by sigma^2), sigma the RMS of the reduced states rounded to a power of
  // two, so the conversions of the stored parameters are exact.
  double sigma = 1.0;
  if ((rc = output_scale(D, st, &sigma))) return rc;
  const float inv_sigma = (float)(1.0 / sigma);
  float* out_layer = (float*)m->master.p + m->off_w[m->dims.depth];
  const int64_t n_out = m->off_b[m->dims.depth] + m->dims.r_u - m->off_w[m->dims.depth];
  saa_launch::scale(out_layer, n_out, inv_sigma, st);
  DevBuf perm_dev;
  if ((rc = perm_dev.alloc(sizeof(int) * D->N))) {
    saa_launch::scale(out_layer, n_out, (float)sigma, st);
    return rc;
  }
  std::vector<int> perm(D->N);
  const int steps = (int)(D->N / B);
  double* loss = (double*)w.loss.p;
  uint64_t& rng = ts->rng;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(e0, st);
  for (int ep = 0; ep < cfg->epochs; ++ep) {
    for (int64_t i = 0; i < D->N; ++i) perm[i] = (int)i;
    for (int64_t i = D->N - 1; i > 0; --i) {   // Fisher-Yates
      const int64_t j = (int64_t)(splitmix64(rng) % (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    if ((rc = check_hip(hipMemcpyAsync(perm_dev.p, perm.data(), sizeof(int) * D->N, hipMemcpyHostToDevice, st))))
      break;
    saa_launch::sum_parts(loss, 0, loss + 2, 0, st);   // zero the epoch sum
    const float lr =
        (float)((cfg->lr_drop_epoch > 0 && ts->epoch >= cfg->lr_drop_epoch) ? cfg->lr_late : cfg->lr);
    for (int s = 0; s < steps; ++s) {
      load_batch(m, D, w, (const int*)perm_dev.p + (int64_t)s * B, B);
      if ((rc = loss_grad(m, w, B, cfg->dino, true, bf, inv_sigma))) break;
      saa_launch::sum_parts(loss, 2, loss + 2, 1, st);
      ++ts->step;
      const float c1 = 1.0f - std::pow((float)cfg->beta1, (float)ts->step);
      const float c2 = 1.0f - std::pow((float)cfg->beta2, (float)ts->step);
      saa_launch::adam((float*)m->master.p, F(w.grad), F(w.m), F(w.v), m->n_params, lr, (float)cfg->beta1,
                       (float)cfg->beta2, (float)cfg->adam_eps, c1, c2, st);
    }
    if (rc) break;
    ++ts->epoch;
    if (epoch_loss) {
      double tot = 0.0;
      if ((rc = check_hip(hipMemcpyAsync(&tot, loss + 2, sizeof(double), hipMemcpyDeviceToHost, st))) ||
          (rc = check_hip(hipStreamSynchronize(st))))
        break;
      epoch_loss[ep] = sigma * sigma * tot / ((double)steps * B);   // in the data's units
    }
  }
  (void)hipEventRecord(e1, st);
  saa_launch::scale(out_layer, n_out, (float)sigma, st);   // back to the data's units
  if (!rc) rc = saa_model::pack(m);
  if (!rc) rc = check_hip(hipStreamSynchronize(st));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (seconds) *seconds = ms * 1e-3;
  if (!rc) rc = mrdino_set_qoi(m, D->c.data(), D->c0);
  return rc;
}

int mrdino_data_errors(mrdino_model* m, mrdino_data* D, double* err_state, double* err_jac) {
  if (!m || !D || !compatible(m, D)) return SAA_E_INVALID;
  const int B = (int)std::min<int64_t>(256, D->N);
  int rc = alloc_ws(m, B);
  if (rc) return rc;
  TrainWs& w = train_state(m)->ws;
  hipStream_t st = m->st;
  DevBuf seq, acc;
  if ((rc = seq.alloc(sizeof(int) * D->N)) || (rc = acc.alloc_zero(sizeof(double) * 4, st))) return rc;
  std::vector<int> id(D->N);
  for (int64_t i = 0; i < D->N; ++i) id[i] = (int)i;
  if ((rc = check_hip(hipMemcpyAsync(seq.p, id.data(), sizeof(int) * D->N, hipMemcpyHostToDevice, st)))) return rc;
  double* a = (double*)acc.p;
  double* loss = (double*)w.loss.p;
  for (int64_t s0 = 0; s0 < D->N; s0 += B) {
    const int b = (int)std::min<int64_t>(B, D->N - s0);
    load_batch(m, D, w, (const int*)seq.p + s0, b);
    if ((rc = loss_grad(m, w, b, 1, false, false))) return rc;
    saa_launch::sum_parts(loss + 0, 1, a + 0, 1, st);
    saa_launch::sum_parts(loss + 1, 1, a + 1, 1, st);
  }
  int nb = 0;
  double ref[2], num[2];
  // reference norms in chunks that fit the partial-sum buffer
  {
    DevBuf parts;
    const int64_t ny = D->N * D->r_u, nj = D->N * D->d_z * D->r_u;
    if ((rc = parts.alloc(sizeof(double) * ((nj + 1023) / 1024 + 1)))) return rc;
    nb = saa_launch::sumsq(F(D->Y), ny, (double*)parts.p, st);
    saa_launch::sum_parts((double*)parts.p, nb, a + 2, 0, st);
    nb = saa_launch::sumsq(F(D->JY), nj, (double*)parts.p, st);
    saa_launch::sum_parts((double*)parts.p, nb, a + 3, 0, st);
    double h[4];
    if ((rc = check_hip(hipMemcpyAsync(h, a, sizeof(h), hipMemcpyDeviceToHost, st))) ||
        (rc = check_hip(hipStreamSynchronize(st))))
      return rc;
    num[0] = h[0];
    num[1] = h[1];
    ref[0] = h[2];
    ref[1] = h[3];
  }
  if (err_state) *err_state = std::sqrt(num[0] / ref[0]);
  if (err_jac) *err_jac = std::sqrt(num[1] / ref[1]);
  return check_hip(hipGetLastError());
}

}  // extern "C"
