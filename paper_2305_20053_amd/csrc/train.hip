// Kernels of MR-DINO construction (paper Sec. 3.3-3.4): mass-weighted POD
// products, reduced data projections, and the derivative-informed training
// step (forward, forward-mode Jacobian, hand-derived reverse pass, Adam).
//
// Layouts (row-major): activations H, A are B x W; tangents are (B d_Z) x W
// with row b d_Z + k holding the derivative with respect to z_k of sample b;
// reduced targets Y are B x r_u and JY (B d_Z) x r_u.
#include <rocblas/rocblas.h>
#include <algorithm>

#include "common.h"
#include "runtime.h"

namespace {

__device__ __forceinline__ float gelu_f(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float npdf_f(float a) { return 0.39894228040143268f * __expf(-0.5f * a * a); }
__device__ __forceinline__ float dgelu_f(float a) { return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * npdf_f(a); }
__device__ __forceinline__ float d2gelu_f(float a) { return npdf_f(a) * (2.0f - a * a); }

}  // namespace

// out[s][p] = (M_II (u_s - ubar))_p on the (n-1)^2 interior grid (dense
// interior order), consistent P1 mass: h^2/12 (6 u_p + E + W + N + S + NE + SW).
// ubar may be null (treated as zero).
template <typename T>
__global__ void saa_k_mass_rows(const T* U, int64_t ldu, const T* ubar, T* out, int64_t ldo, int n, int64_t rows) {
  const int m = n - 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * m * m) return;
  const int64_t s = t / ((int64_t)m * m);
  const int p = (int)(t - s * m * m);
  const int j = p / m, i = p - j * m;
  const T* u = U + s * ldu;
  auto val = [&](int ii, int jj) -> T {
    if (ii < 0 || jj < 0 || ii >= m || jj >= m) return (T)0;
    const int q = jj * m + ii;
    return ubar ? u[q] - ubar[q] : u[q];
  };
  const T h2 = (T)1 / (T)((n) * (n));
  out[s * ldo + p] = h2 / (T)12 *
                     ((T)6 * val(i, j) + val(i + 1, j) + val(i - 1, j) + val(i, j + 1) + val(i, j - 1) +
                      val(i + 1, j + 1) + val(i - 1, j - 1));
}

// Column means of a rows x cols matrix (fixed summation order per column).
template <typename T>
__global__ void saa_k_colmean(const T* X, int64_t rows, int cols, int64_t ldx, T* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  T s = (T)0;
  for (int64_t r = 0; r < rows; ++r) s += X[r * ldx + c];
  out[c] = s / (T)rows;
}

// Training inputs: X[s] = [xi_hat (leading r_m KL coordinates); z_s] in FP32.
__global__ void saa_k_train_inputs(const double* xi, int nkl, const int* order, int r_m, const double* Z, int d_z,
                                   int64_t N, float* X) {
  const int w = r_m + d_z;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * w) return;
  const int64_t s = t / w;
  const int c = (int)(t - s * w);
  X[t] = (float)(c < r_m ? xi[s * nkl + order[c]] : Z[s * d_z + (c - r_m)]);
}

// Gather a minibatch: dst[b] = src[idx[b]] (rows of `width` floats).
__global__ void saa_k_gather_rows(const float* src, int64_t width, const int* idx, int B, float* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * width) return;
  const int64_t b = t / width, c = t - b * width;
  dst[t] = src[(int64_t)idx[b] * width + c];
}

// Layer epilogue: A += bias (per column); H = GELU(A).
__global__ void saa_k_bias_gelu(float* A, const float* bias, float* H, int64_t rows, int cols, int act) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const float a = A[t] + bias[t % cols];
  A[t] = a;
  if (H) H[t] = act ? gelu_f(a) : a;
}

// First-layer tangents: JA[b d_Z + k][f] = W_0[f][r_m + k]; JH = GELU'(A) JA.
__global__ void saa_k_tangent0(const float* W0, int ldw, int r_m, int d_z, const float* A, int B, int W, float* JA,
                               float* JH) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * d_z * W) return;
  const int f = (int)(t % W);
  const int64_t row = t / W;
  const int k = (int)(row % d_z);
  const int64_t b = row / d_z;
  const float ja = W0[(int64_t)f * ldw + r_m + k];
  JA[t] = ja;
  JH[t] = dgelu_f(A[b * W + f]) * ja;
}

// JH = GELU'(A) JA (row b d_Z + k of JA uses row b of A).
__global__ void saa_k_tangent_scale(const float* JA, const float* A, int B, int d_z, int W, float* JH) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * d_z * W) return;
  const int f = (int)(t % W);
  const int64_t b = t / ((int64_t)d_z * W);
  JH[t] = dgelu_f(A[b * W + f]) * JA[t];
}

// Residuals and loss: E = Phi - y_scale Y (scaled by 2/B into G), partial
// sums of |E|^2 per block into part[blockIdx.x].  y_scale is 1, or the
// inverse power-of-two output scale of training (exact).
__global__ void saa_k_residual(const float* P, const float* Y, int64_t n, float scale, float y_scale, float* G,
                               double* part) {
  __shared__ double red[16];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (t < n) {
    const float e = P[t] - y_scale * Y[t];
    G[t] = scale * e;
    e2 = (double)e * (double)e;
  }
  e2 = block_sum1(e2, red);
  if (threadIdx.x == 0) part[blockIdx.x] = e2;
}

// Reverse through a hidden layer: given gH (B x W), gJH ((B d_Z) x W), A,
// JA: gJA = GELU'(A) gJH (in place into gJH) and
// gA = GELU'(A) gH + GELU''(A) sum_k gJH[b,k] JA[b,k]  (in place into gH).
__global__ void saa_k_layer_back(float* gH, float* gJH, const float* A, const float* JA, int B, int d_z, int W,
                                 int dino) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)B * W) return;
  const int64_t b = t / W;
  const int f = (int)(t % W);
  const float a = A[t];
  const float s1 = dgelu_f(a);
  float ga = s1 * gH[t];
  if (dino) {
    float acc = 0.0f;
    for (int k = 0; k < d_z; ++k) {
      const int64_t r = (b * d_z + k) * W + f;
      acc += gJH[r] * JA[r];
      gJH[r] = s1 * gJH[r];
    }
    ga += d2gelu_f(a) * acc;
  }
  gH[t] = ga;
}

// Column sums (bias gradients): out[c] = sum_r X[r][c].
// Column sums over `rows` rows: 256 threads = 8 row groups x 32 columns; the
// groups are summed in order (deterministic).
__device__ __forceinline__ float colsum_block(const float* X, int64_t rows, int64_t ld, int cols, int c) {
  __shared__ float part[8][32];
  const int cl = threadIdx.x & 31, rg = threadIdx.x >> 5;
  float s = 0.0f;
  if (c < cols)
    for (int64_t r = rg; r < rows; r += 8) s += X[r * ld + c];
  part[rg][cl] = s;
  __syncthreads();
  float t = 0.0f;
  for (int k = 0; k < 8; ++k) t += part[k][cl];
  return t;
}

// out[c] (+)= sum_r X[r][c], X rows x cols row-major.
__global__ void __launch_bounds__(256) saa_k_colsum(const float* X, int64_t rows, int cols, float* out,
                                                    int accumulate) {
  const int c = blockIdx.x * 32 + (threadIdx.x & 31);
  const float t = colsum_block(X, rows, cols, cols, c);
  if (threadIdx.x < 32 && c < cols) out[c] = accumulate ? out[c] + t : t;
}

// dW_0[f][r_m + k] += sum_b gJA_0[b d_Z + k][f]  (the constant first-layer tangent).
__global__ void __launch_bounds__(256) saa_k_w0z_grad(const float* gJA, int B, int d_z, int W, int r_m, int ldw,
                                                      float* dW0) {
  const int c = blockIdx.x * 32 + (threadIdx.x & 31);   // c = k W + f
  const float t = colsum_block(gJA, B, (int64_t)d_z * W, d_z * W, c);
  if (threadIdx.x < 32 && c < d_z * W) dW0[(int64_t)(c % W) * ldw + r_m + c / W] += t;
}

// Adam (bias-corrected), FP32 master parameters.
__global__ void saa_k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.0f - b1) * gt;
  const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// Sum of partial block sums (fixed order) into out[0].
__global__ void saa_k_sum_parts(const double* part, int n, double* out, int accumulate) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  s = block_sum1(s, red);
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + s : s;
}

// out = U - ubar (row-wise; out may alias U).
__global__ void saa_k_center_rows(const double* U, const double* ubar, double* out, int64_t cols, int64_t rows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  out[t] = U[t] - ubar[t % cols];
}

// Partial sums of squares per 1024-thread block.
__global__ void saa_k_sumsq(const float* x, int64_t n, double* part) {
  __shared__ double red[16];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double v = t < n ? (double)x[t] : 0.0;
  const double s = block_sum1(v * v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x[i] *= f for i < n (f a power of two: exact).
__global__ void saa_k_scale(float* x, int64_t n, float f) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] *= f;
}

// Convert float64 -> float32.
__global__ void saa_k_d2f(const double* x, float* y, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = (float)x[t];
}

namespace saa_launch {

static inline unsigned nb(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Row-major FP64 C = op(A) op(B) of the POD (Gram matrix, basis,
// projections) by rocBLAS, a plain library GEMM, on the caller's handle: in
// column-major terms C^T = op(B)^T op(A)^T, so B comes first and each operand
// keeps its transpose flag.  Any rocBLAS status other than success is a
// device error.
int dgemm(rocblas_handle h, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
          const double* B, int ldb, double beta, double* C, int ldc, hipStream_t st) {
  if (!h) return SAA_E_DEVICE;
  if (rocblas_set_stream(h, st) != rocblas_status_success) return SAA_E_DEVICE;
  const rocblas_operation oB = tb ? rocblas_operation_transpose : rocblas_operation_none;
  const rocblas_operation oA = ta ? rocblas_operation_transpose : rocblas_operation_none;
  const rocblas_status s = rocblas_dgemm(h, oB, oA, N, M, K, &alpha, B, ldb, A, lda, &beta, C, ldc);
  return s == rocblas_status_success ? SAA_OK : SAA_E_DEVICE;
}

// A rocBLAS handle with atomics disallowed (reproducible results), or null.
rocblas_handle blas_create() {
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
  if (rocblas_set_atomics_mode(h, rocblas_atomics_not_allowed) != rocblas_status_success) {
    (void)rocblas_destroy_handle(h);
    return nullptr;
  }
  return h;
}
void blas_destroy(rocblas_handle h) {
  if (h) (void)rocblas_destroy_handle(h);
}

void mass_rows(const double* U, int64_t ldu, const double* ubar, double* out, int64_t ldo, int n, int64_t rows,
               hipStream_t st) {
  saa_k_mass_rows<double><<<nb(rows * (int64_t)(n - 1) * (n - 1)), 256, 0, st>>>(U, ldu, ubar, out, ldo, n, rows);
}
void colmean(const double* X, int64_t rows, int cols, int64_t ldx, double* out, hipStream_t st) {
  saa_k_colmean<double><<<nb(cols), 256, 0, st>>>(X, rows, cols, ldx, out);
}
void train_inputs(const double* xi, int nkl, const int* order, int r_m, const double* Z, int d_z, int64_t N, float* X,
                  hipStream_t st) {
  saa_k_train_inputs<<<nb(N * (r_m + d_z)), 256, 0, st>>>(xi, nkl, order, r_m, Z, d_z, N, X);
}
void gather_rows(const float* src, int64_t width, const int* idx, int B, float* dst, hipStream_t st) {
  saa_k_gather_rows<<<nb((int64_t)B * width), 256, 0, st>>>(src, width, idx, B, dst);
}
void bias_gelu(float* A, const float* bias, float* H, int64_t rows, int cols, int act, hipStream_t st) {
  saa_k_bias_gelu<<<nb(rows * cols), 256, 0, st>>>(A, bias, H, rows, cols, act);
}
void tangent0(const float* W0, int ldw, int r_m, int d_z, const float* A, int B, int W, float* JA, float* JH,
              hipStream_t st) {
  saa_k_tangent0<<<nb((int64_t)B * d_z * W), 256, 0, st>>>(W0, ldw, r_m, d_z, A, B, W, JA, JH);
}
void tangent_scale(const float* JA, const float* A, int B, int d_z, int W, float* JH, hipStream_t st) {
  saa_k_tangent_scale<<<nb((int64_t)B * d_z * W), 256, 0, st>>>(JA, A, B, d_z, W, JH);
}
int residual(const float* P, const float* Y, int64_t n, float scale, float y_scale, float* G, double* part,
             hipStream_t st) {
  const unsigned blocks = nb(n, 1024);
  saa_k_residual<<<blocks, 1024, 0, st>>>(P, Y, n, scale, y_scale, G, part);
  return (int)blocks;
}
void layer_back(float* gH, float* gJH, const float* A, const float* JA, int B, int d_z, int W, int dino,
                hipStream_t st) {
  saa_k_layer_back<<<nb((int64_t)B * W), 256, 0, st>>>(gH, gJH, A, JA, B, d_z, W, dino);
}
void colsum(const float* X, int64_t rows, int cols, float* out, int accumulate, hipStream_t st) {
  saa_k_colsum<<<(unsigned)((cols + 31) / 32), 256, 0, st>>>(X, rows, cols, out, accumulate);
}
void w0z_grad(const float* gJA, int B, int d_z, int W, int r_m, int ldw, float* dW0, hipStream_t st) {
  saa_k_w0z_grad<<<(unsigned)((d_z * W + 31) / 32), 256, 0, st>>>(gJA, B, d_z, W, r_m, ldw, dW0);
}
void adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps, float c1,
          float c2, hipStream_t st) {
  saa_k_adam<<<nb(n), 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}
void sum_parts(const double* part, int n, double* out, int accumulate, hipStream_t st) {
  saa_k_sum_parts<<<1, 1024, 0, st>>>(part, n, out, accumulate);
}
void d2f(const double* x, float* y, int64_t n, hipStream_t st) { saa_k_d2f<<<nb(n), 256, 0, st>>>(x, y, n); }
void scale(float* x, int64_t n, float f, hipStream_t st) {
  if (n > 0) saa_k_scale<<<nb(n), 256, 0, st>>>(x, n, f);
}
void center_rows(const double* U, const double* ubar, double* out, int64_t cols, int64_t rows, hipStream_t st) {
  saa_k_center_rows<<<nb(rows * cols), 256, 0, st>>>(U, ubar, out, cols, rows);
}
int sumsq(const float* x, int64_t n, double* part, hipStream_t st) {
  const unsigned blocks = nb(n, 1024);
  saa_k_sumsq<<<blocks, 1024, 0, st>>>(x, n, part);
  return (int)blocks;
}

}  // namespace saa_launch
