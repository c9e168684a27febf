// Symmetric eigensolver on the GPU for the POD Gram matrix (Sec. 3.3):
// cyclic two-sided Jacobi with the round-robin ("circle") ordering, so that
// each round rotates np/2 disjoint index pairs at once (Golub and Van Loan,
// Matrix Computations, Sec. 8.5: the symmetric Schur 2x2 rotation and the
// parallel ordering).  One kernel per round: every thread recomputes the
// rotations of its two pairs from the previous matrix (double buffered, so
// no thread reads a value another one is writing) and writes one 2x2 block
// of J^T A J and its transpose, or rotates one row pair of the accumulated
// eigenvectors.  A sweep is np - 1 rounds; sweeps stop when every
// off-diagonal entry is below 1e-15 of the geometric mean of its two
// diagonal entries (entries of rows with a negligible diagonal: below
// 1e-16 of the largest diagonal entry).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "../../include/saa.h"
#include "common.h"
#include "ctx.h"

namespace {

// Pair k (0 <= k < np/2) of round r (0 <= r < np - 1) for an even np: index
// 0 stays, 1..np-1 turn around a circle (every pair meets once per sweep).
__device__ __forceinline__ void round_pair(int np, int r, int k, int& p, int& q) {
  const int m = np - 1;
  if (k == 0) {
    p = 0;
    q = 1 + r % m;
  } else {
    p = 1 + (r + k) % m;
    q = 1 + (r - k + m) % m;
  }
}

// Rotation (c, s) that diagonalises [[a_pp, a_pq], [a_pq, a_qq]] by
// J^T B J with J = [[c, s], [-s, c]]: tau = (a_qq - a_pp) / (2 a_pq),
// t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1 / sqrt(1 + t^2), s = t c.
__device__ __forceinline__ void schur2(const double* A, int np, int p, int q, double& c, double& s) {
  const double apq = A[(size_t)p * np + q];
  if (apq == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double tau = (A[(size_t)q * np + q] - A[(size_t)p * np + p]) / (2.0 * apq);
  double t;
  if (fabs(tau) > 1e150) t = 0.5 / tau;   // 1 + tau^2 would overflow
  else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// One round: An = J^T A J (blocks with P <= Q, each written with its
// transpose), V = V J.  Threads [0, half^2) take A blocks, [half^2,
// half^2 + np half) take (row, pair) of V.
__global__ void __launch_bounds__(256) saa_k_jacobi_round(const double* A, double* An, double* V, int np, int r) {
  const int half = np / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nA = (int64_t)half * half;
  if (t < nA) {
    const int P = (int)(t / half), Q = (int)(t % half);
    if (P > Q) return;
    int p0, q0, p1, q1;
    round_pair(np, r, P, p0, q0);
    round_pair(np, r, Q, p1, q1);
    double c0, s0, c1, s1;
    schur2(A, np, p0, q0, c0, s0);
    schur2(A, np, p1, q1, c1, s1);
    const double b00 = A[(size_t)p0 * np + p1], b01 = A[(size_t)p0 * np + q1];
    const double b10 = A[(size_t)q0 * np + p1], b11 = A[(size_t)q0 * np + q1];
    const double x00 = c0 * b00 - s0 * b10, x01 = c0 * b01 - s0 * b11;
    const double x10 = s0 * b00 + c0 * b10, x11 = s0 * b01 + c0 * b11;
    const double y00 = x00 * c1 - x01 * s1, y01 = x00 * s1 + x01 * c1;
    const double y10 = x10 * c1 - x11 * s1, y11 = x10 * s1 + x11 * c1;
    if (P == Q) {   // the 2x2 diagonal block: the pair is annihilated
      An[(size_t)p0 * np + p0] = y00;
      An[(size_t)q0 * np + q0] = y11;
      An[(size_t)p0 * np + q0] = 0.0;
      An[(size_t)q0 * np + p0] = 0.0;
      return;
    }
    An[(size_t)p0 * np + p1] = y00;
    An[(size_t)p1 * np + p0] = y00;
    An[(size_t)p0 * np + q1] = y01;
    An[(size_t)q1 * np + p0] = y01;
    An[(size_t)q0 * np + p1] = y10;
    An[(size_t)p1 * np + q0] = y10;
    An[(size_t)q0 * np + q1] = y11;
    An[(size_t)q1 * np + q0] = y11;
    return;
  }
  const int64_t tv = t - nA;
  if (tv >= (int64_t)np * half) return;
  const int i = (int)(tv / half), P = (int)(tv % half);
  int p, q;
  round_pair(np, r, P, p, q);
  double c, s;
  schur2(A, np, p, q, c, s);
  if (s == 0.0) return;
  double* v = V + (size_t)i * np;
  const double vp = v[p], vq = v[q];
  v[p] = vp * c - vq * s;
  v[q] = vp * s + vq * c;
}

// Largest off-diagonal measure of row i (entries j > i), see the header.
__global__ void __launch_bounds__(256) saa_k_jacobi_off(const double* A, int np, double amax, double* part) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  const double aii = fabs(A[(size_t)i * np + i]);
  double m = 0.0;
  for (int j = i + 1 + threadIdx.x; j < np; j += 256) {
    const double aij = fabs(A[(size_t)i * np + j]);
    const double d = sqrt(aii * fabs(A[(size_t)j * np + j]));
    m = fmax(m, d > 1e-14 * amax ? aij / d : 10.0 * aij / amax);
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[i] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Padded copy A (n x n) -> Ap (np x np, zero border) and V = I (np x np).
__global__ void saa_k_jacobi_init(const double* A, int n, double* Ap, double* V, int np) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)np * np) return;
  const int i = (int)(t / np), j = (int)(t % np);
  // symmetrised input
  Ap[t] = (i < n && j < n) ? 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]) : 0.0;
  V[t] = (i == j) ? 1.0 : 0.0;
}

__global__ void saa_k_jacobi_diag(const double* A, int np, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) d[i] = A[(size_t)i * np + i];
}

// Vout[i][k] = V[i][perm[k]] for i, k < n (eigenvectors as columns, sorted).
__global__ void saa_k_jacobi_gather(const double* V, int np, const int* perm, int n, double* Vout) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), k = (int)(t % n);
  Vout[t] = V[(size_t)i * np + perm[k]];
}

}  // namespace

extern "C" int saa_sym_eig_gpu(int n, const double* A_dev, double* w, double* V_dev, void* hip_stream,
                               int* sweeps_out) {
  if (n < 1 || n > 16384 || !A_dev || !w || !V_dev) return SAA_E_INVALID;
  hipStream_t st = (hipStream_t)hip_stream;
  const int np = (n + 1) & ~1;   // even, >= 2
  saa_rt::DevBuf A0, A1, V, dg, part, perm;
  int rc;
  const size_t mb = sizeof(double) * (size_t)np * np;
  if ((rc = A0.alloc(mb)) || (rc = A1.alloc(mb)) || (rc = V.alloc(mb)) || (rc = dg.alloc(sizeof(double) * np)) ||
      (rc = part.alloc(sizeof(double) * np)) || (rc = perm.alloc(sizeof(int) * n)))
    return rc;
  const int64_t tot = (int64_t)np * np;
  saa_k_jacobi_init<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(A_dev, n, (double*)A0.p, (double*)V.p, np);
  double* Ac = (double*)A0.p;
  double* An = (double*)A1.p;
  std::vector<double> d(np), pm(np);
  const int half = np / 2;
  const int64_t tasks = (int64_t)half * half + (int64_t)np * half;
  const unsigned grid = (unsigned)((tasks + 255) / 256);
  int sweep = 0;
  for (;; ++sweep) {
    saa_k_jacobi_diag<<<(np + 255) / 256, 256, 0, st>>>(Ac, np, (double*)dg.p);
    if ((rc = saa_rt::check_hip(hipMemcpyAsync(d.data(), dg.p, sizeof(double) * np, hipMemcpyDeviceToHost, st))) ||
        (rc = saa_rt::check_hip(hipStreamSynchronize(st))))
      return rc;
    double amax = 0.0;
    for (double x : d) amax = std::max(amax, std::fabs(x));
    if (!(amax > 0.0)) amax = 1.0;
    saa_k_jacobi_off<<<np, 256, 0, st>>>(Ac, np, amax, (double*)part.p);
    if ((rc = saa_rt::check_hip(hipMemcpyAsync(pm.data(), part.p, sizeof(double) * np, hipMemcpyDeviceToHost, st))) ||
        (rc = saa_rt::check_hip(hipStreamSynchronize(st))))
      return rc;
    double off = 0.0;
    for (double x : pm) off = std::max(off, x);
    if (!(off == off)) return SAA_E_NOCONV;
    if (off <= 1e-15 || sweep == 60) break;
    for (int r = 0; r < np - 1; ++r) {
      // the diagonal blocks are written by their (P, P) threads; the other
      // entries by the (P, Q) / (Q, P) writes, so An is complete after a round
      saa_k_jacobi_round<<<grid, 256, 0, st>>>(Ac, An, (double*)V.p, np, r);
      std::swap(Ac, An);
    }
  }
  // eigenvalues in decreasing order, eigenvectors as columns
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] > d[b]; });
  for (int k = 0; k < n; ++k) w[k] = d[order[k]];
  if ((rc = saa_rt::check_hip(hipMemcpyAsync(perm.p, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, st))))
    return rc;
  const int64_t nn = (int64_t)n * n;
  saa_k_jacobi_gather<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>((double*)V.p, np, (const int*)perm.p, n, V_dev);
  if ((rc = saa_rt::check_hip(hipGetLastError())) || (rc = saa_rt::check_hip(hipStreamSynchronize(st)))) return rc;
  if (sweeps_out) *sweeps_out = sweep;
  return sweep == 60 ? SAA_E_NOCONV : SAA_OK;
}
