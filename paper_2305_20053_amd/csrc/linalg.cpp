// Host symmetric eigensolver for the small POD Gram matrix (n_pod x n_pod):
// Householder reduction to tridiagonal form, then the implicit QL iteration
// with Wilkinson shifts, accumulating the orthogonal transformations.
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/saa.h"

namespace {

// Reduce the symmetric n x n matrix A (row-major, overwritten) to tridiagonal
// form T = Q^T A Q.  On return d holds diag(T), e[i] the (i, i-1) entry
// (e[0] = 0) and A holds Q (row-major).
void tridiagonalize(int n, double* A, double* d, double* e) {
  auto a = [&](int i, int j) -> double& { return A[(int64_t)i * n + j]; };
  std::vector<double> v(n), p(n);
  // Householder vectors are stored in the rows of A below the tridiagonal.
  for (int k = n - 1; k >= 2; --k) {
    // annihilate a(k, 0..k-2) using the reflector built from row k, columns 0..k-1
    double scale = 0.0;
    for (int j = 0; j < k; ++j) scale += std::fabs(a(k, j));
    if (scale == 0.0) {
      e[k] = a(k, k - 1);
      d[k] = 0.0;   // marks "no reflector"
      continue;
    }
    double sigma = 0.0;
    for (int j = 0; j < k; ++j) {
      v[j] = a(k, j) / scale;
      sigma += v[j] * v[j];
    }
    const double alpha = (v[k - 1] >= 0.0) ? -std::sqrt(sigma) : std::sqrt(sigma);
    e[k] = scale * alpha;
    const double h = sigma - v[k - 1] * alpha;   // = |u|^2 / 2 for u = v - alpha e_{k-1}
    v[k - 1] -= alpha;
    // p = A u / h on the leading k x k block, then w = p - (u.p / 2h) u
    for (int i = 0; i < k; ++i) {
      double s = 0.0;
      for (int j = 0; j < k; ++j) s += a(i, j) * v[j];
      p[i] = s / h;
    }
    double up = 0.0;
    for (int i = 0; i < k; ++i) up += v[i] * p[i];
    const double kk = up / (2.0 * h);
    for (int i = 0; i < k; ++i) p[i] -= kk * v[i];
    // A <- A - u w^T - w u^T on the leading block
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) a(i, j) -= v[i] * p[j] + p[i] * v[j];
    for (int j = 0; j < k; ++j) a(k, j) = v[j];   // keep u for the accumulation
    d[k] = h;
  }
  if (n > 1) {   // (for n = 1 there is no entry (1, 0): d and e hold one element)
    e[1] = a(1, 0);
    d[1] = 0.0;
  }
  d[0] = 0.0;
  e[0] = 0.0;
  // accumulate Q = H_{n-1} ... H_2 applied to the identity, innermost first
  std::vector<double> Q((int64_t)n * n, 0.0);
  auto q = [&](int i, int j) -> double& { return Q[(int64_t)i * n + j]; };
  for (int i = 0; i < n; ++i) q(i, i) = 1.0;
  std::vector<double> sv(n);
  for (int k = 2; k < n; ++k) {
    const double h = d[k];
    if (h == 0.0) continue;
    // Q <- (I - u u^T / h) Q on rows 0..k-1 (u = stored row k, length k):
    // s = u^T Q / h, then Q -= u s^T, both as row sweeps
    for (int j = 0; j < n; ++j) sv[j] = 0.0;
    for (int i = 0; i < k; ++i) {
      const double ui = a(k, i);
      const double* qi = &q(i, 0);
      for (int j = 0; j < n; ++j) sv[j] += ui * qi[j];
    }
    for (int j = 0; j < n; ++j) sv[j] /= h;
    for (int i = 0; i < k; ++i) {
      const double ui = a(k, i);
      double* qi = &q(i, 0);
      for (int j = 0; j < n; ++j) qi[j] -= ui * sv[j];
    }
  }
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int64_t t = 0; t < (int64_t)n * n; ++t) A[t] = Q[t];
}

// Eigenvalues of the symmetric tridiagonal (d, e) by implicit QL with
// Wilkinson shifts; the rotations are applied to the rows of Zt (= Z^T, so
// that row i of Zt ends as eigenvector i).
int tridiagonal_ql(int n, double* d, double* e, double* Zt) {
  for (int i = 1; i < n; ++i) e[i - 1] = e[i];
  if (n > 0) e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) return SAA_E_NOCONV;
      // Wilkinson shift from the leading 2 x 2 block at l
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      for (; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double* zi = Zt + (int64_t)i * n;   // rotate rows i, i+1 of Zt
        double* zj = zi + n;
        for (int k = 0; k < n; ++k) {
          f = zj[k];
          zj[k] = s * zi[k] + c * f;
          zi[k] = c * zi[k] - s * f;
        }
      }
      if (r == 0.0 && i >= l) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return SAA_OK;
}

}  // namespace

extern "C" int saa_sym_eig(int n, const double* A, double* w, double* V) {
  if (n < 1 || !A || !w || !V) return SAA_E_INVALID;
  for (int64_t t = 0; t < (int64_t)n * n; ++t)
    if (!std::isfinite(A[t])) return SAA_E_INVALID;
  std::vector<double> M(A, A + (int64_t)n * n), d(n), e(n);
  // symmetrise
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const double s = 0.5 * (M[(int64_t)i * n + j] + M[(int64_t)j * n + i]);
      M[(int64_t)i * n + j] = M[(int64_t)j * n + i] = s;
    }
  tridiagonalize(n, M.data(), d.data(), e.data());
  // transpose Q so that the QL rotations work on contiguous rows
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) std::swap(M[(int64_t)i * n + j], M[(int64_t)j * n + i]);
  int rc = tridiagonal_ql(n, d.data(), e.data(), M.data());
  if (rc) return rc;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) std::swap(M[(int64_t)i * n + j], M[(int64_t)j * n + i]);
  // sort descending, columns of V are the eigenvectors
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (d[idx[j]] > d[idx[i]]) std::swap(idx[i], idx[j]);
  for (int c = 0; c < n; ++c) {
    w[c] = d[idx[c]];
    for (int r = 0; r < n; ++r) V[(int64_t)r * n + c] = M[(int64_t)r * n + idx[c]];
  }
  return SAA_OK;
}
