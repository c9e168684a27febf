// Smoothed-CVaR SAA reduction (paper Sec. 2.1-2.2, eq. (CVaR_saa_ouu)).
//
//   J_hat(z, t) = t + 1/(N (1-beta)) sum_i s_eps(q_i - t) + alpha/2 |z|^2
//
// with the C^2 quartic smoothing s_eps of the plus function.  t* minimises
// J_hat over t: Phi(t) = sum_i s_eps'(q_i - t) is continuous, non-increasing,
// equals N at min(q) - eps and 0 at max(q), and t* solves Phi = N (1-beta).
// The root is bracketed by [min q - eps, max q] and found by a safeguarded
// Newton iteration (bisection whenever the Newton step leaves the bracket or
// stalls), then polished by one Newton step kept inside the final bracket.
// The gradient
// is the chain rule (eq. (ouu_risk_gradient)) with weights
// w_i = s_eps'(q_i - t*) / (N (1-beta)); since dJ_hat/dt = 0 at t*, no t*
// derivative enters it.
//
// One workgroup does the whole reduction with a fixed summation order, so the
// result is bitwise reproducible.
#include <cfloat>

#include "common.h"
#include "pde.h"

namespace {

constexpr int CBS = 1024;

__device__ __forceinline__ double sp_val(double x, double e) {
  if (x <= 0.0) return 0.0;
  if (x >= e) return x - 0.5 * e;
  const double r = x / e;
  return x * r * r * (1.0 - 0.5 * r);      // x^3/e^2 - x^4/(2 e^3)
}
__device__ __forceinline__ double sp_d1(double x, double e) {
  if (x <= 0.0) return 0.0;
  if (x >= e) return 1.0;
  const double r = x / e;
  return r * r * (3.0 - 2.0 * r);          // 3x^2/e^2 - 2x^3/e^3
}
__device__ __forceinline__ double sp_d2(double x, double e) {
  if (x <= 0.0 || x >= e) return 0.0;
  const double r = x / e;
  return 6.0 * r * (1.0 - r) / e;          // 6x/e^2 - 6x^2/e^3
}

}  // namespace


// phase & 1: determine t (minimiser, or t_in when t_mode = 1) -> tstar[0].
// phase & 2: J, dJ/dt, grad -> out[0] = J, out[1] = dJ/dt, out[2..2+dz) = grad.
// Optional per-sample solver stats (any pointer may be null) -> stats.
__global__ void __launch_bounds__(CBS) saa_k_cvar(const double* q, const double* g, int64_t N, int dz,
                                                  double beta, double eps, double alpha, const double* z,
                                                  int t_mode, double t_in, int phase, double* tstar,
                                                  double* out, const int* newton, const int* lin,
                                                  const int* flag, const int* lin_adj, const int* did,
                                                  CvarStats* stats) {
  __shared__ double red[64 * (CBS / SAA_WAVE)];
  __shared__ double tsh;
  const double target = (double)N * (1.0 - beta);
  if (stats) {
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double nm = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += CBS) {
      if (newton) {
        nm = fmax(nm, (double)newton[i]);
        s[4] += (double)newton[i];
      }
      if (flag) s[0] += (flag[i] != 0) ? 1.0 : 0.0;
      if (did) s[1] += (double)did[i];
      if (lin) s[2] += (double)lin[i];
      if (lin_adj) s[3] += (double)lin_adj[i];
    }
    block_sum<5>(s, red);
    nm = block_max1(nm, red);
    if (threadIdx.x == 0) {
      stats->newton_max = (int)nm;
      stats->n_unconverged = (int)s[0];
      stats->n_adjoints = (int)s[1];
      stats->lin_state = (long long)s[2];
      stats->lin_adjoint = (long long)s[3];
      stats->newton_total = (long long)s[4];
    }
  }
  if (phase & 1) {
    double t;
    if (t_mode == 1) {
      t = t_in;
    } else {
      double mn = INFINITY, mx = -INFINITY;
      for (int64_t i = threadIdx.x; i < N; i += CBS) {
        mn = fmin(mn, q[i]);
        mx = fmax(mx, q[i]);
      }
      double lo = block_min1(mn, red) - eps;
      double hi = block_max1(mx, red);
      // Safeguarded Newton on Phi(t) = target inside the bracket [lo, hi]
      // (Phi(lo) > target >= Phi(hi)): every pass evaluates Phi and Phi',
      // shrinks the bracket by the sign of Phi - target, and takes the Newton
      // step when it lands strictly inside the bracket and at least halves the
      // previous step, else the midpoint.  It ends when the bracket stops
      // shrinking (as the plain bisection) or the Newton step reaches the
      // float64 rounding level of t; the polish below then takes one more
      // Newton step.  A handful of passes instead of ~60 bisections.  A NaN or
      // empty bracket skips the loop; the cap never binds on finite input.
      double tc = 0.5 * (lo + hi);
      t = tc;
      double dx_old = hi - lo;
      for (int guard = 0; guard < 4096 && lo < hi; ++guard) {
        double v[2] = {0.0, 0.0};
        for (int64_t i = threadIdx.x; i < N; i += CBS) {
          v[0] += sp_d1(q[i] - tc, eps);
          v[1] += sp_d2(q[i] - tc, eps);
        }
        block_sum<2>(v, red);
        if (v[0] > target) lo = tc;
        else hi = tc;
        const double mid = 0.5 * (lo + hi);
        t = mid;
        if (mid <= lo || mid >= hi) break;
        double tn = mid;
        if (v[1] > 0.0) {
          const double tnew = tc + (v[0] - target) / v[1];   // Phi' = -sum s''
          if (tnew > lo && tnew < hi && fabs(tnew - tc) <= 0.5 * dx_old) tn = tnew;
        }
        const double dx = fabs(tn - tc);
        dx_old = dx;
        tc = tn;
        t = tn;
        if (dx <= 4.0 * DBL_EPSILON * fabs(tn)) break;
      }
      double v[2] = {0.0, 0.0};
      for (int64_t i = threadIdx.x; i < N; i += CBS) {
        v[0] += sp_d1(q[i] - t, eps);
        v[1] += sp_d2(q[i] - t, eps);
      }
      block_sum<2>(v, red);
      const double slope = -v[1];
      if (slope < 0.0) {
        const double tn = t - (v[0] - target) / slope;
        if (tn >= lo && tn <= hi) t = tn;
      }
    }
    if (threadIdx.x == 0) {
      tstar[0] = t;
      tsh = t;
    }
    __syncthreads();
  } else {
    if (threadIdx.x == 0) tsh = tstar[0];
    __syncthreads();
  }
  if (!(phase & 2)) return;
  const double t = tsh;
  const double scale = 1.0 / target;
  double v[2] = {0.0, 0.0};
  for (int64_t i = threadIdx.x; i < N; i += CBS) {
    v[0] += sp_val(q[i] - t, eps);
    v[1] += sp_d1(q[i] - t, eps);
  }
  block_sum<2>(v, red);
  double zz = 0.0;
  for (int k = 0; k < dz; ++k) zz += z[k] * z[k];
  if (threadIdx.x == 0) {
    out[0] = t + scale * v[0] + 0.5 * alpha * zz;
    out[1] = 1.0 - scale * v[1];
  }
  for (int k0 = 0; k0 < dz; k0 += 8) {
    double a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += CBS) {
      const double w = sp_d1(q[i] - t, eps);
      if (w != 0.0) {
        const double* gi = g + i * dz;
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (k0 + c < dz) a[c] += w * gi[k0 + c];
      }
    }
    block_sum<8>(a, red);
    if (threadIdx.x == 0) {
      for (int c = 0; c < 8 && k0 + c < dz; ++c) out[2 + k0 + c] = scale * a[c] + alpha * z[k0 + c];
    }
  }
}

namespace saa_launch {
void cvar(const double* q, const double* g, int64_t N, int dz, double beta, double eps, double alpha,
          const double* z, int t_mode, double t_in, int phase, double* tstar, double* out, const int* newton,
          const int* lin, const int* flag, const int* lin_adj, const int* did, void* stats, hipStream_t st) {
  saa_k_cvar<<<1, CBS, 0, st>>>(q, g, N, dz, beta, eps, alpha, z, t_mode, t_in, phase, tstar, out, newton, lin,
                                flag, lin_adj, did, (CvarStats*)stats);
}
}  // namespace saa_launch
