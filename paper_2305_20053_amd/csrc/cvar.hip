// Smoothed-CVaR SAA reduction (paper Sec. 2.1-2.2, eq. (CVaR_saa_ouu)).
//
//   J_hat(z, t) = t + 1/(N (1-beta)) sum_i s_eps(q_i - t) + alpha/2 |z|^2
//
// with the C^2 quartic smoothing s_eps of the plus function.  t* minimises
// J_hat over t: Phi(t) = sum_i s_eps'(q_i - t) is continuous, non-increasing,
// equals N at min(q) - eps and 0 at max(q), and t* solves Phi = N (1-beta).
//
// The search keeps a bracket [lo, hi] with Phi(lo) > target >= Phi(hi) and
// runs as a short fixed sequence of launches:
//  1. minmax (G workgroups): partial min / max of q -> initial bracket
//     [min q - eps, max q];
//  2. up to PASSES bracketing passes (G workgroups), certified by counting:
//     s_eps' is 1 beyond eps and 0 below 0, so
//         #{q > t + eps} <= Phi(t) <= #{q > t};
//     a probe t with #{q > t + eps} > target is a valid lo, one with
//     #{q > t} <= target a valid hi.  Each pass histograms every q against
//     NP equispaced probes (exact binary search over the probe values) and
//     the bracket shrinks about NP/2-fold, until it is a few eps wide;
//  3. compact (G workgroups): samples in (lo, hi + eps) are the only ones
//     whose s_eps' varies inside the bracket; they are gathered into a small
//     "active" set and the samples at or above hi + eps are counted (their
//     s_eps' is 1 throughout the bracket);
//  4. solve (1 workgroup): the active set is sorted in LDS (a fixed summation
//     order) and a safeguarded Newton iteration on
//         Phi(t) = #{q >= hi + eps} + sum_active s_eps'(q_a - t)
//     runs inside the bracket (bisection when a step leaves it or stalls),
//     followed by one polish step.  If the active set overflows its capacity
//     the same iteration runs over all N samples.
// Every workgroup recomputes the bracket from the previous launches' results
// with the same arithmetic, so all of them agree on it without a grid barrier.
// For beta = 0 (target = N) every t <= min(q) - eps is a minimiser with the
// same J and weights; t* = min(q) - eps is returned.
//
// The value and gradient (eq. (ouu_risk_gradient), chain rule with weights
// w_i = s_eps'(q_i - t*) / (N (1-beta)); dJ_hat/dt = 0 at t*, so no t*
// derivative enters) are per-workgroup partial sums over contiguous chunks,
// reduced in chunk order by one workgroup.  All sums have a fixed order, so
// results are bitwise reproducible.
#include <cfloat>

#include "common.h"
#include "pde.h"

namespace {

constexpr int RBS = 256;          // threads of the multi-workgroup passes
constexpr int SBS = 1024;         // threads of the single-workgroup kernels
constexpr int NP = 64;            // probes per bracketing pass
constexpr int NB = NP + 1;        // histogram bins: number of probes below q
constexpr int PASSES = 4;         // bracketing passes (shrink ~32x each)
constexpr int CAP = 8192;         // active-set capacity (doubles in LDS)
constexpr int GMAX = 256;         // workgroups of the multi-workgroup passes
constexpr int PSTRIDE = 2 + SAA_MAX_DZ;

// Device workspace, carved from one allocation of cvar_work_bytes().
struct CvarWork {
  double* mm;                  // [GMAX][2] partial min / max of q
  unsigned long long* hist;    // [PASSES][2][NB] probe histograms
  unsigned long long* act;     // [0] active-set size, [1] #{q >= hi + eps}
  double* aval;                // [CAP] active q values
  double* part;                // [GMAX][PSTRIDE] partial sums of the value / gradient
};

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

// Probe j of a pass over [lo, hi]; non-decreasing in j for any rounding.
__device__ __forceinline__ double probe(double lo, double step, int j) { return lo + (double)(j + 1) * step; }

// #{j < NP : probe(j) + shift < x}, exact (binary search over monotone probes).
__device__ __forceinline__ int probes_below(double x, double lo, double step, double shift) {
  int a = 0, b = NP;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (probe(lo, step, m) + shift < x) a = m + 1;
    else b = m;
  }
  return a;
}

struct Bracket {
  double lo, hi;
  bool live;   // the bracketing passes are still refining it
};

// Bracket after `passes` bracketing passes, recomputed from the workspace.
// Called by every thread of a block; all threads get the same result.
// `sh` holds 2 NB counts of LDS, `red` the block_sum scratch.
__device__ Bracket bracket_after(const CvarWork& w, int G, int passes, double eps, double target, double N,
                                 double* red, unsigned long long* sh) {
  double mn = INFINITY, mx = -INFINITY;
  for (int b = threadIdx.x; b < G; b += blockDim.x) {
    mn = fmin(mn, w.mm[2 * b]);
    mx = fmax(mx, w.mm[2 * b + 1]);
  }
  Bracket br;
  br.lo = block_min1(mn, red) - eps;
  br.hi = block_max1(mx, red);
  br.live = target < N;
  for (int p = 0; p < passes; ++p) {
    br.live = br.live && (br.hi - br.lo > 4.0 * eps);
    if (!br.live) break;
    for (int k = threadIdx.x; k < 2 * NB; k += blockDim.x) sh[k] = w.hist[(size_t)p * 2 * NB + k];
    __syncthreads();
    const double step = (br.hi - br.lo) / (NP + 1);
    unsigned long long c1 = 0, c2 = 0;   // #{q > probe j}, #{q > probe j + eps}
    double nlo = br.lo, nhi = br.hi;
    for (int j = NP - 1; j >= 0; --j) {
      c1 += sh[j + 1];
      c2 += sh[NB + j + 1];
      const double pj = probe(br.lo, step, j);
      if ((double)c2 > target && pj > nlo) nlo = pj;
      if ((double)c1 <= target && pj < nhi) nhi = pj;
    }
    __syncthreads();
    if (!(nhi - nlo < br.hi - br.lo)) {
      br.live = false;
      break;
    }
    br.lo = nlo;
    br.hi = nhi;
  }
  return br;
}

__device__ __forceinline__ void chunk_of(int64_t N, int G, int64_t& i0, int64_t& i1) {
  const int64_t chunk = (N + G - 1) / G;
  i0 = (int64_t)blockIdx.x * chunk;
  i1 = i0 + chunk < N ? i0 + chunk : N;
}

// Safeguarded Newton for Phi(t) = target inside [lo, hi]; phi(t, v) returns
// v[0] = Phi(t), v[1] = -Phi'(t) = sum s_eps''.  Block-uniform.
template <class F>
__device__ double newton_in_bracket(double lo, double hi, double target, F phi) {
  double tc = 0.5 * (lo + hi);
  double t = tc;
  double dx_old = hi - lo;
  for (int guard = 0; guard < 4096 && lo < hi; ++guard) {
    double v[2];
    phi(tc, v);
    if (v[0] > target) lo = tc;
    else hi = tc;
    const double mid = 0.5 * (lo + hi);
    t = mid;
    if (mid <= lo || mid >= hi) break;
    double tn = mid;
    if (v[1] > 0.0) {
      const double tnew = tc + (v[0] - target) / v[1];
      if (tnew > lo && tnew < hi && fabs(tnew - tc) <= 0.5 * dx_old) tn = tnew;
    }
    const double dx = fabs(tn - tc);
    dx_old = dx;
    tc = tn;
    t = tn;
    if (dx <= 4.0 * DBL_EPSILON * fabs(tn)) break;
  }
  double v[2];
  phi(t, v);
  if (v[1] > 0.0) {   // polish, kept inside the final bracket
    const double tn = t + (v[0] - target) / v[1];
    if (tn >= lo && tn <= hi) t = tn;
  }
  return t;
}

}  // namespace

// 1. partial min / max per workgroup; workgroup 0 clears the counters.
__global__ void __launch_bounds__(RBS) saa_k_cvar_minmax(const double* q, int64_t N, CvarWork w, int G) {
  __shared__ double red[RBS / SAA_WAVE];
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  double mn = INFINITY, mx = -INFINITY;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RBS) {
    mn = fmin(mn, q[i]);
    mx = fmax(mx, q[i]);
  }
  mn = block_min1(mn, red);
  mx = block_max1(mx, red);
  if (threadIdx.x == 0) {
    w.mm[2 * blockIdx.x] = mn;
    w.mm[2 * blockIdx.x + 1] = mx;
  }
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < PASSES * 2 * NB; k += RBS) w.hist[k] = 0;
    if (threadIdx.x < 2) w.act[threadIdx.x] = 0;
  }
}

// 2. bracketing pass p: probe histograms of this workgroup's chunk.
__global__ void __launch_bounds__(RBS) saa_k_cvar_probe(const double* q, int64_t N, CvarWork w, int G, int p,
                                                        double eps, double target) {
  __shared__ double red[RBS / SAA_WAVE];
  __shared__ unsigned long long sh[2 * NB];
  __shared__ unsigned int hl[2 * NB];
  const Bracket br = bracket_after(w, G, p, eps, target, (double)N, red, sh);
  if (!(br.live && br.hi - br.lo > 4.0 * eps)) return;
  for (int k = threadIdx.x; k < 2 * NB; k += RBS) hl[k] = 0;
  __syncthreads();
  const double step = (br.hi - br.lo) / (NP + 1);
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RBS) {
    const double qi = q[i];
    atomicAdd(&hl[probes_below(qi, br.lo, step, 0.0)], 1u);
    atomicAdd(&hl[NB + probes_below(qi, br.lo, step, eps)], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * NB; k += RBS)
    if (hl[k]) atomicAdd(&w.hist[(size_t)p * 2 * NB + k], (unsigned long long)hl[k]);
}

// 3. gather the active set (lo < q < hi + eps); count q >= hi + eps.
__global__ void __launch_bounds__(RBS) saa_k_cvar_compact(const double* q, int64_t N, CvarWork w, int G,
                                                          double eps, double target) {
  __shared__ double red[RBS / SAA_WAVE];
  __shared__ unsigned long long sh[2 * NB];
  const Bracket br = bracket_after(w, G, PASSES, eps, target, (double)N, red, sh);
  if (!(target < (double)N)) return;
  const double top = br.hi + eps;
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  double above = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RBS) {
    const double qi = q[i];
    if (qi >= top) {
      above += 1.0;
    } else if (qi > br.lo) {
      const unsigned long long k = atomicAdd(&w.act[0], 1ull);
      if (k < (unsigned long long)CAP) w.aval[k] = qi;
    }
  }
  above = block_sum1(above, red);
  if (threadIdx.x == 0 && above > 0.0) atomicAdd(&w.act[1], (unsigned long long)above);
}

// 4. t* (or t_in when t_mode = 1) -> tstar[0].
__global__ void __launch_bounds__(SBS) saa_k_cvar_solve(const double* q, int64_t N, CvarWork w, int G, double eps,
                                                        double target, int t_mode, double t_in, double* tstar) {
  __shared__ double red[2 * (SBS / SAA_WAVE)];
  __shared__ unsigned long long sh[2 * NB];
  __shared__ double s[CAP];
  double t;
  if (t_mode == 1) {
    t = t_in;
  } else {
    const Bracket br = bracket_after(w, G, PASSES, eps, target, (double)N, red, sh);
    if (!(target < (double)N)) {
      t = br.lo;   // beta = 0: every t <= min q - eps is a minimiser
    } else {
      const unsigned long long na = w.act[0];
      if (na <= (unsigned long long)CAP) {
        const int n = (int)na;
        const double above = (double)w.act[1];
        int npad = 1;
        while (npad < n) npad <<= 1;
        for (int i = threadIdx.x; i < npad; i += SBS) s[i] = i < n ? w.aval[i] : INFINITY;
        __syncthreads();
        // bitonic sort: the arrival order of the active set is not fixed
        for (int k = 2; k <= npad; k <<= 1) {
          for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < npad; i += SBS) {
              const int l = i ^ j;
              if (l > i) {
                const double a = s[i], b = s[l];
                if ((a > b) == ((i & k) == 0)) {
                  s[i] = b;
                  s[l] = a;
                }
              }
            }
            __syncthreads();
          }
        }
        t = newton_in_bracket(br.lo, br.hi, target, [&](double tc, double* v) {
          double a[2] = {0.0, 0.0};
          for (int i = threadIdx.x; i < n; i += SBS) {
            a[0] += sp_d1(s[i] - tc, eps);
            a[1] += sp_d2(s[i] - tc, eps);
          }
          block_sum<2>(a, red);
          v[0] = above + a[0];
          v[1] = a[1];
        });
      } else {
        t = newton_in_bracket(br.lo, br.hi, target, [&](double tc, double* v) {
          double a[2] = {0.0, 0.0};
          for (int64_t i = threadIdx.x; i < N; i += SBS) {
            a[0] += sp_d1(q[i] - tc, eps);
            a[1] += sp_d2(q[i] - tc, eps);
          }
          block_sum<2>(a, red);
          v[0] = a[0];
          v[1] = a[1];
        });
      }
    }
  }
  if (threadIdx.x == 0) tstar[0] = t;
}

// 5. per-workgroup partial sums: sum s_eps, sum s_eps', sum s_eps' dq/dz.
__global__ void __launch_bounds__(RBS) saa_k_cvar_part(const double* q, const double* g, int64_t N, int dz,
                                                       CvarWork w, int G, double eps, const double* tstar) {
  __shared__ double red[8 * (RBS / SAA_WAVE)];
  const double t = tstar[0];
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  double v[2] = {0.0, 0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RBS) {
    const double x = q[i] - t;
    v[0] += sp_val(x, eps);
    v[1] += sp_d1(x, eps);
  }
  block_sum<2>(v, red);
  double* pp = w.part + (size_t)blockIdx.x * PSTRIDE;
  if (threadIdx.x == 0) {
    pp[0] = v[0];
    pp[1] = v[1];
  }
  for (int k0 = 0; k0 < dz; k0 += 8) {
    double a[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) a[c] = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += RBS) {
      const double wi = sp_d1(q[i] - t, eps);
      if (wi != 0.0) {
        const double* gi = g + i * dz;
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (k0 + c < dz) a[c] += wi * gi[k0 + c];
      }
    }
    block_sum<8>(a, red);
    if (threadIdx.x == 0)
      for (int c = 0; c < 8 && k0 + c < dz; ++c) pp[2 + k0 + c] = a[c];
  }
}

// 6. reduce the partials in chunk order -> out[0] = J, out[1] = dJ/dt,
// out[2..2+dz) = grad (when `outputs`); optional per-sample solver stats.
__global__ void __launch_bounds__(SBS) saa_k_cvar_final(int64_t N, int dz, CvarWork w, int G, double target,
                                                        double alpha, const double* z, const double* tstar,
                                                        int outputs, double* out, const int* newton, const int* lin,
                                                        const int* flag, const int* lin_adj, const int* did,
                                                        CvarStats* stats) {
  __shared__ double red[5 * (SBS / SAA_WAVE)];
  if (stats) {
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double nm = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += SBS) {
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
  if (!outputs) return;
  const int k = threadIdx.x;
  if (k >= 2 + dz) return;
  double acc = 0.0;
  for (int b = 0; b < G; ++b) acc += w.part[(size_t)b * PSTRIDE + k];
  const double scale = 1.0 / target;
  if (k == 0) {
    double zz = 0.0;
    for (int c = 0; c < dz; ++c) zz += z[c] * z[c];
    out[0] = tstar[0] + scale * acc + 0.5 * alpha * zz;
  } else if (k == 1) {
    out[1] = 1.0 - scale * acc;
  } else {
    out[k] = scale * acc + alpha * z[k - 2];
  }
}

namespace saa_launch {

size_t cvar_work_bytes() {
  return sizeof(double) * 2 * GMAX + sizeof(unsigned long long) * (PASSES * 2 * NB + 2) + sizeof(double) * CAP +
         sizeof(double) * (size_t)GMAX * PSTRIDE;
}

// phase & 1: t (minimiser, or t_in when t_mode = 1) -> tstar[0];
// phase & 2: J, dJ/dt, grad -> out; stats (if non-null) -> stats.
void cvar(const double* q, const double* g, int64_t N, int dz, double beta, double eps, double alpha,
          const double* z, int t_mode, double t_in, int phase, double* tstar, double* out, const int* newton,
          const int* lin, const int* flag, const int* lin_adj, const int* did, void* stats, void* work,
          hipStream_t st) {
  CvarWork w;
  char* p = (char*)work;
  w.mm = (double*)p;
  p += sizeof(double) * 2 * GMAX;
  w.part = (double*)p;
  p += sizeof(double) * (size_t)GMAX * PSTRIDE;
  w.aval = (double*)p;
  p += sizeof(double) * CAP;
  w.hist = (unsigned long long*)p;
  p += sizeof(unsigned long long) * PASSES * 2 * NB;
  w.act = (unsigned long long*)p;
  const int64_t gw = (N + 1023) / 1024;
  const int G = (int)(gw < 1 ? 1 : gw > GMAX ? GMAX : gw);
  const double target = (double)N * (1.0 - beta);
  if (phase & 1) {
    if (t_mode != 1) {
      saa_k_cvar_minmax<<<G, RBS, 0, st>>>(q, N, w, G);
      for (int ps = 0; ps < PASSES; ++ps) saa_k_cvar_probe<<<G, RBS, 0, st>>>(q, N, w, G, ps, eps, target);
      saa_k_cvar_compact<<<G, RBS, 0, st>>>(q, N, w, G, eps, target);
    }
    saa_k_cvar_solve<<<1, SBS, 0, st>>>(q, N, w, G, eps, target, t_mode, t_in, tstar);
  }
  if (phase & 2) saa_k_cvar_part<<<G, RBS, 0, st>>>(q, g, N, dz, w, G, eps, tstar);
  if ((phase & 2) || stats)
    saa_k_cvar_final<<<1, SBS, 0, st>>>(N, dz, w, G, target, alpha, z, tstar, (phase & 2) ? 1 : 0, out, newton, lin,
                                        flag, lin_adj, did, (CvarStats*)stats);
}

}  // namespace saa_launch
