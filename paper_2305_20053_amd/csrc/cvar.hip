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
//     PP = 256 equispaced probes (exact binary search over the probe values)
//     and the bracket shrinks about 128-fold, until it is a few eps wide;
//  3. compact (G workgroups): samples in (lo, hi + eps) are the only ones
//     whose s_eps' varies inside the bracket; each workgroup gathers its
//     "active" samples in index order and counts those at or above hi + eps
//     (their s_eps' is 1 throughout the bracket);
//  3b. only if the active set overflows its capacity (q within a few eps of
//     each other, as trained surrogates give): RPASSES refinement passes
//     (G workgroups) evaluate Phi exactly at 64 points of the bracket and
//     keep the crossing pair;
//  4. solve (1 workgroup): the active samples are concatenated in workgroup
//     order in LDS and a safeguarded Newton iteration on
//         Phi(t) = #{q >= hi + eps} + sum_active s_eps'(q_a - t)
//     runs inside the bracket (bisection when a step leaves it or stalls),
//     followed by one polish step; after an overflow, the root of the cubic
//     through Phi at four points of the last refinement pass around the
//     crossing.
// Every wave recomputes the bracket from the previous launches' results with
// the same arithmetic, so all of them agree on it without a grid barrier.
// For beta = 0 (target = N) every t <= min(q) - eps is a minimiser with the
// same J and weights; t* = min(q) - eps is returned.
//
// The value and gradient (eq. (ouu_risk_gradient), chain rule with weights
// w_i = s_eps'(q_i - t*) / (N (1-beta)); dJ_hat/dt = 0 at t*, so no t*
// derivative enters) are per-workgroup partial sums over contiguous chunks,
// reduced in chunk order by one workgroup.  Every sum has a fixed order, so
// results are bitwise reproducible.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <mutex>

#include "../../include/saa.h"
#include "common.h"
#include "pde.h"

namespace {

constexpr int RBS = 256;          // threads of the multi-workgroup passes
constexpr int SBS = 1024;         // threads of the single-workgroup kernels
constexpr int NP = 64;            // points per refinement pass (one per lane)
constexpr int PP = 256;           // probes per bracketing pass (four per lane)
constexpr int PPL = PP / 64;      // probes of one lane: 4 lane .. 4 lane + 3
constexpr int PASSES = 2;         // bracketing passes (shrink ~128x each)
constexpr int CAP = 1024;         // active-set capacity (doubles in LDS); larger sets take the refinement passes
constexpr int SEG = 1024;         // active-set capacity per workgroup
constexpr int GMAX = 256;         // workgroups of the multi-workgroup passes
constexpr int TILE = 4 * RBS;     // samples per compaction tile
constexpr int PSTRIDE = 2 + SAA_MAX_DZ;
constexpr int WAVE_NEWTON = 256;  // active sets up to this size are solved by one wave
constexpr int RPASSES = 3;        // refinement passes when the active set overflows
constexpr int RFB = 1024;         // threads of the refinement passes (16 waves share a chunk)
constexpr int SLOTS = 8;          // copies of each atomic counter (workgroup b adds to copy b % SLOTS)

// Workspace of one reduction: per-workgroup min / max and partial sums, the
// active-set segments, the refinement sums, the probe histograms and the
// active-set counters (about 2.3 MB, independent of N).
constexpr size_t kCvarWorkBytes =
    sizeof(double) * ((size_t)2 * GMAX + (size_t)GMAX * PSTRIDE + (size_t)GMAX * SEG) +
    sizeof(unsigned long long) * RPASSES * SLOTS * NP + sizeof(int) * ((size_t)PASSES * SLOTS * 2 * PP + 2 * GMAX + SLOTS);
constexpr int kMaxDevices = 64;
static_assert(NP == SAA_WAVE && PPL * SAA_WAVE == PP && PPL == 4, "refinement point per lane, four probes per lane");
static_assert(GMAX % SAA_WAVE == 0, "partial rows per lane in the final reduction");
static_assert(SAA_MAX_DZ <= SAA_WAVE, "one gradient component per lane");

// Device workspace, carved from one allocation of cvar_work_bytes().
struct CvarWork {
  double* mm;     // [GMAX][2] partial min / max of q
  double* part;   // [PSTRIDE][GMAX] partial sums of the value / gradient (column c of workgroup b at c GMAX + b)
  double* aval;   // [GMAX][SEG] active q values per workgroup, in index order
  // The counters that every workgroup adds to are kept in SLOTS copies, so
  // that fewer atomics meet on one address; readers add the copies up.
  int* hist;      // [PASSES][SLOTS][2][PP] probe histograms: entry j counts q with j + 1 probes below (no
                  // entry for 0: the counts only enter through #{q > probe j})
  int* nact;      // [GMAX] active samples per workgroup
  int* nabove;    // [GMAX] samples at or above hi + eps per workgroup
  int* act_total; // [SLOTS] active samples over all workgroups
  unsigned long long* fix;   // [RPASSES][SLOTS][NP] Phi at the refinement points, fixed point
  double fscale;  // the fixed-point scale: 2^38, lowered for N >= 2^24 so N fscale < 2^62
};

// s_eps and its derivatives; ie = 1 / e (one division per kernel, not per sample)
__device__ __forceinline__ double sp_val(double x, double e, double ie) {
  if (x <= 0.0) return 0.0;
  if (x >= e) return x - 0.5 * e;
  const double r = x * ie;
  return x * r * r * (1.0 - 0.5 * r);      // x^3/e^2 - x^4/(2 e^3)
}
__device__ __forceinline__ double sp_d1(double x, double e, double ie) {
  if (x <= 0.0) return 0.0;
  if (x >= e) return 1.0;
  const double r = x * ie;
  return r * r * (3.0 - 2.0 * r);          // 3x^2/e^2 - 2x^3/e^3
}
__device__ __forceinline__ double sp_d2(double x, double e, double ie) {
  if (x <= 0.0 || x >= e) return 0.0;
  const double r = x * ie;
  return 6.0 * r * (1.0 - r) * ie;         // 6x/e^2 - 6x^2/e^3
}

// Wave-wide max / min / integer sums and suffix sums from DPP row moves and
// lane reads.  They run at the head of every pass, on the serial path of the
// reduction, where shuffles routed through the LDS unit cost several times
// more.  Max, min and integer sums are exact, so the results do not depend on
// the combining order.
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);   // lanes without a source read 0
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  return __hiloint2double(dpp_mov<CTRL>(__double2hiint(v)), dpp_mov<CTRL>(__double2loint(v)));
}
__device__ __forceinline__ double lane_read(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
constexpr int DPP_XOR1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;
constexpr int DPP_SHR = 0x110;        // + n: row_shr:n

template <bool MAX>
__device__ __forceinline__ double wave_ext(double v) {
  auto op = [](double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); };
  v = op(v, dpp_mov<DPP_XOR1>(v));          // quads
  v = op(v, dpp_mov<DPP_XOR2>(v));
  v = op(v, dpp_mov<DPP_HALF_MIRROR>(v));   // rows of 8, then 16
  v = op(v, dpp_mov<DPP_MIRROR>(v));
  return op(op(lane_read(v, 0), lane_read(v, 16)), op(lane_read(v, 32), lane_read(v, 48)));
}
__device__ __forceinline__ double fast_max(double v) { return wave_ext<true>(v); }
// Sum over the lanes in one fixed tree order (quads, half rows, rows, then
// ((row 0 + row 1) + (row 2 + row 3))); every lane gets the same value.
__device__ __forceinline__ double fast_sum(double v) {
  v += dpp_mov<DPP_XOR1>(v);
  v += dpp_mov<DPP_XOR2>(v);
  v += dpp_mov<DPP_HALF_MIRROR>(v);
  v += dpp_mov<DPP_MIRROR>(v);
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}
__device__ __forceinline__ double fast_min(double v) { return wave_ext<false>(v); }

// Inclusive prefix sum over the lanes; *total gets the sum of all 64.
__device__ __forceinline__ int wave_prefix(int v, int* total) {
  v += dpp_mov<DPP_SHR + 1>(v);   // inclusive scans of each row of 16
  v += dpp_mov<DPP_SHR + 2>(v);
  v += dpp_mov<DPP_SHR + 4>(v);
  v += dpp_mov<DPP_SHR + 8>(v);
  const int t0 = __builtin_amdgcn_readlane(v, 15), t1 = __builtin_amdgcn_readlane(v, 31);
  const int t2 = __builtin_amdgcn_readlane(v, 47), t3 = __builtin_amdgcn_readlane(v, 63);
  const int row = (threadIdx.x & (SAA_WAVE - 1)) >> 4;
  *total = t0 + t1 + t2 + t3;
  return v + (row >= 1 ? t0 : 0) + (row >= 2 ? t1 : 0) + (row >= 3 ? t2 : 0);
}
__device__ __forceinline__ int fast_sum(int v) {
  int t;
  (void)wave_prefix(v, &t);
  return t;
}
// sum_{k >= lane} v_k
__device__ __forceinline__ int wave_suffix(int v) {
  int t;
  const int p = wave_prefix(v, &t);
  return t - p + v;
}

// Probe j of a pass over [lo, hi]; non-decreasing in j for any rounding.
__device__ __forceinline__ double probe(double lo, double step, int j) { return lo + (double)(j + 1) * step; }

// #{j < PP : probe(j) + shift < x}, exact (binary search over monotone probes).
__device__ __forceinline__ int probes_below(double x, double lo, double step, double shift) {
  int a = 0, b = PP;
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

// Bracket after `passes` bracketing passes, recomputed from the workspace by
// each wave on its own (lane l evaluates probes 4 l .. 4 l + 3); every wave of
// every workgroup gets the same result.  No LDS, no barrier.
__device__ Bracket bracket_after(const CvarWork& w, int G, int passes, double eps, double target, double N) {
  const int lane = threadIdx.x & (SAA_WAVE - 1);
  // every load is issued up front (none depends on the bracket): one memory
  // round trip instead of one per pass; entries 4 l .. 4 l + 3 of a row are
  // one 16-byte load
  double mn = INFINITY, mx = -INFINITY;
  int4 hc1[PASSES], hc2[PASSES];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    hc1[p] = make_int4(0, 0, 0, 0);
    hc2[p] = make_int4(0, 0, 0, 0);
    if (p < passes) {
#pragma unroll
      for (int k = 0; k < SLOTS; ++k) {
        const int4 a = *(const int4*)(w.hist + (size_t)(p * SLOTS + k) * 2 * PP + PPL * lane);
        const int4 b = *(const int4*)(w.hist + (size_t)(p * SLOTS + k) * 2 * PP + PP + PPL * lane);
        hc1[p].x += a.x;
        hc1[p].y += a.y;
        hc1[p].z += a.z;
        hc1[p].w += a.w;
        hc2[p].x += b.x;
        hc2[p].y += b.y;
        hc2[p].z += b.z;
        hc2[p].w += b.w;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < GMAX / SAA_WAVE; ++k) {
    const int b = lane + k * SAA_WAVE;
    if (b < G) {
      mn = fmin(mn, w.mm[2 * b]);
      mx = fmax(mx, w.mm[2 * b + 1]);
    }
  }
  Bracket br;
  br.lo = fast_min(mn) - eps;
  br.hi = fast_max(mx);
  br.live = target < N;
#pragma unroll
  for (int p = 0; p < PASSES; ++p) {
    if (p >= passes) break;
    br.live = br.live && (br.hi - br.lo > 4.0 * eps);
    if (!br.live) break;
    // #{q > probe j} = sum of the entries j .. PP - 1 (and the same with
    // probe j + eps): suffix sums over the lanes' totals, then within a lane
    const int4 e1 = hc1[p], e2 = hc2[p];
    const int s1 = wave_suffix(e1.x + e1.y + e1.z + e1.w), s2 = wave_suffix(e2.x + e2.y + e2.z + e2.w);
    const int c1[PPL] = {s1, s1 - e1.x, s1 - e1.x - e1.y, s1 - e1.x - e1.y - e1.z};
    const int c2[PPL] = {s2, s2 - e2.x, s2 - e2.x - e2.y, s2 - e2.x - e2.y - e2.z};
    const double step = (br.hi - br.lo) / (PP + 1);
    double lo_c = br.lo, hi_c = br.hi;
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const double pj = probe(br.lo, step, PPL * lane + i);
      if ((double)c2[i] > target) lo_c = fmax(lo_c, pj);
      if ((double)c1[i] <= target) hi_c = fmin(hi_c, pj);
    }
    const double nlo = fast_max(lo_c);
    const double nhi = fast_min(hi_c);
    if (!(nhi - nlo < br.hi - br.lo)) {
      br.live = false;
      break;
    }
    br.lo = nlo;
    br.hi = nhi;
  }
  return br;
}

// Active samples over all workgroups (above CAP: overflow).
__device__ __forceinline__ int active_total(const CvarWork& w) {
  int t = 0;
#pragma unroll
  for (int k = 0; k < SLOTS; ++k) t += w.act_total[k];
  return t;
}

// The bracket (and the overflow flag) computed by wave 0 of the workgroup
// and passed to the others through LDS (sb: 4 doubles), so that the
// workgroup reads the shared counters once rather than once per wave.  All
// threads must call.
struct Shared {
  Bracket br;
  bool overflow;
};
__device__ Shared shared_bracket(const CvarWork& w, int G, int passes, double eps, double target, double N,
                                 double* sb) {
  if (threadIdx.x < SAA_WAVE) {
    const Bracket br = bracket_after(w, G, passes, eps, target, N);
    const bool ov = active_total(w) > CAP;
    if (threadIdx.x == 0) {
      sb[0] = br.lo;
      sb[1] = br.hi;
      sb[2] = br.live ? 1.0 : 0.0;
      sb[3] = ov ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  Shared r;
  r.br.lo = sb[0];
  r.br.hi = sb[1];
  r.br.live = sb[2] != 0.0;
  r.overflow = sb[3] != 0.0;
  return r;
}

__device__ __forceinline__ void chunk_of(int64_t N, int G, int64_t& i0, int64_t& i1) {
  const int64_t chunk = (N + G - 1) / G;
  i0 = (int64_t)blockIdx.x * chunk;
  i1 = i0 + chunk < N ? i0 + chunk : N;
}

// Safeguarded Newton for Phi(t) = target inside [lo, hi]; phi(t, v) returns
// v[0] = Phi(t), v[1] = -Phi'(t) = sum s_eps''.  Uniform over its callers.
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

// Exclusive prefix sum over the block of one int per thread (thread order);
// returns the block total.  `sh` holds blockDim.x / 64 ints of LDS.
__device__ int block_scan(int v, int* excl, int* sh) {
  const int lane = threadIdx.x & (SAA_WAVE - 1), wid = threadIdx.x / SAA_WAVE;
  const int nw = blockDim.x / SAA_WAVE;
  int x = v;
#pragma unroll
  for (int off = 1; off < SAA_WAVE; off <<= 1) {
    const int y = __shfl_up(x, off, SAA_WAVE);
    if (lane >= off) x += y;
  }
  if (lane == SAA_WAVE - 1) sh[wid] = x;
  __syncthreads();
  int base = 0, total = 0;
  for (int k = 0; k < nw; ++k) {
    base += k < wid ? sh[k] : 0;
    total += sh[k];
  }
  __syncthreads();
  *excl = base + x - v;
  return total;
}

}  // namespace

// 1. partial min / max per workgroup; the workgroups together clear the
// counters of the later passes.
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
  const int gt = blockIdx.x * RBS + threadIdx.x, gs = G * RBS;
  for (int k = gt; k < PASSES * SLOTS * 2 * PP; k += gs) w.hist[k] = 0;
  for (int k = gt; k < RPASSES * SLOTS * NP; k += gs) w.fix[k] = 0;
  for (int k = gt; k < SLOTS; k += gs) w.act_total[k] = 0;
}

// 2. bracketing pass p: probe histograms of this workgroup's chunk.
__global__ void __launch_bounds__(RBS) saa_k_cvar_probe(const double* q, int64_t N, CvarWork w, int G, int p,
                                                        double eps, double target) {
  __shared__ int hl[2 * PP];
  __shared__ double sb[4];
  const Bracket br = shared_bracket(w, G, p, eps, target, (double)N, sb).br;
  if (!(br.live && br.hi - br.lo > 4.0 * eps)) return;
  for (int k = threadIdx.x; k < 2 * PP; k += RBS) hl[k] = 0;
  __syncthreads();
  const double step = (br.hi - br.lo) / (PP + 1);
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  // samples below every probe are not counted; those above every probe
  // (entry PP - 1) are counted in registers, so the LDS atomics only see
  // the samples in between
  int edge[2] = {0, 0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RBS) {
    const double qi = q[i];
    const int b1 = probes_below(qi, br.lo, step, 0.0);
    const int b2 = probes_below(qi, br.lo, step, eps);
    if (b1 == PP) ++edge[0];
    else if (b1 > 0) atomicAdd(&hl[b1 - 1], 1);
    if (b2 == PP) ++edge[1];
    else if (b2 > 0) atomicAdd(&hl[PP + b2 - 1], 1);
  }
  edge[0] = fast_sum(edge[0]);
  edge[1] = fast_sum(edge[1]);
  if ((threadIdx.x & (SAA_WAVE - 1)) == 0) {
    atomicAdd(&hl[PP - 1], edge[0]);
    atomicAdd(&hl[2 * PP - 1], edge[1]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * PP; k += RBS)
    if (hl[k]) atomicAdd(&w.hist[(size_t)(p * SLOTS + blockIdx.x % SLOTS) * 2 * PP + k], hl[k]);
}

// 3. gather this workgroup's active samples (lo < q < hi + eps) in index
// order; count the samples at or above hi + eps.
__global__ void __launch_bounds__(RBS) saa_k_cvar_compact(const double* q, int64_t N, CvarWork w, int G,
                                                          double eps, double target) {
  __shared__ int sh[RBS / SAA_WAVE];
  __shared__ double sb[4];
  const Bracket br = shared_bracket(w, G, PASSES, eps, target, (double)N, sb).br;
  if (!(target < (double)N)) return;
  const double top = br.hi + eps;
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  double* seg = w.aval + (size_t)blockIdx.x * SEG;
  int base = 0, above = 0;
  for (int64_t t0 = i0; t0 < i1; t0 += TILE) {
    double v[4];
    bool a[4];
    int n = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {   // thread-contiguous samples keep index order
      const int64_t i = t0 + 4 * threadIdx.x + r;
      v[r] = i < i1 ? q[i] : -INFINITY;
      above += v[r] >= top ? 1 : 0;
      a[r] = v[r] < top && v[r] > br.lo;
      n += a[r] ? 1 : 0;
    }
    int pos;
    const int tot = block_scan(n, &pos, sh);
    pos += base;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (a[r]) {
        if (pos < SEG) seg[pos] = v[r];
        ++pos;
      }
    }
    base += tot;
  }
  above = fast_sum(above);
  if ((threadIdx.x & (SAA_WAVE - 1)) == 0) sh[threadIdx.x / SAA_WAVE] = above;
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0;
    for (int k = 0; k < RBS / SAA_WAVE; ++k) a += sh[k];
    w.nact[blockIdx.x] = base;
    w.nabove[blockIdx.x] = a;
    // a segment overflow counts as an overflow of the whole active set
    if (base > 0) atomicAdd(&w.act_total[blockIdx.x % SLOTS], base > SEG ? base + CAP + 1 : base);
  }
}

// Bracket after the count passes and `passes` refinement passes.  Pass r
// evaluated Phi exactly at the 64 points lo + j (hi - lo) / 63 (sums over all
// workgroups in fixed point, so their order does not matter); the new
// bracket is the pair of neighbouring points where Phi crosses the target.
// Once a refinement pass has run, pv[0..3] hold Phi at the four points
// j0 .. j0 + 3 of the last pass around the crossing pair (jl, jl + 1) and
// *lo4 = point j0, *h = the point spacing (pv[0] = -1 otherwise).  Every wave
// gets the same result.
struct Refined {
  Bracket br;
  double pv[4], lo4, h;
  int k;   // the crossing pair is points k, k + 1 of the four
};
__device__ Refined bracket_refined(const CvarWork& w, int G, int passes, double eps, double target, double N) {
  const int lane = threadIdx.x & (SAA_WAVE - 1);
  Refined R;
  R.br = bracket_after(w, G, PASSES, eps, target, N);
  R.pv[0] = -1.0;
  R.lo4 = R.h = 0.0;
  R.k = 0;
  unsigned long long f[RPASSES];
#pragma unroll
  for (int r = 0; r < RPASSES; ++r) {
    f[r] = 0ull;
    if (r < passes)
#pragma unroll
      for (int k = 0; k < SLOTS; ++k) f[r] += w.fix[(r * SLOTS + k) * NP + lane];
  }
#pragma unroll
  for (int r = 0; r < RPASSES; ++r) {
    Bracket& br = R.br;
    if (r >= passes || !(br.hi - br.lo > 8.0 * DBL_EPSILON * fmax(fabs(br.lo), fabs(br.hi)))) break;
    const double step = (br.hi - br.lo) / (NP - 1);
    const double pv = (double)f[r] / w.fscale;
    const int jl = (int)fast_max((double)((lane < NP - 1 && pv > target) ? lane : 0));
    const int j0 = jl < 1 ? 0 : (jl > NP - 3 ? NP - 4 : jl - 1);   // four points inside 0 .. 63
#pragma unroll
    for (int i = 0; i < 4; ++i) R.pv[i] = lane_read(pv, j0 + i);
    R.k = jl - j0;
    R.lo4 = br.lo + (double)j0 * step;
    R.h = step;
    const double tl = br.lo + (double)jl * step;
    const double th = jl + 1 == NP - 1 ? br.hi : br.lo + (double)(jl + 1) * step;
    br.lo = tl;
    br.hi = th;
  }
  return R;
}

// Root in [lo, hi] of the cubic through Phi at four equispaced points
// (pv[i] at lo4 + i h; the crossing pair is points k, k + 1, with lo, hi
// their abscissae): Newton from the secant point, kept inside [lo, hi].
// After three refinement passes h is about 4 eps / 63^3, and the cubic's
// error there is far below the rounding of t.
__device__ double cubic_root(const Refined& R, double target) {
  const double* p = R.pv;
  // Newton form on nodes 0, 1, 2, 3 (unit spacing)
  const double d1 = p[1] - p[0], d2 = (p[2] - 2.0 * p[1] + p[0]) * 0.5,
               d3 = (p[3] - 3.0 * p[2] + 3.0 * p[1] - p[0]) / 6.0;
  auto P = [&](double x) { return p[0] + x * (d1 + (x - 1.0) * (d2 + (x - 2.0) * d3)); };
  auto dP = [&](double x) {
    return d1 + d2 * (2.0 * x - 1.0) + d3 * (3.0 * x * x - 6.0 * x + 2.0);
  };
  const double a = (double)R.k, b = a + 1.0;
  const double pa = p[R.k], pb = p[R.k + 1];
  double x = pa > pb ? a + (pa - target) / (pa - pb) : a + 0.5;
  x = fmin(fmax(x, a), b);
  for (int it = 0; it < 4; ++it) {
    const double dp = dP(x);
    if (!(dp < 0.0)) break;
    x = fmin(fmax(x - (P(x) - target) / dp, a), b);
  }
  const double t = R.lo4 + x * R.h;
  return fmin(fmax(t, R.br.lo), R.br.hi);
}

// 3b. refinement pass r (only when the active set overflowed its capacity):
// Phi at 64 points of the current bracket, lane j evaluating point j over the
// window samples of this workgroup's chunk.  Wave k of the 16 takes the
// tile's samples k, k + 16, ..., four at a time (independent chains).
__global__ void __launch_bounds__(RFB) saa_k_cvar_refine(const double* q, int64_t N, CvarWork w, int G, int r,
                                                         double eps, double target) {
  constexpr int NWV = RFB / SAA_WAVE;
  __shared__ double part[NWV][NP];
  __shared__ double qt[TILE];
  __shared__ double sb[4];
  if (!(target < (double)N)) return;
  if (threadIdx.x < SAA_WAVE) {   // wave 0 finds the bracket; the others take it from LDS
    const bool ov = active_total(w) > CAP;
    const Refined R = bracket_refined(w, G, r, eps, target, (double)N);
    if (threadIdx.x == 0) {
      sb[0] = R.br.lo;
      sb[1] = R.br.hi;
      sb[2] = ov ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  Bracket br;
  br.lo = sb[0];
  br.hi = sb[1];
  if (sb[2] == 0.0) return;   // no overflow: no refinement
  if (!(br.hi - br.lo > 8.0 * DBL_EPSILON * fmax(fabs(br.lo), fabs(br.hi)))) return;
  const int lane = threadIdx.x & (SAA_WAVE - 1), wid = threadIdx.x / SAA_WAVE;
  const double ie = 1.0 / eps;
  const double step = (br.hi - br.lo) / (NP - 1);
  const double tj = lane == NP - 1 ? br.hi : br.lo + (double)lane * step;
  const double top = br.hi + eps, lo = br.lo;
  auto term = [&](double x) { return x >= top ? 1.0 : (x > lo ? sp_d1(x - tj, eps, ie) : 0.0); };
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t t0 = i0; t0 < i1; t0 += TILE) {
    const int nt = (int)(i1 - t0 < TILE ? i1 - t0 : TILE);
    for (int i = threadIdx.x; i < nt; i += RFB) qt[i] = q[t0 + i];
    __syncthreads();
    int i = wid;
    for (; i + 3 * NWV < nt; i += 4 * NWV) {
      const double x0 = qt[i], x1 = qt[i + NWV], x2 = qt[i + 2 * NWV], x3 = qt[i + 3 * NWV];
      acc[0] += term(x0);
      acc[1] += term(x1);
      acc[2] += term(x2);
      acc[3] += term(x3);
    }
    for (; i < nt; i += NWV) acc[0] += term(qt[i]);
    __syncthreads();
  }
  part[wid][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (wid == 0) {
    double v = 0.0;
    for (int k = 0; k < NWV; ++k) v += part[k][lane];
    if (v > 0.0)
      atomicAdd(&w.fix[(r * SLOTS + blockIdx.x % SLOTS) * NP + lane], (unsigned long long)llrint(v * w.fscale));
  }
}

// 4. t* (or t_in when t_mode = 1), by one workgroup of BSZ threads; every
// thread returns the same value.  LDS: s holds CAP doubles, off GMAX + 1
// ints, sh BSZ / 64 ints, red 2 BSZ / 64 doubles.
template <int BSZ>
__device__ double cvar_tstar(const CvarWork& w, int64_t N, int G, double eps, double target, int t_mode,
                             double t_in, double* s, int* off, int* sh, double* red, double* sb) {
  const int lane = threadIdx.x & (SAA_WAVE - 1);
  const double ie = 1.0 / eps;
  if (t_mode == 1) return t_in;
  const Shared S = shared_bracket(w, G, PASSES, eps, target, (double)N, sb);
  const Bracket br = S.br;
  if (!(target < (double)N)) return br.lo;   // beta = 0: every t <= min q - eps is a minimiser
  if (S.overflow) {
    // overflow (a segment overflow also pushes the total above CAP): the
    // refinement passes narrowed the bracket to (hi - lo) ~ 4 eps / 63^3;
    // the cubic through Phi at four points of the last pass finishes t*
    // (wave 0 computes it, the others take it from LDS)
    if (threadIdx.x < SAA_WAVE) {
      const Refined R = bracket_refined(w, G, RPASSES, eps, target, (double)N);
      double t = 0.5 * (R.br.lo + R.br.hi);
      if (R.pv[0] >= 0.0) t = cubic_root(R, target);
      if (threadIdx.x == 0) sb[0] = t;
    }
    __syncthreads();
    return sb[0];
  }
  // concatenate the per-workgroup active sets in workgroup order
  const int cb = threadIdx.x < G ? w.nact[threadIdx.x] : 0;
  const int ab = threadIdx.x < G ? w.nabove[threadIdx.x] : 0;
  bool fits = true;
  int ex;
  const int n = block_scan(cb, &ex, sh);
  if (threadIdx.x < G) off[threadIdx.x] = ex;
  if (threadIdx.x < G && cb > SEG) fits = false;
  int ex2;
  const double above = (double)block_scan(ab, &ex2, sh);
  // the total is <= CAP here, so no segment overflowed and n <= CAP
  fits = __syncthreads_and(fits) && n <= CAP;
  if (threadIdx.x == 0) off[G] = n;
  __syncthreads();
  double t = 0.5 * (br.lo + br.hi);   // (fits always holds here)
  if (fits) {
    for (int r = threadIdx.x; r < n; r += BSZ) {
      int a = 0, b = G;   // last workgroup with off <= r
      while (b - a > 1) {
        const int m = (a + b) >> 1;
        if (off[m] <= r) a = m;
        else b = m;
      }
      s[r] = w.aval[(size_t)a * SEG + (r - off[a])];
    }
    __syncthreads();
    if (n <= WAVE_NEWTON) {   // every wave on its own, no barriers
      t = newton_in_bracket(br.lo, br.hi, target, [&](double tc, double* v) {
        double a0 = 0.0, a1 = 0.0;
        for (int i = lane; i < n; i += SAA_WAVE) {
          a0 += sp_d1(s[i] - tc, eps, ie);
          a1 += sp_d2(s[i] - tc, eps, ie);
        }
        v[0] = above + fast_sum(a0);
        v[1] = fast_sum(a1);
      });
    } else {
      t = newton_in_bracket(br.lo, br.hi, target, [&](double tc, double* v) {
        double a[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < n; i += BSZ) {
          a[0] += sp_d1(s[i] - tc, eps, ie);
          a[1] += sp_d2(s[i] - tc, eps, ie);
        }
        // block sums: DPP within each wave, then the waves in order
        constexpr int NW = BSZ / SAA_WAVE;
        a[0] = fast_sum(a[0]);
        a[1] = fast_sum(a[1]);
        if (lane == 0) {
          red[threadIdx.x / SAA_WAVE] = a[0];
          red[NW + threadIdx.x / SAA_WAVE] = a[1];
        }
        __syncthreads();
        double s0 = 0.0, s1 = 0.0;
        for (int k = 0; k < NW; ++k) {
          s0 += red[k];
          s1 += red[NW + k];
        }
        __syncthreads();
        v[0] = above + s0;
        v[1] = s1;
      });
    }
  }
  return t;
}

// t* -> tstar[0].
__global__ void __launch_bounds__(SBS) saa_k_cvar_solve(int64_t N, CvarWork w, int G, double eps, double target,
                                                        int t_mode, double t_in, double* tstar) {
  __shared__ double red[2 * (SBS / SAA_WAVE)];
  __shared__ int off[GMAX + 1];
  __shared__ int sh[SBS / SAA_WAVE];
  __shared__ double s[CAP];
  __shared__ double sb[4];
  const double t = cvar_tstar<SBS>(w, N, G, eps, target, t_mode, t_in, s, off, sh, red, sb);
  if (threadIdx.x == 0) tstar[0] = t;
}

// Per-sample value v and weight d = dv/dq of a risk measure written as a mean
// of v(q_i) (t = tstar[0]):
//  RISK_CVAR      v = s_eps(q - t), d = s_eps'(q - t)        (eq. (CVaR_saa_ouu))
//  RISK_MEAN      v = q,            d = 1                    (eq. (saa))
//  RISK_MEAN_VAR  v = q + kappa (q - t)^2, d = 1 + 2 kappa (q - t), t = mean q
//                 (d/dq_i of the SAA variance: the mean's own derivative
//                 cancels since sum (q - t) = 0)
//  RISK_POF       v = s_eps'(q - t), d = s_eps''(q - t),     t = tau
//  RISK_BPOE      v = s_eps(a (q - tau) + 1), d = a s_eps'(a (q - tau) + 1),
//                 t = a, the minimiser over a >= 0 (d/da of the mean is 0
//                 there, so a does not move with z); a = infinity: v = d = 0
template <int KIND>
__device__ __forceinline__ void risk_terms(double qi, double t, double eps, double ie, double kappa, double tau,
                                           double& v, double& d) {
  if (KIND == SAA_RISK_CVAR) {
    const double x = qi - t;
    v = sp_val(x, eps, ie);
    d = sp_d1(x, eps, ie);
  } else if (KIND == SAA_RISK_MEAN) {
    v = qi;
    d = 1.0;
  } else if (KIND == SAA_RISK_MEAN_VAR) {
    const double x = qi - t;
    v = qi + kappa * x * x;
    d = 1.0 + 2.0 * kappa * x;
  } else if (KIND == SAA_RISK_POF) {
    const double x = qi - t;
    v = sp_d1(x, eps, ie);
    d = sp_d2(x, eps, ie);
  } else {
    if (!(t < INFINITY)) {
      v = 0.0;
      d = 0.0;
    } else {
      const double y = t * (qi - tau) + 1.0;
      v = sp_val(y, eps, ie);
      d = t * sp_d1(y, eps, ie);
    }
  }
}

// 5. per-workgroup partial sums: sum v, sum d, sum d dq/dz (see risk_terms).
// The weighted samples of each tile are listed in LDS; wave k of the block
// then takes every (RBS/64)-th of them with lane c accumulating component c.
template <int KIND>
__global__ void __launch_bounds__(RBS) saa_k_cvar_part(const double* q, const double* g, int64_t N, int dz,
                                                       CvarWork w, int G, double eps, double kappa, double tau,
                                                       const double* tstar) {
  __shared__ double red[2 * (RBS / SAA_WAVE)];
  __shared__ int sh[RBS / SAA_WAVE];
  __shared__ int li[TILE];
  __shared__ double lw[TILE];
  __shared__ double gw[RBS / SAA_WAVE][SAA_WAVE];
  const int lane = threadIdx.x & (SAA_WAVE - 1), wid = threadIdx.x / SAA_WAVE;
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  // the first tile's q is loaded before t (its latency overlaps that of t)
  double qv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = i0 + 4 * threadIdx.x + r;
    qv[r] = i < i1 ? q[i] : 0.0;
  }
  const double t = tstar[0];
  const double ie = 1.0 / eps;
  double v[2] = {0.0, 0.0};
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t t0 = i0; t0 < i1; t0 += TILE) {
    double d[4];
    int n = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = t0 + 4 * threadIdx.x + r;
      d[r] = 0.0;
      if (i < i1) {
        double vi;
        risk_terms<KIND>(t0 == i0 ? qv[r] : q[i], t, eps, ie, kappa, tau, vi, d[r]);
        v[0] += vi;
        v[1] += d[r];
      }
      n += d[r] != 0.0 ? 1 : 0;
    }
    int pos;
    const int tot = block_scan(n, &pos, sh);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (d[r] != 0.0) {
        li[pos] = 4 * threadIdx.x + r;
        lw[pos] = d[r];
        ++pos;
      }
    }
    __syncthreads();
    // wave k takes the weighted samples k, k + 4, ... in turn into four
    // accumulators (four independent load chains; a fixed order)
    constexpr int NW = RBS / SAA_WAVE;
    if (lane < dz) {
      int r = wid;
      for (; r + 3 * NW < tot; r += 4 * NW) {
        const double g0 = g[(t0 + li[r]) * dz + lane], g1 = g[(t0 + li[r + NW]) * dz + lane];
        const double g2 = g[(t0 + li[r + 2 * NW]) * dz + lane], g3 = g[(t0 + li[r + 3 * NW]) * dz + lane];
        acc[0] += lw[r] * g0;
        acc[1] += lw[r + NW] * g1;
        acc[2] += lw[r + 2 * NW] * g2;
        acc[3] += lw[r + 3 * NW] * g3;
      }
      for (; r < tot; r += NW) acc[0] += lw[r] * g[(t0 + li[r]) * dz + lane];
    }
    __syncthreads();
  }
  block_sum<2>(v, red);
  gw[wid][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  double* pp = w.part + blockIdx.x;   // column c of this workgroup's row at pp[c GMAX]
  if (threadIdx.x == 0) {
    pp[0] = v[0];
    pp[GMAX] = v[1];
  }
  if (threadIdx.x < dz) {
    double a = 0.0;
    for (int k = 0; k < RBS / SAA_WAVE; ++k) a += gw[k][threadIdx.x];
    pp[(size_t)(2 + threadIdx.x) * GMAX] = a;
  }
}

// 6. reduce the partials in a fixed order -> out[0] = J, out[1] = dJ/dt,
// out[2..2+dz) = grad (when `outputs`); optional per-sample solver stats.
__global__ void __launch_bounds__(SBS) saa_k_cvar_final(int64_t N, int dz, CvarWork w, int G, double target,
                                                        int kind, double alpha, const double* z, const double* tstar,
                                                        int outputs, double* out, const int* newton, const int* lin,
                                                        const int* flag, const int* lin_adj, const int* did,
                                                        CvarStats* stats) {
  constexpr int NW = SBS / SAA_WAVE;
  __shared__ double red[5 * NW];
  __shared__ double col[NW][PSTRIDE];
  __shared__ double zsh[SAA_WAVE];
  if (stats && !newton && !lin && !flag && !lin_adj && !did) {   // no per-sample solver (surrogate)
    if (threadIdx.x == 0) *stats = CvarStats{};
  } else if (stats) {
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
  // wave w sums columns w, w + NW, ... (at most CPW of them); lane l adds the
  // partial rows l, l + 64, l + 128, l + 192 in that order (loads
  // unconditional: rows clamped, zero weight past G), then a fixed-order
  // butterfly across the lanes
  const int lane = threadIdx.x & (SAA_WAVE - 1), wid = threadIdx.x / SAA_WAVE;
  const int ncol = 2 + dz;
  constexpr int CPW = (PSTRIDE + NW - 1) / NW;
  constexpr int RPL = GMAX / SAA_WAVE;
  double x[CPW][RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int b = lane + SAA_WAVE * r < G ? lane + SAA_WAVE * r : G - 1;
#pragma unroll
    for (int cc = 0; cc < CPW; ++cc) {
      const int c = wid + NW * cc < PSTRIDE ? wid + NW * cc : PSTRIDE - 1;
      x[cc][r] = w.part[(size_t)c * GMAX + b];
    }
  }
#pragma unroll
  for (int cc = 0; cc < CPW; ++cc) {
    double a = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) a += lane + SAA_WAVE * r < G ? x[cc][r] : 0.0;
    a = fast_sum(a);
    const int c = wid + NW * cc;
    if (lane == 0 && c < ncol) col[0][c] = a;
  }
  const int k = threadIdx.x;
  double zz = 0.0;
  if (k < SAA_WAVE) {   // |z|^2 by the whole of wave 0, one load per lane (z may be in host memory)
    const double zl = k < dz ? z[k] : 0.0;
    zsh[k] = zl;
    zz = fast_sum(zl * zl);
  }
  __syncthreads();
  if (k >= ncol) return;
  const double acc = col[0][k];
  const double scale = 1.0 / target;   // 1 / (N (1 - beta)) for CVaR, else 1 / N
  const bool cv = kind == SAA_RISK_CVAR;
  if (k == 0) {
    out[0] = (cv ? tstar[0] : 0.0) + scale * acc + 0.5 * alpha * zz;
  } else if (k == 1) {
    out[1] = cv ? 1.0 - scale * acc : 0.0;
  } else {
    out[k] = scale * acc + alpha * zsh[k - 2];
  }
}

// Mean of q for RISK_MEAN_VAR: per-workgroup partial sums (chunk order) ...
__global__ void __launch_bounds__(RBS) saa_k_risk_sum(const double* q, int64_t N, CvarWork w, int G) {
  __shared__ double red[2 * (RBS / SAA_WAVE)];
  int64_t i0, i1;
  chunk_of(N, G, i0, i1);
  double s[1] = {0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += RBS) s[0] += q[i];
  block_sum<1>(s, red);
  if (threadIdx.x == 0) w.mm[2 * blockIdx.x] = s[0];
}

// ... reduced in workgroup order by one wave -> tstar[0]; tau (POF), 0 (MEAN).
__global__ void __launch_bounds__(SAA_WAVE) saa_k_risk_t(int64_t N, CvarWork w, int G, int kind, double tau,
                                                         double* tstar) {
  if (kind != SAA_RISK_MEAN_VAR) {
    if (threadIdx.x == 0) tstar[0] = kind == SAA_RISK_POF ? tau : 0.0;
    return;
  }
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int b = 0; b < G; ++b) s += w.mm[2 * b];
  if (threadIdx.x == 0) tstar[0] = s / (double)N;
}

// a* of the buffered probability of exceedance (one workgroup): psi(a) =
// -sum_i s_eps'(a x_i + 1) x_i with x_i = q_i - tau is non-increasing in a
// (the mean of s_eps(a x + 1) is convex in a); a* = 0 when psi(0) <= 0, else
// the root of psi, bracketed by doubling and found by the safeguarded Newton
// iteration of the t* search; a* = infinity when no q_i exceeds tau.
__global__ void __launch_bounds__(SBS) saa_k_risk_bpoe(const double* q, int64_t N, double tau, double eps,
                                                       double* tstar) {
  __shared__ double red[2 * (SBS / SAA_WAVE)];
  const double ie = 1.0 / eps;
  auto psi = [&](double a, double* v) {
    double s[2] = {0.0, 0.0};
    for (int64_t i = threadIdx.x; i < N; i += SBS) {
      const double x = q[i] - tau;
      const double y = a * x + 1.0;
      s[0] -= sp_d1(y, eps, ie) * x;
      s[1] += sp_d2(y, eps, ie) * x * x;
    }
    block_sum<2>(s, red);
    v[0] = s[0];
    v[1] = s[1];
  };
  double qmax = -INFINITY;
  for (int64_t i = threadIdx.x; i < N; i += SBS) qmax = fmax(qmax, q[i]);
  qmax = block_max1(qmax, red);
  double a = 0.0;
  double v[2];
  psi(0.0, v);
  if (!(qmax > tau)) {
    a = INFINITY;
  } else if (v[0] > 0.0) {
    double lo = 0.0, hi = 1.0 / (qmax - tau);
    for (int k = 0; k < 200; ++k) {   // uniform over the block (block sums)
      psi(hi, v);
      if (!(v[0] > 0.0)) break;
      lo = hi;
      hi *= 4.0;
    }
    a = newton_in_bracket(lo, hi, 0.0, psi);
  }
  if (threadIdx.x == 0) tstar[0] = a;
}

// The workspace of the allocation-free reduction (saa_risk_reduce_noalloc):
// one copy per device, held until the process ends; every call on a device
// shares it (overlapping calls on one device race).
static_assert(kCvarWorkBytes == SAA_REDUCE_SCRATCH_BYTES, "the header states the workspace size");
static __device__ __align__(256) unsigned char scratch[kCvarWorkBytes];

namespace saa_launch {

size_t cvar_work_bytes() { return kCvarWorkBytes; }

// Device address of this device's copy of `scratch` (the workspace of the
// allocation-free reduction), looked up once per device with that device
// current and kept; the array's host-side name is never passed to a kernel.
int cvar_scratch(void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return SAA_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return SAA_E_DEVICE;
    }
    addr[dev] = p;
  }
  *out = addr[dev];
  return SAA_OK;
}

// phase & 1: t (minimiser, or t_in when t_mode = 1) -> tstar[0];
// phase & 2: J, dJ/dt, grad -> out; stats (if non-null) -> stats.
static CvarWork carve(void* work) {
  CvarWork w;
  char* p = (char*)work;
  w.mm = (double*)p;
  p += sizeof(double) * 2 * GMAX;
  w.part = (double*)p;
  p += sizeof(double) * (size_t)GMAX * PSTRIDE;
  w.aval = (double*)p;
  p += sizeof(double) * (size_t)GMAX * SEG;
  w.fix = (unsigned long long*)p;
  p += sizeof(unsigned long long) * RPASSES * SLOTS * NP;
  w.hist = (int*)p;
  p += sizeof(int) * PASSES * SLOTS * 2 * PP;
  w.nact = (int*)p;
  p += sizeof(int) * GMAX;
  w.nabove = (int*)p;
  p += sizeof(int) * GMAX;
  w.act_total = (int*)p;
  w.fscale = 1.0;
  return w;
}

static int groups(int64_t N) {   // 256 samples per workgroup, up to GMAX workgroups
  const int64_t gw = (N + 255) / 256;
  return (int)(gw < 1 ? 1 : gw > GMAX ? GMAX : gw);
}

void cvar(const double* q, const double* g, int64_t N, int dz, double beta, double eps, double alpha,
          const double* z, int t_mode, double t_in, int phase, double* tstar, double* out, const int* newton,
          const int* lin, const int* flag, const int* lin_adj, const int* did, void* stats, void* work,
          hipStream_t st) {
  CvarWork w = carve(work);
  w.fscale = std::ldexp(1.0, std::min(38, 61 - std::ilogb((double)N)));   // N < 2^(ilogb N + 1)
  const int G = groups(N);
  const double target = (double)N * (1.0 - beta);
  if (phase & 1) {
    if (t_mode != 1) {
      saa_k_cvar_minmax<<<G, RBS, 0, st>>>(q, N, w, G);
      for (int ps = 0; ps < PASSES; ++ps) saa_k_cvar_probe<<<G, RBS, 0, st>>>(q, N, w, G, ps, eps, target);
      saa_k_cvar_compact<<<G, RBS, 0, st>>>(q, N, w, G, eps, target);
      for (int r = 0; r < RPASSES; ++r) saa_k_cvar_refine<<<G, RFB, 0, st>>>(q, N, w, G, r, eps, target);
    }
    saa_k_cvar_solve<<<1, SBS, 0, st>>>(N, w, G, eps, target, t_mode, t_in, tstar);
  }
  if (phase & 2) saa_k_cvar_part<SAA_RISK_CVAR><<<G, RBS, 0, st>>>(q, g, N, dz, w, G, eps, 0.0, 0.0, tstar);
  if ((phase & 2) || stats)
    saa_k_cvar_final<<<1, SBS, 0, st>>>(N, dz, w, G, target, SAA_RISK_CVAR, alpha, z, tstar, (phase & 2) ? 1 : 0,
                                        out, newton, lin, flag, lin_adj, did, (CvarStats*)stats);
}

// Expectation-type risk measures (Sec. 2.1): phase & 1: t -> tstar[0] (mean of
// q for MEAN_VAR, in a fixed order; tau for POF; 0 for MEAN); phase & 2:
// J = (1/N) sum v_i + alpha/2 |z|^2, dJ/dt = 0, grad = (1/N) sum d_i dq_i/dz
// + alpha z (risk_terms).  Same workspace and result layout as cvar().
void risk(const double* q, const double* g, int64_t N, int dz, int kind, double eps, double kappa, double tau,
          double alpha, const double* z, int phase, double* tstar, double* out, const int* newton, const int* lin,
          const int* flag, const int* lin_adj, const int* did, void* stats, void* work, hipStream_t st) {
  const CvarWork w = carve(work);
  const int G = groups(N);
  if (phase & 1) {
    if (kind == SAA_RISK_BPOE) {
      saa_k_risk_bpoe<<<1, SBS, 0, st>>>(q, N, tau, eps, tstar);
    } else {
      if (kind == SAA_RISK_MEAN_VAR) saa_k_risk_sum<<<G, RBS, 0, st>>>(q, N, w, G);
      saa_k_risk_t<<<1, SAA_WAVE, 0, st>>>(N, w, G, kind, tau, tstar);
    }
  }
  if (phase & 2) {
    switch (kind) {
      case SAA_RISK_MEAN:
        saa_k_cvar_part<SAA_RISK_MEAN><<<G, RBS, 0, st>>>(q, g, N, dz, w, G, eps, kappa, tau, tstar);
        break;
      case SAA_RISK_MEAN_VAR:
        saa_k_cvar_part<SAA_RISK_MEAN_VAR><<<G, RBS, 0, st>>>(q, g, N, dz, w, G, eps, kappa, tau, tstar);
        break;
      case SAA_RISK_POF:
        saa_k_cvar_part<SAA_RISK_POF><<<G, RBS, 0, st>>>(q, g, N, dz, w, G, eps, kappa, tau, tstar);
        break;
      default:
        saa_k_cvar_part<SAA_RISK_BPOE><<<G, RBS, 0, st>>>(q, g, N, dz, w, G, eps, kappa, tau, tstar);
    }
  }
  if ((phase & 2) || stats)
    saa_k_cvar_final<<<1, SBS, 0, st>>>(N, dz, w, G, (double)N, kind, alpha, z, tstar, (phase & 2) ? 1 : 0, out,
                                        newton, lin, flag, lin_adj, did, (CvarStats*)stats);
}

}  // namespace saa_launch
