// PDE form on the unit cube: batched trilinear (Q1) finite-element Newton
// solves of -div(exp(m) grad u) + r u^3 = sum_k z_k f_k, u = 0 on the
// boundary (the equation of paper Sec. 4.2, eq. (elliptic_pde), in 3D), the
// tracking QoI and the adjoint gradient dq/dz = F^T lambda, A(u) lambda =
// dq/du (Sec. 2.3, eq. (ouu_qoi_gradient)).
//
// As in 2D, one workgroup owns one sample for its whole solve (256, 512 or
// 1024 threads, chosen by timing; at 48^3, N = 256 512 threads are fastest,
// 256 and 1024 take 1.6x as long):
// Newton in the state precision, inner multigrid-preconditioned CG in the
// solver precision, every decision taken on the device.
//
// Discretisation facts used here (they follow from the trilinear element
// matrices with one kappa per element, kappa_e = mean of exp(m) over its
// eight vertices):
//  * the unit-cube element stiffness is 1/3 on its diagonal, 0 between
//    vertices joined by an element edge and -1/12 across face and body
//    diagonals; scaled by h for a cell of side h.  So a node couples to its
//    12 edge-diagonal neighbours (offsets like (1,1,0), two elements each),
//    its 8 body-diagonal neighbours (one element each) and to itself
//    ((h/3) x the sum of its 8 element kappas), and not to its 6 face
//    neighbours: a 21-point stencil;
//  * reaction and source are lumped with the weight h^3 of an interior node;
//  * the consistent mass is the tensor product of the 1D mass h/6 [1 4 1];
//  * the Gaussian sources of the s x s x s lattice factor into three 1D
//    Gaussians, so F z and F^T lambda are separable sums over three 1D
//    tables (the d_Z x nodes matrix F is never formed).
//
// Multigrid: trilinear prolongation P, restriction P^T (27-point full
// weighting), coarse stiffness rediscretised with each coarse element's kappa
// the mean of its eight children, coarse reaction P^T of the fine lumped
// reaction; damped Jacobi smoothing with omega = 8/9 (for the Q1 stencil the
// Jacobi-scaled symbol lies in [0.75, 1.5] on the high frequencies, so this
// omega damps them by at least 1/3 per sweep); V(1,1) cycles, four sweeps
// from zero on the coarsest grid.  Pre- and post-smoothing are the same
// symmetric sweep, so the V-cycle is a symmetric positive definite
// preconditioner and CG applies.
#include "common.h"
#include "outer.h"
#include "pde3.h"

namespace {

// Threads per sample: the state and adjoint kernels are instantiated for
// 256, 512 and 1024 threads (template BSZ) and the runtime times the three
// once per context and precision (see saa_rt::tune3); the node loops step by
// blockDim.x.  The setup kernel uses HB threads.
constexpr int HB = 512;
constexpr int COARSE_SWEEPS = 4;   // even: the coarsest result lands in T

// Visit nodes p = tid, tid + blockDim.x, ... of an (n+1)^3 grid with (i, j, k).
template <typename F>
__device__ __forceinline__ void for_nodes3(int n, F&& f) {
  const int np = n + 1, np2 = np * np;
  const int total = np2 * np;
  int p = threadIdx.x;
  // Opaque per pass: keeps the per-thread start (and the 64-bit addresses
  // derived from it) inside each pass instead of hoisted out of the solver
  // loops, where one live address set per pass exhausts the registers.
  asm volatile("" : "+v"(p));
  if (p >= total) return;
  int k = p / np2;
  int j = (p - k * np2) / np;
  int i = p - k * np2 - j * np;
  const int bs = (int)blockDim.x;
  const int sk = bs / np2;
  const int sj = (bs - sk * np2) / np;
  const int si = bs - sk * np2 - sj * np;
  for (; p < total; p += bs) {
    f(p, i, j, k);
    i += si;
    if (i >= np) {
      i -= np;
      ++j;
    }
    j += sj;
    if (j >= np) {
      j -= np;
      ++k;
    }
    k += sk;
  }
}

__device__ __forceinline__ bool inner3(int i, int j, int k, int n) {
  return i > 0 && j > 0 && k > 0 && i < n && j < n && k < n;
}

#ifndef SAA_PDE3_BATCH
#define SAA_PDE3_BATCH 1
#endif
// interior nodes per thread per step of a batched pass (2 and 4 measured no
// faster at 48^3: the extra registers cost what the extra loads in flight gain)
constexpr int UB = SAA_PDE3_BATCH;

template <typename T>
struct Two {
  T a, b;
};

// Interior nodes of an (n+1)^3 grid in batches of U visits per thread:
// compute(p, i, j, k) (loads and arithmetic only) runs for the U nodes first
// and store(p, value) after, so the loads of all U nodes are in flight
// together (a store could alias a later node's loads and would otherwise
// order them).  Visits that are not interior nodes compute at the interior
// node (1, 1, 1) (every stencil read in bounds) and store nothing.
template <int U, typename C, typename S>
__device__ __forceinline__ void for_inner3(int n, C&& compute, S&& store) {
  const int np = n + 1, np2 = np * np;
  const int total = np2 * np;
  const int psafe = np2 + np + 1;
  int p = threadIdx.x;
  asm volatile("" : "+v"(p));
  int k = p / np2;
  int j = (p - k * np2) / np;
  int i = p - k * np2 - j * np;
  const int bs = (int)blockDim.x;
  const int sk = bs / np2;
  const int sj = (bs - sk * np2) / np;
  const int si = bs - sk * np2 - sj * np;
  for (; p < total; p += U * bs) {
    int q[U], qi[U], qj[U], qk[U];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      in[u] = p + u * bs < total && inner3(i, j, k, n);
      q[u] = in[u] ? p + u * bs : psafe;
      qi[u] = in[u] ? i : 1;
      qj[u] = in[u] ? j : 1;
      qk[u] = in[u] ? k : 1;
      i += si;
      if (i >= np) {
        i -= np;
        ++j;
      }
      j += sj;
      if (j >= np) {
        j -= np;
        ++k;
      }
      k += sk;
    }
    decltype(compute(0, 1, 1, 1)) r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = compute(q[u], qi[u], qj[u], qk[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (in[u]) store(q[u], r[u]);
  }
}

// Sum over the 20 coupled neighbours q of p of (sum of the kappas of the
// elements containing p and q) x x(q).  The element with lowest corner
// p - a - b np - c np2 (a, b, c in {0, 1}) holds kappa e_abc and contains the
// neighbours of p at offsets (+-1 per coordinate: + for bit 0, - for bit 1).
// The operator is (A x)_p = D_p x_p - (h/12) off_sum.
template <typename TA, typename TE, typename XF>
__device__ __forceinline__ TA off_sum(const TE* E, int p, int np, int np2, XF&& x) {
  const TA e000 = (TA)E[p], e100 = (TA)E[p - 1], e010 = (TA)E[p - np], e110 = (TA)E[p - np - 1];
  const TA e001 = (TA)E[p - np2], e101 = (TA)E[p - np2 - 1], e011 = (TA)E[p - np2 - np];
  const TA e111 = (TA)E[p - np2 - np - 1];
  auto u = [&](int dx, int dy, int dz) { return (TA)x(p + dx + dy * np + dz * np2); };
  TA s = (e000 + e001) * u(1, 1, 0) + (e100 + e101) * u(-1, 1, 0) + (e010 + e011) * u(1, -1, 0) +
         (e110 + e111) * u(-1, -1, 0);
  s += (e000 + e010) * u(1, 0, 1) + (e100 + e110) * u(-1, 0, 1) + (e001 + e011) * u(1, 0, -1) +
       (e101 + e111) * u(-1, 0, -1);
  s += (e000 + e100) * u(0, 1, 1) + (e010 + e110) * u(0, -1, 1) + (e001 + e101) * u(0, 1, -1) +
       (e011 + e111) * u(0, -1, -1);
  s += e000 * u(1, 1, 1) + e100 * u(-1, 1, 1) + e010 * u(1, -1, 1) + e110 * u(-1, -1, 1) + e001 * u(1, 1, -1) +
       e101 * u(-1, 1, -1) + e011 * u(1, -1, -1) + e111 * u(-1, -1, -1);
  return s;
}

// Column march over the interior nodes of an n^3-cell grid.  Work item w
// takes the interior column (i, j) = (1 + c % (n-1), 1 + c / (n-1)),
// c = w mod (n-1)^2, and one half of its k range (items below (n-1)^2: k = 1
// .. n/2, the others k = n/2 + 1 .. n - 1), so consecutive threads walk
// neighbouring columns and their loads coalesce.  At step k the window holds
// x at (i + dx, j + dy, k + dz), dx, dy, dz in {-1, 0, 1}, and the kappas of
// the 8 elements with lowest corners (i - 1 + a, j - 1 + b, k - 1 + c);
// plane k + 2 of x and element plane k + 1 are loaded before the body of step
// k runs (the body's stores would otherwise order the next step's loads
// behind them).  Plane indices are clamped to n, inside the (n+1)^3 arrays.
template <typename TA>
struct Win3 {
  TA x[3][3][3];   // x[dz + 1][dy + 1][dx + 1]
  TA e[2][2][2];   // e[c][b][a]: element with lowest corner (i - 1 + a, j - 1 + b, k - 1 + c)
  __device__ __forceinline__ TA centre() const { return x[1][1][1]; }
};

// off_sum on a window: the element e_abc of off_sum (lowest corner
// p - a - b np - c np2) is e[1 - c][1 - b][1 - a].
template <typename TA>
__device__ __forceinline__ TA off_sum_w(const Win3<TA>& w) {
  const TA e000 = w.e[1][1][1], e100 = w.e[1][1][0], e010 = w.e[1][0][1], e110 = w.e[1][0][0];
  const TA e001 = w.e[0][1][1], e101 = w.e[0][1][0], e011 = w.e[0][0][1], e111 = w.e[0][0][0];
  auto u = [&](int dx, int dy, int dz) { return w.x[dz + 1][dy + 1][dx + 1]; };
  TA s = (e000 + e001) * u(1, 1, 0) + (e100 + e101) * u(-1, 1, 0) + (e010 + e011) * u(1, -1, 0) +
         (e110 + e111) * u(-1, -1, 0);
  s += (e000 + e010) * u(1, 0, 1) + (e100 + e110) * u(-1, 0, 1) + (e001 + e011) * u(1, 0, -1) +
       (e101 + e111) * u(-1, 0, -1);
  s += (e000 + e100) * u(0, 1, 1) + (e010 + e110) * u(0, -1, 1) + (e001 + e101) * u(0, 1, -1) +
       (e011 + e111) * u(0, -1, -1);
  s += e000 * u(1, 1, 1) + e100 * u(-1, 1, 1) + e010 * u(1, -1, 1) + e110 * u(-1, -1, 1) + e001 * u(1, 1, -1) +
       e101 * u(-1, 1, -1) + e011 * u(1, -1, -1) + e111 * u(-1, -1, -1);
  return s;
}

template <typename TA>
__device__ __forceinline__ TA kappa_sum_w(const Win3<TA>& w) {
  return ((w.e[0][0][0] + w.e[0][0][1]) + (w.e[0][1][0] + w.e[0][1][1])) +
         ((w.e[1][0][0] + w.e[1][0][1]) + (w.e[1][1][0] + w.e[1][1][1]));
}

template <typename TA, typename XL, typename EL, typename Body>
__device__ __forceinline__ void march3(int n, XL&& xload, EL&& eload, Body&& body) {
  const int np = n + 1, np2 = np * np, nc = n - 1, ncol = nc * nc, kh = n / 2;
  int w = threadIdx.x;
  asm volatile("" : "+v"(w));
  for (; w < 2 * ncol; w += (int)blockDim.x) {
    const int half = w >= ncol ? 1 : 0;
    const int c = w - half * ncol;
    const int j = 1 + c / nc, i = 1 + c - (j - 1) * nc;
    const int k0 = half ? kh + 1 : 1, k1 = half ? n - 1 : kh;
    if (k0 > k1) continue;
    const int base = i + j * np;   // node (i, j, 0)
    auto xplane = [&](TA (&d)[3][3], int kk) {
      const int q = base + kk * np2;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) d[dy + 1][dx + 1] = xload(q + dy * np + dx);
    };
    auto eplane = [&](TA (&d)[2][2], int kk) {
      const int q = base + kk * np2 - np - 1;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) d[b][a] = eload(q + b * np + a);
    };
    Win3<TA> W;
    xplane(W.x[0], k0 - 1);
    xplane(W.x[1], k0);
    xplane(W.x[2], k0 + 1);
    eplane(W.e[0], k0 - 1);
    eplane(W.e[1], k0);
    for (int k = k0; k <= k1; ++k) {
      TA xa[3][3], ea[2][2];
      xplane(xa, k + 2 <= n ? k + 2 : n);
      eplane(ea, k + 1 <= n - 1 ? k + 1 : n - 1);
      body(base + k * np2, W);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          W.x[0][dy][dx] = W.x[1][dy][dx];
          W.x[1][dy][dx] = W.x[2][dy][dx];
          W.x[2][dy][dx] = xa[dy][dx];
        }
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          W.e[0][b][a] = W.e[1][b][a];
          W.e[1][b][a] = ea[b][a];
        }
    }
  }
}

template <typename TE>
__device__ __forceinline__ double kappa_sum8(const TE* E, int p, int np, int np2) {
  return (double)E[p] + (double)E[p - 1] + (double)E[p - np] + (double)E[p - np - 1] + (double)E[p - np2] +
         (double)E[p - np2 - 1] + (double)E[p - np2 - np] + (double)E[p - np2 - np - 1];
}

// (M x)_p / h^3 for the consistent Q1 mass: weights (1/6)^3 prod_d (4 or 1).
template <typename TX>
__device__ __forceinline__ double mass3(const TX* x, int p, int np, int np2) {
  double acc = 0.0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    double pl = 0.0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int q = p + dy * np + dz * np2;
      const double row = (double)x[q - 1] + 4.0 * (double)x[q] + (double)x[q + 1];
      pl += (dy == 0 ? 4.0 : 1.0) * row;
    }
    acc += (dz == 0 ? 4.0 : 1.0) * pl;
  }
  return acc * (1.0 / 216.0);
}

template <typename TS>
struct Lvl3 {
  int n, np, np2;
  TS hq;          // h_l / 12
  const TS* E;
  const TS* D;
  TS* X;
  TS* B;
  TS* T;
};

template <typename TS>
__device__ __forceinline__ Lvl3<TS> lvl3(const Pde3Geo& g, const Mg3Bufs<TS>& m, int l) {
  Lvl3<TS> L;
  L.n = g.n[l];
  L.np = L.n + 1;
  L.np2 = L.np * L.np;
  L.hq = (TS)(g.h * (double)(1 << l) / 12.0);
  L.E = m.E + g.off[l];
  L.D = m.D + g.off[l];
  L.X = m.X + g.off[l];
  L.B = m.B + g.off[l];
  L.T = m.T + g.off[l];
  return L;
}

// (P^T t) at the coarse node whose fine image is c: 27-point full weighting
// with weight 2^-(number of non-zero offsets).
template <typename TS>
__device__ __forceinline__ TS full_weight(const TS* t, int c, int np, int np2) {
  TS acc = (TS)0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    TS pl = (TS)0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int q = c + dy * np + dz * np2;
      const TS row = (TS)0.5 * (t[q - 1] + t[q + 1]) + t[q];
      pl += (dy == 0 ? (TS)1 : (TS)0.5) * row;
    }
    acc += (dz == 0 ? (TS)1 : (TS)0.5) * pl;
  }
  return acc;
}

// Restriction of the fine vector t to the coarse level C: C.B = P^T t at the
// interior coarse nodes, and the first smoothing sweep from zero,
// C.X = omega C.B / C.D.
template <typename TS>
__device__ void restrict3(const Lvl3<TS>& F, const TS* t, const Lvl3<TS>& C, TS omega) {
  for_inner3<UB>(
      C.n,
      [&](int P, int I, int J, int K) {
        return Two<TS>{full_weight(t, 2 * I + 2 * J * F.np + 2 * K * F.np2, F.np, F.np2), C.D[P]};
      },
      [&](int P, const Two<TS>& v) {
        C.B[P] = v.a;
        C.X[P] = omega * v.a / v.b;
      });
}

// x += P xc: trilinear interpolation of the coarse vector (zero on the coarse
// boundary).  With i0 = i / 2 and i1 = i0 + (i mod 2) per coordinate, the
// interpolant is the mean of the 8 values at (i0|i1, j0|j1, k0|k1): an even
// index repeats its coarse node (weight 1), an odd one averages two.  Fine
// columns (i, j) march in k: the bilinear mean over (i0|i1, j0|j1) of coarse
// plane K serves the fine planes 2K - 1, 2K and 2K + 1, so a fine node costs
// about two coarse loads instead of eight.
template <typename TS>
__device__ void prolong_add3(const Lvl3<TS>& F, TS* x, const Lvl3<TS>& C, const TS* xc) {
  const int n = F.n, nc = n - 1, ncol = nc * nc, kh = n / 2;
  int w = threadIdx.x;
  asm volatile("" : "+v"(w));
  for (; w < 2 * ncol; w += (int)blockDim.x) {
    const int half = w >= ncol ? 1 : 0;
    const int c = w - half * ncol;
    const int j = 1 + c / nc, i = 1 + c - (j - 1) * nc;
    const int k0 = half ? kh + 1 : 1, k1 = half ? n - 1 : kh;
    if (k0 > k1) continue;
    const int a0 = (i >> 1) + (j >> 1) * C.np;   // coarse (i0, j0, 0)
    const int da = i & 1, db = (j & 1) * C.np;
    auto bil = [&](int K) {
      const int q = a0 + K * C.np2;
      return (TS)0.25 * ((xc[q] + xc[q + da]) + (xc[q + db] + xc[q + da + db]));
    };
    int K = k0 >> 1;
    TS lo = bil(K);                                   // coarse plane K = k >> 1
    TS hi = (k0 & 1) ? bil(K + 1) : lo;               // plane K + (k & 1)
    for (int k = k0; k <= k1; ++k) {
      const int p = i + j * F.np + k * F.np2;
      x[p] += (TS)0.5 * (lo + hi);
      // next fine plane k + 1: K' = (k + 1) >> 1
      if (k & 1) {   // k odd -> k + 1 even: both ends are plane K + 1
        lo = hi;
      } else if (k < k1) {   // k even -> k + 1 odd: planes K and K + 1
        hi = bil((k >> 1) + 1);
      }
    }
  }
}

// Grids of at least this many cells per side run their stencil passes as
// column marches; smaller ones have too few columns to occupy the threads.
constexpr int MARCH_MIN_N = 16;

// t = b - A x on the interior of level L.
template <typename TS>
__device__ void residual3(const Lvl3<TS>& L, const TS* b, const TS* x, TS* t) {
  if (L.n >= MARCH_MIN_N) {
    march3<TS>(
        L.n, [&](int q) { return x[q]; }, [&](int q) { return L.E[q]; },
        [&](int p, const Win3<TS>& W) { t[p] = b[p] - (L.D[p] * W.centre() - L.hq * off_sum_w(W)); });
    return;
  }
  for_inner3<UB>(
      L.n,
      [&](int p, int, int, int) {
        return b[p] - (L.D[p] * x[p] - L.hq * off_sum<TS>(L.E, p, L.np, L.np2, [&](int q) { return x[q]; }));
      },
      [&](int p, TS v) { t[p] = v; });
}

// One damped Jacobi sweep dst = src + omega (b - A src) / D.
template <typename TS>
__device__ void jacobi3(const Lvl3<TS>& L, const TS* b, const TS* src, TS* dst, TS omega) {
  if (L.n >= MARCH_MIN_N) {
    march3<TS>(
        L.n, [&](int q) { return src[q]; }, [&](int q) { return L.E[q]; },
        [&](int p, const Win3<TS>& W) {
          const TS xs = W.centre(), d = L.D[p];
          dst[p] = xs + omega * (b[p] - (d * xs - L.hq * off_sum_w(W))) / d;
        });
    return;
  }
  for_inner3<UB>(
      L.n,
      [&](int p, int, int, int) {
        const TS xs = src[p], d = L.D[p];
        const TS ax = d * xs - L.hq * off_sum<TS>(L.E, p, L.np, L.np2, [&](int q) { return src[q]; });
        return xs + omega * (b[p] - ax) / d;
      },
      [&](int p, TS v) { dst[p] = v; });
}

// V(1,1) cycle on the levels l0.. given B[l0] and the first sweep X[l0] (set
// by the restriction from level l0 - 1); the result is left in T[l0].
template <typename TS>
__device__ void vcycle3_from(const Pde3Geo& g, const Mg3Bufs<TS>& m, int l0, TS omega) {
  const int lc = g.L - 1;
  for (int l = l0; l < lc; ++l) {
    const Lvl3<TS> L = lvl3(g, m, l);
    residual3(L, (const TS*)L.B, (const TS*)L.X, L.T);
    __syncthreads();
    restrict3(L, (const TS*)L.T, lvl3(g, m, l + 1), omega);
    __syncthreads();
  }
  const Lvl3<TS> C = lvl3(g, m, lc);
  // one copy of the sweep with alternating buffers (unrolled copies raise
  // the register pressure of the whole kernel)
#pragma unroll 1
  for (int sw = 1; sw < COARSE_SWEEPS; ++sw) {
    const TS* src = (sw & 1) ? C.X : C.T;
    TS* dst = (sw & 1) ? C.T : C.X;
    jacobi3(C, (const TS*)C.B, src, dst, omega);
    __syncthreads();
  }
  for (int l = lc - 1; l >= l0; --l) {
    const Lvl3<TS> L = lvl3(g, m, l);
    const Lvl3<TS> Cl = lvl3(g, m, l + 1);
    prolong_add3(L, L.X, Cl, (const TS*)Cl.T);
    __syncthreads();
    jacobi3(L, (const TS*)L.B, (const TS*)L.X, L.T, omega);
    __syncthreads();
  }
}

// Operator diagonals for the linearisation at u: level 0 gets the lumped
// reaction 3 r h^3 u^2, coarser levels its restriction P^T (kept in T while
// the hierarchy is walked).
template <typename TW, typename TS>
__device__ void build_diagonals3(const Pde3Geo& g, const Mg3Bufs<TS>& m, const TW* u) {
  const double c3 = 3.0 * g.r * g.h * g.h * g.h;
  {
    const Lvl3<TS> L0 = lvl3(g, m, 0);
    TS* D = m.D + g.off[0];
    const TS* KD = m.KD + g.off[0];
    for_nodes3(L0.n, [&](int p, int i, int j, int k) {
      if (!inner3(i, j, k, L0.n)) return;
      const double uu = (double)u[p];
      const TS rc = (TS)(c3 * uu * uu);
      L0.T[p] = rc;
      D[p] = KD[p] + rc;
    });
  }
  __syncthreads();
  for (int l = 1; l < g.L; ++l) {
    const Lvl3<TS> F = lvl3(g, m, l - 1), C = lvl3(g, m, l);
    TS* D = m.D + g.off[l];
    const TS* KD = m.KD + g.off[l];
    for_nodes3(C.n, [&](int P, int I, int J, int K) {
      if (!inner3(I, J, K, C.n)) return;
      const TS rc = full_weight((const TS*)F.T, 2 * I + 2 * J * F.np + 2 * K * F.np2, F.np, F.np2);
      C.T[P] = rc;
      D[P] = KD[P] + rc;
    });
    __syncthreads();
  }
}

// Preconditioned CG on A x = b with b in m.cr (overwritten by the residual),
// x in m.cx; one V(1,1) cycle per iteration.  Fine-level passes: A p (with
// p = z + beta p_old formed from neighbour values), the x / r update with the
// first smoothing sweep of the next cycle, the residual, the restriction, the
// prolongation and the post-smoothing sweep with r . z.  Returns the
// iteration count; clears *ok when not converged.
template <typename TS>
__device__ int pcg3(const Pde3Geo& g, const Mg3Bufs<TS>& m, double rtol, int max_it, double* red, bool* ok) {
  const TS omega = (TS)(8.0 / 9.0);
  const Lvl3<TS> L0 = lvl3(g, m, 0);
  const Lvl3<TS> L1 = lvl3(g, m, 1);
  const int n = L0.n;
  double rr0 = 0.0;
  for_nodes3(n, [&](int p, int i, int j, int k) {
    if (!inner3(i, j, k, n)) return;
    const TS r = m.cr[p];
    rr0 += (double)r * (double)r;
    m.cx[p] = (TS)0;
    L0.X[p] = omega * r / L0.D[p];
  });
  rr0 = block_sum1(rr0, red);
  if (!(rr0 > 0.0)) {
    *ok = (rr0 == 0.0);
    return 0;
  }
  const double tol2 = rtol * rtol * rr0;
  TS* z = L0.T;
  TS* pc = m.cp;
  TS* pn = L0.B;   // the level-0 right-hand side slot is free: directions alternate with cp
  TS beta = (TS)0;
  double rz = 0.0;
  for (int it = 0; it <= max_it; ++it) {
    if (it > 0) {
      double pq = 0.0;
      const TS* po = pc;
      march3<TS>(
          n, [&](int q) { return z[q] + beta * po[q]; },   // zero on the boundary
          [&](int q) { return L0.E[q]; },
          [&](int p, const Win3<TS>& W) {
            const TS pp = W.centre();
            const TS q = L0.D[p] * pp - L0.hq * off_sum_w(W);
            pn[p] = pp;
            m.cq[p] = q;
            pq += (double)pp * (double)q;
          });
      TS* t = pc;
      pc = pn;
      pn = t;
      pq = block_sum1(pq, red);
      if (!(pq > 0.0)) {
        *ok = false;
        return it;
      }
      const TS a = (TS)(rz / pq);
      double rr = 0.0;
      struct Upd {
        TS x, r, d;
      };
      for_inner3<UB>(
          n, [&](int p, int, int, int) { return Upd{m.cx[p] + a * pc[p], m.cr[p] - a * m.cq[p], L0.D[p]}; },
          [&](int p, const Upd& v) {
            m.cx[p] = v.x;
            m.cr[p] = v.r;
            rr += (double)v.r * (double)v.r;
            L0.X[p] = omega * v.r / v.d;
          });
      rr = block_sum1(rr, red);
      if (rr <= tol2) return it;
    }
    march3<TS>(
        n, [&](int q) { return L0.X[q]; }, [&](int q) { return L0.E[q]; },
        [&](int p, const Win3<TS>& W) { L0.T[p] = m.cr[p] - (L0.D[p] * W.centre() - L0.hq * off_sum_w(W)); });
    __syncthreads();
    restrict3(L0, (const TS*)L0.T, L1, omega);
    __syncthreads();
    vcycle3_from(g, m, 1, omega);
    prolong_add3(L0, L0.X, L1, (const TS*)L1.T);
    __syncthreads();
    double rzn = 0.0;
    march3<TS>(
        n, [&](int q) { return L0.X[q]; }, [&](int q) { return L0.E[q]; },
        [&](int p, const Win3<TS>& W) {
          const TS xs = W.centre(), d = L0.D[p], r = m.cr[p];
          const TS zz = xs + omega * (r - (d * xs - L0.hq * off_sum_w(W))) / d;
          z[p] = zz;
          rzn += (double)r * (double)zz;
        });
    rzn = block_sum1(rzn, red);
    beta = (TS)(it > 0 ? rzn / rz : 0.0);
    rz = rzn;
  }
  *ok = false;
  return max_it;
}

template <typename TS>
__device__ __forceinline__ Mg3Bufs<TS> sample_bufs3(const Mg3Bufs<TS>& all, const Pde3Geo& g, int64_t s) {
  Mg3Bufs<TS> m;
  const int64_t ls = s * g.lstride, ns = s * g.nodes;
  m.E = all.E + ls;
  m.KD = all.KD + ls;
  m.D = all.D + ls;
  m.X = all.X + ls;
  m.B = all.B + ls;
  m.T = all.T + ls;
  m.cx = all.cx + ns;
  m.cr = all.cr + ns;
  m.cp = all.cp + ns;
  m.cq = all.cq + ns;
  return m;
}

// (K u)_p with the fine stiffness of the FP64 element kappas K, in precision TW.
template <typename TW>
__device__ __forceinline__ TW stiff3(const double* K, const TW* u, int p, int np, int np2, double h) {
  const TW kd = (TW)(h / 3.0 * kappa_sum8(K, p, np, np2));
  return kd * u[p] - (TW)(h / 12.0) * off_sum<TW>(K, p, np, np2, [&](int q) { return u[q]; });
}

// Defect correction for A(u) x = b (A in precision TW from the FP64 element
// kappas plus 3 r h^3 u^2; inner PCG in TS).  The diagonals must be built
// for u.  Returns the inner CG iterations; clears *ok on failure.
template <typename TW, typename TS>
__device__ int dc_solve3(const Pde3Geo& g, const Mg3Bufs<TS>& m, const SolveParams& sp, const double* K,
                         const TW* u, const TW* b, TW* x, double* red, bool* ok) {
  const int n = g.n[0], np = n + 1, np2 = np * np;
  const double c3 = 3.0 * g.r * g.h * g.h * g.h;
  int lin = 0;
  for_nodes3(n, [&](int p, int i, int j, int k) {
    x[p] = (TW)0;
    if (inner3(i, j, k, n)) m.cr[p] = (TS)b[p];
  });
  __syncthreads();
  OuterCtl ctl;
  ctl.eta = sp.lin_rtol;
  int pass;
  for (pass = 0; pass < sp.max_dc; ++pass) {
    bool cg_ok = true;
    lin += pcg3(g, m, ctl.eta, sp.max_lin, red, &cg_ok);
    double v[2] = {0.0, 0.0};
    for_nodes3(n, [&](int p, int i, int j, int k) {
      if (!inner3(i, j, k, n)) return;
      const TW d = (TW)m.cx[p];
      const TW xn = x[p] + d;
      x[p] = xn;
      v[0] += (double)d * (double)d;
      v[1] += (double)xn * (double)xn;
    });
    block_sum<2>(v, red);
    if (!(v[0] == v[0]) || !(v[1] == v[1])) {
      *ok = false;
      break;
    }
    if (outer_converged(ctl, v[0], v[1], sp.adj_tol, sp.lin_rtol)) break;
    march3<TW>(
        n, [&](int q) { return x[q]; }, [&](int q) { return (TW)K[q]; },
        [&](int p, const Win3<TW>& W) {
          const TW uu = u[p], xc = W.centre();
          const TW kx = (TW)(g.h / 3.0) * kappa_sum_w(W) * xc - (TW)(g.h / 12.0) * off_sum_w(W);
          m.cr[p] = (TS)(b[p] - (kx + (TW)c3 * uu * uu * xc));
        });
    __syncthreads();
  }
  if (pass == sp.max_dc) *ok = false;
  return lin;
}

}  // namespace

// ---------------------------------------------------------------------------
// Setup kernels (once per sample set)
// ---------------------------------------------------------------------------

// Nodal exp(m) of each sample on the plane z = kz (one block per sample and
// plane), evaluated separably: T1[j][k] = sum_l a_jkl xi_jkl sin(l pi z),
// T2[j][y] = sum_k T1[j][k] sin(k pi y), m = sum_j T2[j][y] sin(j pi x).
// S[j][i] = sin((j+1) pi i / n).
__global__ void __launch_bounds__(256) saa_k_field3(const double* xi, const double* S, const double* amp,
                                                    double* em, int K1, int n, int64_t N) {
  extern __shared__ double sh[];
  const int np = n + 1;
  const int64_t s = blockIdx.x / np;
  const int kz = (int)(blockIdx.x - s * np);
  if (s >= N) return;
  double* T1 = sh;
  double* T2 = sh + K1 * K1;
  const double* x = xi + s * K1 * K1 * K1;
  for (int t = threadIdx.x; t < K1 * K1; t += blockDim.x) {
    double acc = 0.0;
    for (int l = 0; l < K1; ++l) acc += amp[t * K1 + l] * x[t * K1 + l] * S[l * np + kz];
    T1[t] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < K1 * np; t += blockDim.x) {
    const int j = t / np, y = t - j * np;
    double acc = 0.0;
    for (int k = 0; k < K1; ++k) acc += T1[j * K1 + k] * S[k * np + y];
    T2[t] = acc;
  }
  __syncthreads();
  double* out = em + s * (int64_t)np * np * np + (int64_t)kz * np * np;
  for (int p = threadIdx.x; p < np * np; p += blockDim.x) {
    const int y = p / np, xx = p - y * np;
    double acc = 0.0;
    for (int j = 0; j < K1; ++j) acc += T2[j * np + y] * S[j * np + xx];
    out[p] = exp(acc);
  }
}

// Element kappas on every level (fine: vertex mean of exp(m), also kept in
// FP64 for the residuals; coarse: mean of the eight children) and the
// stiffness diagonals.  One block per sample.
template <typename TS>
__global__ void __launch_bounds__(HB) saa_k_hierarchy3(Pde3Geo g, const double* em_all, double* k64_all,
                                                       Mg3Bufs<TS> all, int64_t N) {
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  const double* e = em_all + s * g.nodes;
  double* k64 = k64_all + s * g.nodes;
  Mg3Bufs<TS> m = sample_bufs3(all, g, s);
  {
    const int n = g.n[0], np = n + 1, np2 = np * np;
    TS* E = m.E + g.off[0];
    for_nodes3(n, [&](int p, int i, int j, int k) {
      double v = 0.0;
      if (i < n && j < n && k < n)
        v = 0.125 * (e[p] + e[p + 1] + e[p + np] + e[p + np + 1] + e[p + np2] + e[p + np2 + 1] + e[p + np2 + np] +
                     e[p + np2 + np + 1]);
      k64[p] = v;
      E[p] = (TS)v;
    });
  }
  __syncthreads();
  for (int l = 1; l < g.L; ++l) {
    const int nc = g.n[l], npc = nc + 1, nf = g.n[l - 1], npf = nf + 1;
    const TS* Ef = m.E + g.off[l - 1];
    TS* Ec = m.E + g.off[l];
    for_nodes3(nc, [&](int P, int I, int J, int K) {
      double v = 0.0;
      if (I < nc && J < nc && K < nc) {
        const int c = 2 * I + 2 * J * npf + 2 * K * npf * npf;
        v = 0.125 * kappa_sum8(Ef, c + 1 + npf + npf * npf, npf, npf * npf);
      }
      Ec[P] = (TS)v;
    });
    (void)npc;
    __syncthreads();
  }
  for (int l = 0; l < g.L; ++l) {
    const int n = g.n[l], np = n + 1, np2 = np * np;
    const double hl = g.h * (double)(1 << l);
    const TS* E = m.E + g.off[l];
    TS* KD = m.KD + g.off[l];
    TS* D = m.D + g.off[l];
    for_nodes3(n, [&](int p, int i, int j, int k) {
      TS d = (TS)0;
      if (inner3(i, j, k, n)) d = (TS)(hl / 3.0 * (l == 0 ? kappa_sum8(k64, p, np, np2) : kappa_sum8(E, p, np, np2)));
      KD[p] = d;
      D[p] = d;
    });
  }
}

// ---------------------------------------------------------------------------
// State solve: Newton (precision TW) with inner MG-PCG (precision TS), then
// q = (u - ut)^T M (u - ut).  One block per sample; all samples share z.
// ---------------------------------------------------------------------------
// One sample's 3D state solve (shared by the single-problem kernel and the
// mixed-dimension launch); red, zs and Gs are LDS scratch of the caller.
template <typename TW, typename TS, int BSZ>
__device__ __forceinline__ void state3_sample(const Pde3Geo& g, const double* Z, int64_t z_stride,
                                              const double* k64_all, TW* u_all, TW* f_all, const Mg3Bufs<TS>& all,
                                              const SolveParams& sp, double* q_out, int* newton_out, int* lin_out,
                                              int* flag_out, int64_t s, double* red, double* zs, double* Gs) {
  const int n = g.n[0], np = n + 1, np2 = np * np, ns = g.s;
  const double* K = k64_all + s * g.nodes;
  TW* u = u_all + s * g.nodes;
  TW* f = f_all + s * g.nodes;
  Mg3Bufs<TS> m = sample_bufs3(all, g, s);
  if (threadIdx.x < g.dz) zs[threadIdx.x] = Z[s * z_stride + threadIdx.x];   // z_stride 0: one shared control
  for (int t = threadIdx.x; t < ns * np; t += BSZ) Gs[t] = g.G[t];
  __syncthreads();
  // f = F z: lumped separable sources; u = 0
  for_nodes3(n, [&](int p, int i, int j, int k) {
    double acc = 0.0;
    if (inner3(i, j, k, n)) {
      for (int c = 0; c < ns; ++c)
        for (int b = 0; b < ns; ++b) {
          double t = 0.0;
          for (int a = 0; a < ns; ++a) t += zs[a + ns * (b + ns * c)] * Gs[a * np + i];
          acc += Gs[c * np + k] * Gs[b * np + j] * t;
        }
      acc *= g.src_c;
    }
    f[p] = (TW)acc;
    u[p] = (TW)0;
  });
  __syncthreads();
  const double c1 = g.r * g.h * g.h * g.h;
  int flags = 0, lin = 0, it = 0;
  bool conv = false;
  OuterCtl ctl;
  ctl.eta = sp.lin_rtol;
  for (it = 0; it < sp.max_newton; ++it) {
    march3<TW>(
        n, [&](int q) { return u[q]; }, [&](int q) { return (TW)K[q]; },
        [&](int p, const Win3<TW>& W) {
          const TW uu = W.centre();
          const TW ku = (TW)(g.h / 3.0) * kappa_sum_w(W) * uu - (TW)(g.h / 12.0) * off_sum_w(W);
          m.cr[p] = (TS)(f[p] - (ku + (TW)c1 * uu * uu * uu));
        });
    __syncthreads();
    build_diagonals3<TW, TS>(g, m, u);
    bool ok = true;
    lin += pcg3(g, m, ctl.eta, sp.max_lin, red, &ok);
    if (!ok) flags |= SAA_FLAG_CG;
    double v[2] = {0.0, 0.0};
    for_nodes3(n, [&](int p, int i, int j, int k) {
      if (!inner3(i, j, k, n)) return;
      const TW d = (TW)m.cx[p];
      const TW un = u[p] + d;
      u[p] = un;
      v[0] += (double)d * (double)d;
      v[1] += (double)un * (double)un;
    });
    block_sum<2>(v, red);
    if (!(v[0] == v[0]) || !(v[1] == v[1])) {
      flags |= SAA_FLAG_NAN;
      break;
    }
    if (outer_converged(ctl, v[0], v[1], sp.newton_tol, sp.lin_rtol)) {
      conv = true;
      ++it;
      break;
    }
  }
  if (!conv) flags |= SAA_FLAG_NEWTON;
  const double h3 = g.h * g.h * g.h;
  double qa = 0.0;
  for_nodes3(n, [&](int p, int i, int j, int k) {
    if (!inner3(i, j, k, n)) return;
    qa += (double)u[p] * (h3 * mass3(u, p, np, np2) - 2.0 * g.mt[p]);
  });
  qa = block_sum1(qa, red);
  if (threadIdx.x == 0) {
    q_out[s] = qa + g.ctt;
    newton_out[s] = it;
    lin_out[s] = lin;
    flag_out[s] = flags;
  }
}

template <typename TW, typename TS, int BSZ>
__global__ void __launch_bounds__(BSZ) saa_k_state3(Pde3Geo g, const double* Z, int64_t z_stride,
                                                   const double* k64_all, TW* u_all, TW* f_all, Mg3Bufs<TS> all,
                                                   SolveParams sp, double* q_out, int* newton_out, int* lin_out,
                                                   int* flag_out, int64_t N) {
  __shared__ double red[SAA_MAX_DZ * (BSZ / SAA_WAVE)];
  __shared__ double zs[SAA_MAX_DZ];
  __shared__ double Gs[4 * 97];
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  state3_sample<TW, TS, BSZ>(g, Z, z_stride, k64_all, u_all, f_all, all, sp, q_out, newton_out, lin_out, flag_out, s,
                             red, zs, Gs);
}

// ---------------------------------------------------------------------------
// Adjoint: A(u) lambda = 2 (M (u - ut))_I, g = F^T lambda (Sec. 2.3) for the
// samples whose risk weight can be non-zero (the activity rules of the 2D
// kernel: act 0 CVaR tail q > t, 1 all, 2 0 < q - t < act_w, 3 buffered
// exceedance); the others get a zero g row.
// ---------------------------------------------------------------------------
// One sample's 3D adjoint (shared by the single-problem kernel and the
// mixed-dimension launch); red and Gs are LDS scratch of the caller.
template <typename TW, typename TS, int BSZ>
__device__ __forceinline__ void adjoint3_sample(const Pde3Geo& g, const double* k64_all, const TW* u_all, TW* b_all,
                                                TW* lam_all, const Mg3Bufs<TS>& all, const SolveParams& sp,
                                                const double* q, const double* tstar, int act, double act_w,
                                                double* g_out, int* lin_out, int* flag_out, int* did_out, int64_t s,
                                                double* red, double* Gs) {
  const int n = g.n[0], np = n + 1, np2 = np * np, ns = g.s;
  const double xq = q[s] - tstar[0];
  const bool active = act == 1 || (act == 3 ? (tstar[0] > 0.0 && tstar[0] < INFINITY &&
                                               tstar[0] * (q[s] - act_w) + 1.0 > 0.0)
                                            : (xq > 0.0 && (act == 0 || xq < act_w)));
  if (!active) {
    if (threadIdx.x < g.dz) g_out[s * g.dz + threadIdx.x] = 0.0;
    if (threadIdx.x == 0) {
      lin_out[s] = 0;
      did_out[s] = 0;
    }
    return;
  }
  const double* K = k64_all + s * g.nodes;
  const TW* u = u_all + s * g.nodes;
  TW* b = b_all + s * g.nodes;
  TW* lam = lam_all + s * g.nodes;
  Mg3Bufs<TS> m = sample_bufs3(all, g, s);
  for (int t = threadIdx.x; t < ns * np; t += BSZ) Gs[t] = g.G[t];
  const double h3 = g.h * g.h * g.h;
  for_nodes3(n, [&](int p, int i, int j, int k) {
    double v = 0.0;
    if (inner3(i, j, k, n)) v = 2.0 * (h3 * mass3(u, p, np, np2) - g.mt[p]);
    b[p] = (TW)v;
  });
  __syncthreads();
  build_diagonals3<TW, TS>(g, m, u);
  bool ok = true;
  const int lin = dc_solve3<TW, TS>(g, m, sp, K, u, b, lam, red, &ok);
  // g = F^T lambda = src_c sum_p G[a][i] G[b][j] G[c][k] lambda_p, eight controls per pass
  for (int k0 = 0; k0 < g.dz; k0 += 8) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = 0.0;
    for_nodes3(n, [&](int p, int i, int j, int k) {
      if (!inner3(i, j, k, n)) return;
      const double l = (double)lam[p];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int kk = k0 + t;
        if (kk < g.dz) {
          const int a = kk % ns, bb = (kk / ns) % ns, c = kk / (ns * ns);
          v[t] += Gs[a * np + i] * Gs[bb * np + j] * Gs[c * np + k] * l;
        }
      }
    });
    block_sum<8>(v, red);
    if (threadIdx.x == 0)
      for (int t = 0; t < 8 && k0 + t < g.dz; ++t) g_out[s * g.dz + k0 + t] = g.src_c * v[t];
  }
  if (threadIdx.x == 0) {
    lin_out[s] = lin;
    did_out[s] = 1;
    if (!ok) flag_out[s] |= SAA_FLAG_DC;
  }
}

template <typename TW, typename TS, int BSZ>
__global__ void __launch_bounds__(BSZ) saa_k_adjoint3(Pde3Geo g, const double* k64_all, const TW* u_all, TW* b_all,
                                                     TW* lam_all, Mg3Bufs<TS> all, SolveParams sp, const double* q,
                                                     const double* tstar, int act, double act_w, double* g_out,
                                                     int* lin_out, int* flag_out, int* did_out, int64_t N) {
  __shared__ double red[SAA_MAX_DZ * (BSZ / SAA_WAVE)];
  __shared__ double Gs[4 * 97];
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  adjoint3_sample<TW, TS, BSZ>(g, k64_all, u_all, b_all, lam_all, all, sp, q, tstar, act, act_w, g_out, lin_out,
                               flag_out, did_out, s, red, Gs);
}

// ---------------------------------------------------------------------------
// Control Jacobians (training data, Sec. 3.4 eq. (projected_sensitivity)):
// for samples s0 .. s0 + gridDim.x and controls k0 .. k0 + nk, solve
// A(u) x = F e_k (the lumped k-th source, separable) by defect-corrected
// MG-PCG reusing the sample's hierarchy, and write x at the interior nodes
// (interior order, x fastest) to out[((s - s0) nk + k - k0) ld + .] in FP64.
// ---------------------------------------------------------------------------
template <typename TW, typename TS, int BSZ>
__global__ void __launch_bounds__(BSZ) saa_k_linearized3(Pde3Geo g, const double* k64_all, const TW* u_all,
                                                        TW* b_all, TW* x_all, Mg3Bufs<TS> all, SolveParams sp,
                                                        int64_t s0, int k0, int nk, double* out, int64_t ld,
                                                        int* lin_out, int* flag_out, int64_t N) {
  __shared__ double red[SAA_MAX_DZ * (BSZ / SAA_WAVE)];
  __shared__ double Gs[4 * 97];
  const int64_t s = s0 + blockIdx.x;
  if (s >= N) return;
  const int n = g.n[0], np = n + 1, ns = g.s, m1 = n - 1;
  const double* K = k64_all + s * g.nodes;
  const TW* u = u_all + s * g.nodes;
  TW* b = b_all + s * g.nodes;
  TW* x = x_all + s * g.nodes;
  Mg3Bufs<TS> m = sample_bufs3(all, g, s);
  for (int t = threadIdx.x; t < ns * np; t += BSZ) Gs[t] = g.G[t];
  __syncthreads();
  build_diagonals3<TW, TS>(g, m, u);
  int lin = 0;
  bool ok = true;
  for (int kk = k0; kk < k0 + nk; ++kk) {
    const int a = kk % ns, bb = (kk / ns) % ns, c = kk / (ns * ns);
    for_nodes3(n, [&](int p, int i, int j, int k) {
      const double v = inner3(i, j, k, n) ? g.src_c * Gs[a * np + i] * Gs[bb * np + j] * Gs[c * np + k] : 0.0;
      b[p] = (TW)v;
    });
    __syncthreads();
    lin += dc_solve3<TW, TS>(g, m, sp, K, u, b, x, red, &ok);
    double* o = out + ((s - s0) * nk + (kk - k0)) * ld;
    for_nodes3(n, [&](int p, int i, int j, int k) {
      if (inner3(i, j, k, n)) o[(i - 1) + (int64_t)m1 * ((j - 1) + (int64_t)m1 * (k - 1))] = (double)x[p];
    });
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lin_out[s] = lin;
    if (!ok) flag_out[s] |= SAA_FLAG_DC;
  }
}

// Interior values of node vectors: out[s][(i-1) + m (j-1) + m^2 (k-1)] =
// u[s][node (i, j, k)], m = n - 1, in FP64.
template <typename TW>
__global__ void saa_k_interior3(const TW* u_all, double* out, int n, int64_t nodes, int64_t N) {
  const int m = n - 1;
  const int64_t du = (int64_t)m * m * m;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * du) return;
  const int64_t s = t / du;
  const int64_t p = t - s * du;
  const int i = (int)(p % m) + 1, j = (int)((p / m) % m) + 1, k = (int)(p / ((int64_t)m * m)) + 1;
  out[t] = (double)u_all[s * nodes + i + (int64_t)(n + 1) * (j + (int64_t)(n + 1) * k)];
}

// out[s][p] = (M_II (v_s - vbar))_p on the (n-1)^3 interior grid (interior
// order), consistent Q1 mass: the tensor product of the 1D (h/6) [1 4 1]
// (boundary values zero).  vbar may be null.
__global__ void saa_k_mass_rows3(const double* V, int64_t ldv, const double* vbar, double* out, int64_t ldo, int n,
                                 int64_t rows) {
  const int m = n - 1;
  const int64_t du = (int64_t)m * m * m;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * du) return;
  const int64_t s = t / du;
  const int64_t p = t - s * du;
  const int i = (int)(p % m), j = (int)((p / m) % m), k = (int)(p / ((int64_t)m * m));
  const double* v = V + s * ldv;
  const double h = 1.0 / n, w1[3] = {1.0, 4.0, 1.0};
  double acc = 0.0;
  for (int dk = -1; dk <= 1; ++dk) {
    const int kk = k + dk;
    if (kk < 0 || kk >= m) continue;
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= m) continue;
      for (int di = -1; di <= 1; ++di) {
        const int ii = i + di;
        if (ii < 0 || ii >= m) continue;
        const int64_t q = ii + (int64_t)m * (jj + (int64_t)m * kk);
        acc += w1[di + 1] * w1[dj + 1] * w1[dk + 1] * (vbar ? v[q] - vbar[q] : v[q]);
      }
    }
  }
  const double c = h / 6.0;
  out[s * ldo + p] = c * c * c * acc;
}

namespace saa_launch {

void field3(const double* xi, const double* S, const double* amp, double* em, int K1, int n, int64_t N,
            hipStream_t st) {
  const size_t lds = sizeof(double) * ((size_t)K1 * K1 + (size_t)K1 * (n + 1));
  saa_k_field3<<<(unsigned)(N * (n + 1)), 256, lds, st>>>(xi, S, amp, em, K1, n, N);
}

template <typename TS>
void hierarchy3(const Pde3Geo& g, const double* em, double* k64, const Mg3Bufs<TS>& b, int64_t N, hipStream_t st) {
  saa_k_hierarchy3<TS><<<(unsigned)N, HB, 0, st>>>(g, em, k64, b, N);
}
template void hierarchy3<float>(const Pde3Geo&, const double*, double*, const Mg3Bufs<float>&, int64_t, hipStream_t);
template void hierarchy3<double>(const Pde3Geo&, const double*, double*, const Mg3Bufs<double>&, int64_t,
                                 hipStream_t);

template <typename TW, typename TS>
void state3(const Pde3Geo& g, const double* Z, int64_t z_stride, const double* k64, TW* u, TW* f,
            const Mg3Bufs<TS>& b, const SolveParams& sp, double* q, int* newton, int* lin, int* flag, int64_t N,
            int bs, hipStream_t st) {
  switch (bs) {
    case 256:
      saa_k_state3<TW, TS, 256><<<(unsigned)N, 256, 0, st>>>(g, Z, z_stride, k64, u, f, b, sp, q, newton, lin, flag,
                                                             N);
      break;
    case 1024:
      saa_k_state3<TW, TS, 1024><<<(unsigned)N, 1024, 0, st>>>(g, Z, z_stride, k64, u, f, b, sp, q, newton, lin,
                                                               flag, N);
      break;
    default:
      saa_k_state3<TW, TS, 512><<<(unsigned)N, 512, 0, st>>>(g, Z, z_stride, k64, u, f, b, sp, q, newton, lin, flag,
                                                             N);
  }
}

// Control Jacobians of samples [s0, s0 + ns) (512-thread workgroups).
template <typename TW, typename TS>
void linearized3(const Pde3Geo& g, const double* k64, const TW* u, TW* bvec, TW* x, const Mg3Bufs<TS>& b,
                 const SolveParams& sp, int64_t s0, int64_t ns, int k0, int nk, double* out, int64_t ld, int* lin,
                 int* flag, int64_t N, hipStream_t st) {
  saa_k_linearized3<TW, TS, 512><<<(unsigned)ns, 512, 0, st>>>(g, k64, u, bvec, x, b, sp, s0, k0, nk, out, ld, lin,
                                                               flag, N);
}

template <typename TW>
void interior_copy3(const TW* u, double* out, int n, int64_t nodes, int64_t N, hipStream_t st) {
  const int64_t du = (int64_t)(n - 1) * (n - 1) * (n - 1);
  saa_k_interior3<TW><<<(unsigned)((N * du + 255) / 256), 256, 0, st>>>(u, out, n, nodes, N);
}
template void interior_copy3<double>(const double*, double*, int, int64_t, int64_t, hipStream_t);
template void interior_copy3<float>(const float*, double*, int, int64_t, int64_t, hipStream_t);

void mass_rows3(const double* V, int64_t ldv, const double* vbar, double* out, int64_t ldo, int n, int64_t rows,
                hipStream_t st) {
  const int64_t du = (int64_t)(n - 1) * (n - 1) * (n - 1);
  saa_k_mass_rows3<<<(unsigned)((rows * du + 255) / 256), 256, 0, st>>>(V, ldv, vbar, out, ldo, n, rows);
}

template <typename TW, typename TS>
void adjoint3(const Pde3Geo& g, const double* k64, const TW* u, TW* bvec, TW* lam, const Mg3Bufs<TS>& b,
              const SolveParams& sp, const double* q, const double* tstar, int act, double act_w, double* gout,
              int* lin, int* flag, int* did, int64_t N, int bs, hipStream_t st) {
  switch (bs) {
    case 256:
      saa_k_adjoint3<TW, TS, 256><<<(unsigned)N, 256, 0, st>>>(g, k64, u, bvec, lam, b, sp, q, tstar, act, act_w, gout,
                                                               lin, flag, did, N);
      break;
    case 1024:
      saa_k_adjoint3<TW, TS, 1024><<<(unsigned)N, 1024, 0, st>>>(g, k64, u, bvec, lam, b, sp, q, tstar, act, act_w,
                                                                 gout, lin, flag, did, N);
      break;
    default:
      saa_k_adjoint3<TW, TS, 512><<<(unsigned)N, 512, 0, st>>>(g, k64, u, bvec, lam, b, sp, q, tstar, act, act_w, gout,
                                                               lin, flag, did, N);
  }
}

#define SAA_INST3(TW, TS)                                                                                    \
  template void state3<TW, TS>(const Pde3Geo&, const double*, int64_t, const double*, TW*, TW*,              \
                               const Mg3Bufs<TS>&, const SolveParams&, double*, int*, int*, int*, int64_t, int,\
                               hipStream_t);                                                                  \
  template void linearized3<TW, TS>(const Pde3Geo&, const double*, const TW*, TW*, TW*, const Mg3Bufs<TS>&,   \
                                    const SolveParams&, int64_t, int64_t, int, int, double*, int64_t, int*,   \
                                    int*, int64_t, hipStream_t);                                              \
  template void adjoint3<TW, TS>(const Pde3Geo&, const double*, const TW*, TW*, TW*, const Mg3Bufs<TS>&,       \
                                 const SolveParams&, const double*, const double*, int, double, double*, int*, \
                                 int*, int*, int64_t, int, hipStream_t);
SAA_INST3(double, double)
SAA_INST3(double, float)
SAA_INST3(float, float)
#undef SAA_INST3

}  // namespace saa_launch
