// PDE form of the SAA objective: batched P1 finite-element Newton solves of
//   -div(exp(m) grad u) + r u^3 = sum_k z_k f_k,  u = 0 on the boundary
// (paper Sec. 4.2, eq. (elliptic_pde)), the tracking QoI, and the adjoint
// gradient dq/dz = F^T lambda, A(u) lambda = dq/du (Sec. 2.3,
// eq. (ouu_qoi_gradient)).
//
// Design: one workgroup owns one sample for its whole solve.  Samples are
// independent, so every Newton step, every preconditioned-CG iteration and
// every multigrid V-cycle of a sample runs inside one persistent workgroup
// with only workgroup barriers; per-sample convergence decisions are taken on
// the device and no grid-wide synchronisation or host round trip is needed.
//
// Discretisation facts used here (all follow from the P1 element matrices on
// the mesh whose cells are split along the (i,j)-(i+1,j+1) diagonal):
//  * the stiffness matrix is a 5-point stencil: the edge (i,j)-(i+1,j) has
//    weight (kappa_lo(i,j) + kappa_up(i,j-1))/2, the edge (i,j)-(i,j+1) has
//    weight (kappa_up(i,j) + kappa_lo(i-1,j))/2, with kappa_T the mean of
//    exp(m) over the vertices of T; diagonal-edge couplings vanish;
//  * the lumped reaction / source weight of an interior node is h^2;
//  * the consistent mass matrix couples a node to its E, W, N, S, NE and SW
//    neighbours with h^2/12 and to itself with h^2/2;
//  * the P1 spaces of the grids n and n/2 are nested, so prolongation is
//    linear interpolation (midpoints of horizontal, vertical and diagonal
//    coarse edges take the mean of the two end values) and the Galerkin
//    coarse stiffness is again the P1 stencil with each coarse triangle's
//    kappa equal to the mean over its four child triangles.
#include <algorithm>

#include "common.h"
#include "outer.h"
#include "pde.h"

#ifndef SAA_PDE_BLOCK
#define SAA_PDE_BLOCK 1024
#endif
#ifndef SAA_PDE_LDS_FIRST
#define SAA_PDE_LDS_FIRST 1
#endif

namespace {

constexpr int BS = SAA_PDE_BLOCK;      // threads per sample
constexpr int LF = SAA_PDE_LDS_FIRST;  // first multigrid level kept in LDS (FP32 solver)
constexpr int FIELD_BAND = 2048;       // doubles of the field kernel's T band in LDS

// ---------------------------------------------------------------------------
// Node iteration: the calling thread visits nodes p = tid, tid + BS, ... of an
// (n+1)^2 grid, tracking (i, j) incrementally.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void for_nodes(int n, F&& f) {
  const int np = n + 1;
  const int total = np * np;
  int p = threadIdx.x;
  if (p >= total) return;
  int j = p / np;
  int i = p - j * np;
  const int sj = BS / np;
  const int si = BS - sj * np;
  for (; p < total; p += BS) {
    f(p, i, j);
    i += si;
    j += sj;
    if (i >= np) {
      i -= np;
      ++j;
    }
  }
}

__device__ __forceinline__ bool interior(int i, int j, int n) {
  return i > 0 && j > 0 && i < n && j < n;
}

// FP64 edge weights of the fine stiffness computed from nodal exp(m):
// WE(i,j) = [2e(i,j) + 2e(i+1,j) + e(i+1,j+1) + e(i,j-1)] / 6
// WN(i,j) = [2e(i,j) + 2e(i,j+1) + e(i+1,j+1) + e(i-1,j)] / 6
template <typename TW>
__device__ __forceinline__ TW weight_e(const double* e, int p, int np) {
  return (TW)((2.0 * e[p] + 2.0 * e[p + 1] + e[p + np + 1] + e[p - np]) * (1.0 / 6.0));
}
template <typename TW>
__device__ __forceinline__ TW weight_n(const double* e, int p, int np) {
  return (TW)((2.0 * e[p] + 2.0 * e[p + np] + e[p + np + 1] + e[p - 1]) * (1.0 / 6.0));
}

// (K u)_p with the fine stiffness from exp(m), in precision TW.
template <typename TW>
__device__ __forceinline__ TW stiff_apply_em(const double* e, const TW* u, int p, int np) {
  const TW we = weight_e<TW>(e, p, np);
  const TW ww = weight_e<TW>(e, p - 1, np);
  const TW wn = weight_n<TW>(e, p, np);
  const TW ws = weight_n<TW>(e, p - np, np);
  return (we + ww + wn + ws) * u[p] - we * u[p + 1] - ww * u[p - 1] - wn * u[p + np] - ws * u[p - np];
}

// ---------------------------------------------------------------------------
// Multigrid building blocks (precision TS), all for one sample.
// ---------------------------------------------------------------------------
template <typename TS>
struct Level {
  int n, np;
  const TS* WE;
  const TS* WN;
  const TS* D;
};

// Array `gbase` (level-stacked, HBM) at level l, or its LDS copy for l >= 1.
template <typename TS>
__device__ __forceinline__ TS* at_level(TS* gbase, TS* lbase, const PdeGeo& g, int l) {
  return (l >= LF && lbase) ? lbase + (g.off[l] - g.off[LF]) : gbase + g.off[l];
}

template <typename TS>
__device__ __forceinline__ Level<TS> level(const PdeGeo& g, const MgBufs<TS>& m, int l) {
  Level<TS> L;
  L.n = g.n[l];
  L.np = g.n[l] + 1;
  L.WE = at_level(m.WE, m.lWE, g, l);
  L.WN = at_level(m.WN, m.lWN, g, l);
  L.D = at_level(m.D, m.lD, g, l);
  return L;
}

// The same visit split in two: `compute` (loads only) returns the node's new
// values, `store` writes them.  The passes whose computed nodes read no value
// that the pass stores (red-black half sweeps, residuals, the CG vector
// passes) are written this way; it gives the compiler independent loads and
// stores to schedule (the FP32 state kernel at n = 128 runs 5 % faster than
// with one load-compute-store body; visiting two nodes of a thread per group
// before storing was much slower).
template <typename C, typename S>
__device__ __forceinline__ void for_nodes_split(int n, C&& compute, S&& store) {
  for_nodes(n, [&](int p, int i, int j) { store(p, i, j, compute(p, i, j)); });
}

template <typename TS>
__device__ __forceinline__ TS offdiag_sum(const Level<TS>& L, const TS* x, int p) {
  return L.WE[p] * x[p + 1] + L.WE[p - 1] * x[p - 1] + L.WN[p] * x[p + L.np] + L.WN[p - L.np] * x[p - L.np];
}

// One red-black Gauss-Seidel half sweep on colour c: x_p = (b_p + sum w x_q) / D_p.
// If `first`, the other colour is known to be zero and x_p = b_p / D_p.
template <typename TS>
__device__ void gs_half(const Level<TS>& L, const TS* b, TS* x, int c, bool first) {
  auto on = [&](int i, int j) { return interior(i, j, L.n) && ((i + j) & 1) == c; };
  for_nodes_split(
      L.n,
      [&](int p, int i, int j) -> TS {
        if (!on(i, j)) return (TS)0;
        TS s = b[p];
        if (!first) s += offdiag_sum(L, x, p);
        return s / L.D[p];
      },
      [&](int p, int i, int j, TS v) {
        if (on(i, j)) x[p] = v;
      });
  __syncthreads();
}

// Restriction R = P^T from the fine level (n) to the coarse level (n/2).
template <typename TS>
__device__ void restrict_level(int nf, const TS* t, int nc, TS* bc) {
  const int npf = nf + 1;
  for_nodes(nc, [&](int pc, int I, int J) {
    if (interior(I, J, nc)) {
      const int p = (2 * J) * npf + 2 * I;
      bc[pc] = t[p] + (TS)0.5 * (t[p + 1] + t[p - 1] + t[p + npf] + t[p - npf] + t[p + npf + 1] + t[p - npf - 1]);
    }
  });
  __syncthreads();
}

// Fine-level pieces of a V(1,1) cycle fused with the CG vector passes:
//  * the first red half sweep x_red = b_red / D (black taken as zero) is
//    done where the CG residual is updated (pcg);
//  * after the black half sweep the black residuals vanish (every neighbour
//    of a black node is red), so only the red residuals are formed and the
//    restriction reads those: b_c(I,J) = t(2I,2J) + (t(2I+1,2J+1) +
//    t(2I-1,2J-1)) / 2;
//  * the post-smoothing half sweeps also accumulate r . z (z final per colour).
template <typename TS>
__device__ void residual_red(const Level<TS>& L, const TS* b, const TS* x, TS* t) {
  auto on = [&](int i, int j) { return interior(i, j, L.n) && !((i + j) & 1); };
  for_nodes_split(
      L.n,
      [&](int p, int i, int j) -> TS {
        return on(i, j) ? b[p] - (L.D[p] * x[p] - offdiag_sum(L, x, p)) : (TS)0;
      },
      [&](int p, int i, int j, TS v) {
        if (on(i, j)) t[p] = v;
      });
  __syncthreads();
}

template <typename TS>
__device__ void restrict_red(int nf, const TS* t, int nc, TS* bc) {
  const int npf = nf + 1;
  for_nodes_split(
      nc,
      [&](int pc, int I, int J) -> TS {
        if (!interior(I, J, nc)) return (TS)0;
        const int p = (2 * J) * npf + 2 * I;
        return t[p] + (TS)0.5 * (t[p + npf + 1] + t[p - npf - 1]);
      },
      [&](int pc, int I, int J, TS v) {
        if (interior(I, J, nc)) bc[pc] = v;
      });
  __syncthreads();
}

// Half sweep of colour c that also returns this thread's part of sum b_p x_p
// over the nodes of that colour (after their update).
template <typename TS>
__device__ double gs_half_dot(const Level<TS>& L, const TS* b, TS* x, int c) {
  struct BV {
    TS b, v;
  };
  auto on = [&](int i, int j) { return interior(i, j, L.n) && ((i + j) & 1) == c; };
  double acc = 0.0;
  for_nodes_split(
      L.n,
      [&](int p, int i, int j) -> BV {
        if (!on(i, j)) return BV{(TS)0, (TS)0};
        const TS bp = b[p];
        return BV{bp, (bp + offdiag_sum(L, x, p)) / L.D[p]};
      },
      [&](int p, int i, int j, const BV& r) {
        if (on(i, j)) {
          x[p] = r.v;
          acc += (double)r.b * (double)r.v;
        }
      });
  __syncthreads();
  return acc;
}

// Post-smoothing black half sweep fused with the prolongation x += P x_c:
// the red neighbours of a black node are read as x_k + (P x_c)_k (linear
// interpolation at a red fine node: the coincident coarse value at (even,
// even), the mean of the two diagonal ends at (odd, odd)).  The prolonged
// values are never stored: black nodes are overwritten here and red nodes by
// the red half sweep that follows (which reads black neighbours only).
// Returns this thread's part of sum b_p x_p over the black nodes.
template <typename TS>
__device__ double gs_black_prolong(const Level<TS>& L, const TS* b, TS* x, const TS* xc) {
  const int npc = L.n / 2 + 1;
  auto xr = [&](int q, int i, int j) -> TS {   // prolonged value at the red node q = (i, j)
    const int qc = (j >> 1) * npc + (i >> 1);
    const TS v = (i & 1) ? (TS)0.5 * (xc[qc] + xc[qc + npc + 1]) : xc[qc];
    return x[q] + v;
  };
  struct BV {
    TS b, v;
  };
  auto on = [&](int i, int j) { return interior(i, j, L.n) && ((i + j) & 1); };
  double acc = 0.0;
  for_nodes_split(
      L.n,
      [&](int p, int i, int j) -> BV {
        if (!on(i, j)) return BV{(TS)0, (TS)0};
        const TS bp = b[p];
        const TS off = L.WE[p] * xr(p + 1, i + 1, j) + L.WE[p - 1] * xr(p - 1, i - 1, j) +
                       L.WN[p] * xr(p + L.np, i, j + 1) + L.WN[p - L.np] * xr(p - L.np, i, j - 1);
        return BV{bp, (bp + off) / L.D[p]};
      },
      [&](int p, int i, int j, const BV& r) {
        if (on(i, j)) {
          x[p] = r.v;
          acc += (double)r.b * (double)r.v;
        }
      });
  __syncthreads();
  return acc;
}

// V(1,1) cycle from level l0 down and back to l0, its right-hand side already
// restricted to B_l0: red, black (with the red residuals restricted, as on
// the fine level), coarse correction, black fused with the prolongation, red.
// Exact solve on the 3-cell grid: red nodes (1,1), (2,2) and black nodes
// (2,1), (1,2); eliminating the black unknowns leaves a 2 x 2 Schur
// complement (FP64).
template <typename TS>
__device__ __noinline__ void coarsest3(const Level<TS> lc, const TS* B, TS* X) {
  const int np = lc.np;
  const int r0 = np + 1, r1 = 2 * np + 2, b0 = np + 2, b1 = 2 * np + 1;
  // couplings C[r][b] (edge weights): r0-b0 horizontal, r0-b1 vertical,
  // r1-b0 vertical, r1-b1 horizontal
  const double c00 = lc.WE[r0], c01 = lc.WN[r0], c10 = lc.WN[b0], c11 = lc.WE[b1];
  const double ib0 = 1.0 / (double)lc.D[b0], ib1 = 1.0 / (double)lc.D[b1];
  const double s00 = (double)lc.D[r0] - (c00 * c00 * ib0 + c01 * c01 * ib1);
  const double s11 = (double)lc.D[r1] - (c10 * c10 * ib0 + c11 * c11 * ib1);
  const double s01 = -(c00 * c10 * ib0 + c01 * c11 * ib1);
  const double bb0 = B[b0], bb1 = B[b1];
  const double h0 = (double)B[r0] + c00 * bb0 * ib0 + c01 * bb1 * ib1;
  const double h1 = (double)B[r1] + c10 * bb0 * ib0 + c11 * bb1 * ib1;
  const double idet = 1.0 / (s00 * s11 - s01 * s01);
  const double x0 = (s11 * h0 - s01 * h1) * idet, x1 = (s00 * h1 - s01 * h0) * idet;
  X[r0] = (TS)x0;
  X[r1] = (TS)x1;
  X[b0] = (TS)((bb0 + c00 * x0 + c10 * x1) * ib0);
  X[b1] = (TS)((bb1 + c01 * x0 + c11 * x1) * ib1);
}

template <typename TS>
__device__ void vcycle_from(const PdeGeo& g, const MgBufs<TS>& m, int l0) {
  const int L = g.L;
  for (int l = l0; l < L - 1; ++l) {
    const Level<TS> lv = level(g, m, l);
    const TS* b = at_level(m.B, m.lB, g, l);
    TS* x = at_level(m.X, m.lX, g, l);
    TS* t = at_level(m.T, m.lT, g, l);
    gs_half(lv, b, x, 0, true);
    gs_half(lv, b, x, 1, false);
    residual_red(lv, b, (const TS*)x, t);
    restrict_red(g.n[l], (const TS*)t, g.n[l + 1], at_level(m.B, m.lB, g, l + 1));
  }
  {  // coarsest level, solved exactly: one unknown (n = 2); the 3-cell grid
     // of 3 * 2^k hierarchies goes to an out-of-line solver (inlined, its
     // code slows the CG loop of the power-of-two grids by 11 %)
    const int l = L - 1;
    if (threadIdx.x == 0) {
      const Level<TS> lc = level(g, m, l);
      TS* X = at_level(m.X, m.lX, g, l);
      const TS* B = at_level(m.B, m.lB, g, l);
      if (lc.n == 2) {
        const int p = lc.np + 1;
        X[p] = B[p] / lc.D[p];
      } else {
        coarsest3(lc, B, X);
      }
    }
    __syncthreads();
  }
  for (int l = L - 2; l >= l0; --l) {
    const Level<TS> lv = level(g, m, l);
    const TS* b = at_level(m.B, m.lB, g, l);
    TS* x = at_level(m.X, m.lX, g, l);
    (void)gs_black_prolong(lv, b, x, (const TS*)at_level(m.X, m.lX, g, l + 1));
    gs_half(lv, b, x, 0, false);
  }
}

// Lumped reaction 3 r h^2 u^2 on the fine level and its restrictions; sets
// D_l = KD_l + reaction_l on every level.  Uses T as scratch.
template <typename TW, typename TS>
__device__ void build_diagonals(const PdeGeo& g, const MgBufs<TS>& m, const TW* u) {
  const double c = 3.0 * g.r * g.h2;
  struct TD {
    TS t, d;
  };
  for_nodes_split(
      g.n[0],
      [&](int p, int i, int j) -> TD {
        if (!interior(i, j, g.n[0])) return TD{(TS)0, (TS)0};
        const double uu = (double)u[p];
        const TS d = (TS)(c * uu * uu);
        return TD{d, m.KD[p] + d};
      },
      [&](int p, int i, int j, const TD& r) {
        if (interior(i, j, g.n[0])) {
          m.T[p] = r.t;
          m.D[p] = r.d;
        }
      });
  __syncthreads();
  for (int l = 0; l < g.L - 1; ++l) {
    TS* tc = at_level(m.T, m.lT, g, l + 1);
    TS* dc = at_level(m.D, m.lD, g, l + 1);
    const TS* kd = m.KD + g.off[l + 1];
    restrict_level(g.n[l], at_level(m.T, m.lT, g, l), g.n[l + 1], tc);
    for_nodes(g.n[l + 1], [&](int p, int i, int j) {
      if (interior(i, j, g.n[l + 1])) dc[p] = kd[p] + tc[p];
    });
    __syncthreads();
  }
}

// Move the coarse levels (LF..L-1) of one sample into LDS: zero WE, WN, D, X,
// B, T there (boundary entries stay zero) and copy the edge weights.
template <typename TS>
__device__ void setup_lds_levels(const PdeGeo& g, MgBufs<TS>& m, TS* lds) {
  const int64_t cs = g.lstride - g.off[LF];
  m.lWE = lds;
  m.lWN = lds + cs;
  m.lD = lds + 2 * cs;
  m.lX = lds + 3 * cs;
  m.lB = lds + 4 * cs;
  m.lT = lds + 5 * cs;
  for (int64_t i = threadIdx.x; i < 6 * cs; i += BS) lds[i] = (TS)0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < cs; i += BS) {
    m.lWE[i] = m.WE[g.off[LF] + i];
    m.lWN[i] = m.WN[g.off[LF] + i];
  }
  __syncthreads();
}

// Preconditioned CG on A x = b with b in m.cr (overwritten by the residual),
// x in m.cx.  Returns iterations; sets *ok = false if not converged.  The
// preconditioner is one V(1,1) cycle (SolveParams.nu = 1); its fine-level
// passes are folded into the CG vector passes (see vcycle_from and
// restrict_red) and every piece of it appears once in the code.
template <typename TS>
__device__ int pcg(const PdeGeo& g, const MgBufs<TS>& m, double rtol, int max_it, int nu, double* red, bool* ok) {
  (void)nu;
  const Level<TS> L0 = level(g, m, 0);
  const Level<TS>& Ls = L0;   // fine-level smoother operator
  const int n = g.n[0];
  double rr0 = 0.0;
  for_nodes(n, [&](int p, int i, int j) {
    if (interior(i, j, n)) {
      const double r = (double)m.cr[p];
      rr0 += r * r;
      m.cx[p] = (TS)0;
    }
  });
  rr0 = block_sum1(rr0, red);
  if (!(rr0 > 0.0)) {
    *ok = (rr0 == 0.0);
    return 0;
  }
  TS* z = m.X;  // level-0 V-cycle output
  // first red half sweep of the first V-cycle (later ones ride on the update)
  for_nodes(n, [&](int p, int i, int j) {
    if (interior(i, j, n) && !((i + j) & 1)) z[p] = m.cr[p] / Ls.D[p];
  });
  __syncthreads();
  const double tol2 = rtol * rtol * rr0;
  // search directions alternate between cp and the (otherwise unused) level-0
  // part of B; p = z + beta p_old is formed inside the product A p
  // (neighbour values recomputed; beta = 0 in the first iteration, and both
  // buffers only ever hold finite values)
  TS* pc = m.cp;
  TS* pn = m.B;
  TS beta = (TS)0;
  double rz = 0.0;
  struct PQ {
    TS p, q;
  };
  struct XRZ {
    TS x, r, d;
  };
  for (int it = 0; it <= max_it; ++it) {
    if (it > 0) {
      double pq = 0.0;
      const TS* po = pc;
      TS* pw = pn;
      for_nodes_split(
          n,
          [&](int p, int i, int j) -> PQ {
            if (!interior(i, j, n)) return PQ{(TS)0, (TS)0};
            auto pv = [&](int k) { return z[k] + beta * po[k]; };   // zero on the boundary
            const TS pp = pv(p);
            const TS q = L0.D[p] * pp - (L0.WE[p] * pv(p + 1) + L0.WE[p - 1] * pv(p - 1) +
                                         L0.WN[p] * pv(p + L0.np) + L0.WN[p - L0.np] * pv(p - L0.np));
            return PQ{pp, q};
          },
          [&](int p, int i, int j, const PQ& v) {
            if (interior(i, j, n)) {
              pw[p] = v.p;
              m.cq[p] = v.q;
              pq += (double)v.p * (double)v.q;
            }
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
      for_nodes_split(
          n,
          [&](int p, int i, int j) -> XRZ {
            if (!interior(i, j, n)) return XRZ{(TS)0, (TS)0, (TS)1};
            return XRZ{m.cx[p] + a * pc[p], m.cr[p] - a * m.cq[p], !((i + j) & 1) ? Ls.D[p] : (TS)1};
          },
          [&](int p, int i, int j, const XRZ& v) {
            if (interior(i, j, n)) {
              m.cx[p] = v.x;
              m.cr[p] = v.r;
              rr += (double)v.r * (double)v.r;
              if (!((i + j) & 1)) z[p] = v.r / v.d;   // first red half sweep of the next V-cycle
            }
          });
      rr = block_sum1(rr, red);
      if (rr <= tol2) return it;
    }
    // rest of the V-cycle: black sweep, red residuals restricted, coarse
    // levels, post-smoothing (the black half fused with the prolongation)
    // with r . z
    gs_half(Ls, (const TS*)m.cr, z, 1, false);
    residual_red(Ls, (const TS*)m.cr, (const TS*)z, m.T);
    restrict_red(n, (const TS*)m.T, g.n[1], at_level(m.B, m.lB, g, 1));
    vcycle_from(g, m, 1);
    double rzn = gs_black_prolong(Ls, (const TS*)m.cr, z, (const TS*)at_level(m.X, m.lX, g, 1));
    rzn += gs_half_dot(Ls, (const TS*)m.cr, z, 0);
    rzn = block_sum1(rzn, red);
    beta = (TS)(it > 0 ? rzn / rz : 0.0);
    rz = rzn;
  }
  *ok = false;
  return max_it;
}

// Per-sample views of the batched buffers.
template <typename TS>
__device__ __forceinline__ MgBufs<TS> sample_bufs(const MgBufs<TS>& all, const PdeGeo& g, int64_t s) {
  MgBufs<TS> m;
  const int64_t ls = s * g.lstride, ns = s * g.nodes;
  m.WE = all.WE + ls;
  m.WN = all.WN + ls;
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

// Defect correction for A(u) x = b with A in precision TW (exact fine
// stiffness from exp(m) plus 3 r h^2 u^2) and inner PCG in precision TS.
// b and x are TW node vectors.  The multigrid diagonals must already be built
// for u.  Returns the number of inner CG iterations; clears *ok on failure.
template <typename TW, typename TS>
__device__ int dc_solve(const PdeGeo& g, const MgBufs<TS>& m, const SolveParams& sp,
                        const double* em, const TW* u, const TW* b, TW* x, double* red,
                        bool* ok, int* passes) {
  const int n = g.n[0], np = n + 1;
  const double c = 3.0 * g.r * g.h2;
  int lin = 0;
  for_nodes(n, [&](int p, int i, int j) {
    x[p] = (TW)0;
    if (interior(i, j, n)) m.cr[p] = (TS)b[p];
  });
  __syncthreads();
  int pass = 0;
  OuterCtl ctl;
  ctl.eta = sp.lin_rtol;
  for (pass = 0; pass < sp.max_dc; ++pass) {
    bool cg_ok = true;
    lin += pcg(g, m, ctl.eta, sp.max_lin, sp.nu, red, &cg_ok);
    double v[2] = {0.0, 0.0};
    struct DX {
      TW d, xn;
    };
    for_nodes_split(
        n,
        [&](int p, int i, int j) -> DX {
          if (!interior(i, j, n)) return DX{(TW)0, (TW)0};
          const TW d = (TW)m.cx[p];
          return DX{d, x[p] + d};
        },
        [&](int p, int i, int j, const DX& r) {
          if (interior(i, j, n)) {
            x[p] = r.xn;
            v[0] += (double)r.d * (double)r.d;
            v[1] += (double)r.xn * (double)r.xn;
          }
        });
    block_sum<2>(v, red);
    if (!(v[0] == v[0]) || !(v[1] == v[1])) {
      *ok = false;
      break;
    }
    if (outer_converged(ctl, v[0], v[1], sp.adj_tol, sp.lin_rtol)) break;
    // new defect b - A x in precision TW
    for_nodes_split(
        n,
        [&](int p, int i, int j) -> TW {
          if (!interior(i, j, n)) return (TW)0;
          const TW uu = u[p];
          const TW ax = stiff_apply_em<TW>(em, x, p, np) + (TW)c * uu * uu * x[p];
          return b[p] - ax;
        },
        [&](int p, int i, int j, TW r) {
          if (interior(i, j, n)) m.cr[p] = (TS)r;
        });
    __syncthreads();
  }
  if (pass == sp.max_dc) *ok = false;
  *passes = pass + 1;
  return lin;
}

}  // namespace

// ---------------------------------------------------------------------------
// Setup kernels (run once per sample set; not part of an objective evaluation)
// ---------------------------------------------------------------------------

// S[j][i] = sin((j+1) pi i / n), j < K1, 0 <= i <= n.
__global__ void saa_k_sine_table(double* S, int K1, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K1 * (n + 1)) return;
  const int j = t / (n + 1), i = t - j * (n + 1);
  S[t] = sin(M_PI * (double)((j + 1) * i) / (double)n);
}

// FT[k][p] = h^2 f_k(x_p) on interior nodes (lumped P1 load), 0 on the boundary.
__global__ void saa_k_source_matrix(double* FT, int n, int s, double sigma) {
  const int np = n + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nodes = (int64_t)np * np;
  if (t >= nodes * s * s) return;
  const int k = (int)(t / nodes);
  const int p = (int)(t - (int64_t)k * nodes);
  const int j = p / np, i = p - j * np;
  double v = 0.0;
  if (i > 0 && j > 0 && i < n && j < n) {
    const int a = k % s, b = k / s;
    const double h = 1.0 / n;
    const double cx = (a + 1.0) / (s + 1.0), cy = (b + 1.0) / (s + 1.0);
    const double dx = i * h - cx, dy = j * h - cy;
    v = h * h * exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma)) / (sigma * sqrt(2.0 * M_PI));
  }
  FT[t] = v;
}

// Nodal exp(m) of each sample: m = sum_jk a_jk xi_jk sin(j pi x) sin(k pi y),
// evaluated separably.  The K1 x (n+1) intermediate T[j][y] = sum_k a_jk
// xi_jk sin(k pi y) is built in LDS a band of `rows` grid rows at a time, so
// the LDS footprint does not grow with n.  One block per sample.
__global__ void __launch_bounds__(256) saa_k_field(const double* xi, const double* S, const double* amp,
                                                   double* em, int K1, int n, int rows, int64_t N) {
  extern __shared__ double sh[];
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  const int np = n + 1;
  double* axi = sh;                 // K1 x K1
  double* Tjy = sh + K1 * K1;       // K1 x rows: the current band of T
  const double* x = xi + s * K1 * K1;
  for (int t = threadIdx.x; t < K1 * K1; t += blockDim.x) axi[t] = amp[t] * x[t];
  double* e = em + s * (int64_t)np * np;
  for (int y0 = 0; y0 < np; y0 += rows) {
    const int ny = (np - y0 < rows) ? (np - y0) : rows;
    __syncthreads();  // axi written / previous band consumed
    for (int t = threadIdx.x; t < K1 * ny; t += blockDim.x) {
      const int j = t / ny, y = t - j * ny;
      double acc = 0.0;
      for (int k = 0; k < K1; ++k) acc += axi[j * K1 + k] * S[k * np + y0 + y];
      Tjy[t] = acc;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < ny * np; p += blockDim.x) {
      const int y = p / np, xx = p - y * np;
      double acc = 0.0;
      for (int j = 0; j < K1; ++j) acc += Tjy[j * ny + y] * S[j * np + xx];
      e[(int64_t)(y0 + y) * np + xx] = exp(acc);
    }
  }
}

// Multigrid hierarchy of each sample: per-triangle kappa on every level
// (fine: vertex means of exp(m); coarse: mean of the four child triangles),
// then edge weights and stiffness diagonals.  kap: per-sample scratch of
// 2 * sum_l n_l^2 doubles.  One block per sample.
template <typename TS>
__global__ void __launch_bounds__(BS) saa_k_hierarchy(PdeGeo g, const double* em_all, double* kap_all,
                                                      int64_t kstride, MgBufs<TS> all, int64_t s0,
                                                      int64_t N) {
  const int64_t s = s0 + blockIdx.x;
  if (s >= N) return;
  const double* e = em_all + s * g.nodes;
  double* kap = kap_all + (int64_t)blockIdx.x * kstride;
  MgBufs<TS> m = sample_bufs(all, g, s);
  // kappa offsets per level: lo at ko, up at ko + n^2
  int64_t ko = 0;
  for (int l = 0; l < g.L; ++l) {
    const int n = g.n[l];
    double* klo = kap + ko;
    double* kup = klo + (int64_t)n * n;
    if (l == 0) {
      const int np = n + 1;
      for (int c = threadIdx.x; c < n * n; c += BS) {
        const int j = c / n, i = c - j * n;
        const int p = j * np + i;
        klo[c] = (e[p] + e[p + 1] + e[p + np + 1]) / 3.0;
        kup[c] = (e[p] + e[p + np + 1] + e[p + np]) / 3.0;
      }
    } else {
      const int nf = 2 * n;
      const double* flo = kap + ko - 2 * (int64_t)nf * nf;
      const double* fup = flo + (int64_t)nf * nf;
      for (int c = threadIdx.x; c < n * n; c += BS) {
        const int J = c / n, I = c - J * n;
        const int f00 = (2 * J) * nf + 2 * I, f10 = f00 + 1, f01 = f00 + nf, f11 = f00 + nf + 1;
        klo[c] = 0.25 * (flo[f00] + flo[f10] + flo[f11] + fup[f10]);
        kup[c] = 0.25 * (fup[f00] + fup[f11] + fup[f01] + flo[f01]);
      }
    }
    __syncthreads();
    // edge weights and diagonal on the node grid of this level
    const int np = n + 1;
    TS* WE = m.WE + g.off[l];
    TS* WN = m.WN + g.off[l];
    TS* KD = m.KD + g.off[l];
    for (int p = threadIdx.x; p < np * np; p += BS) {
      const int j = p / np, i = p - j * np;
      double we = 0.0, wn = 0.0;
      if (i < n && j >= 1 && j <= n - 1) we = 0.5 * (klo[j * n + i] + kup[(j - 1) * n + i]);
      if (j < n && i >= 1 && i <= n - 1) wn = 0.5 * (kup[j * n + i] + klo[j * n + i - 1]);
      WE[p] = (TS)we;
      WN[p] = (TS)wn;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < np * np; p += BS) {
      const int j = p / np, i = p - j * np;
      TS d = (TS)0;
      if (i > 0 && j > 0 && i < n && j < n) d = WE[p] + WE[p - 1] + WN[p] + WN[p - np];
      KD[p] = d;
      m.D[g.off[l] + p] = d;
    }
    __syncthreads();
    ko += 2 * (int64_t)n * n;
  }
}

// ---------------------------------------------------------------------------
// State solve: Newton (precision TW) with inner MG-PCG (precision TS), then
// the QoI q = (u - ut)^T M (u - ut) over all nodes.  One block per sample.
// Z: controls, sample s uses Z + s * z_stride (z_stride = 0: shared control).
// ---------------------------------------------------------------------------
// One sample's state solve (shared by the single- and multi-problem kernels).
template <typename TW, typename TS, bool LDSC>
__device__ __forceinline__ void state_sample(const PdeGeo& g, const double* FT, const double* Z, int64_t z_stride,
                                             const double* em_all, TW* u_all, TW* f_all, const MgBufs<TS>& all,
                                             const SolveParams& sp, double* q_out, int* newton_out, int* lin_out,
                                             int* flag_out, int64_t s, double* red, double* zs) {
  const int n = g.n[0], np = n + 1;
  const double* em = em_all + s * g.nodes;
  TW* u = u_all + s * g.nodes;
  TW* f = f_all + s * g.nodes;
  MgBufs<TS> m = sample_bufs(all, g, s);
  if (LDSC) {
    extern __shared__ char dyn_lds[];
    setup_lds_levels(g, m, (TS*)dyn_lds);
  }
  if (threadIdx.x < g.dz) zs[threadIdx.x] = Z[s * z_stride + threadIdx.x];
  __syncthreads();
  const double c = g.r * g.h2;
  // Initialising passes write every node (boundary zeros included): the TW
  // buffers are shared by the FP32 and FP64 state precisions.
  // f = F z from the separable factors: f_p = c sum_b G[b][j] sum_a z_{s b + a} G[a][i]
  const int ns = g.src_s;
  for_nodes(n, [&](int p, int i, int j) {
    double acc = 0.0;
    if (interior(i, j, n)) {
      for (int b = 0; b < ns; ++b) {
        double t = 0.0;
        for (int a = 0; a < ns; ++a) t += zs[ns * b + a] * g.src1[a * np + i];
        acc += g.src1[b * np + j] * t;
      }
      acc *= g.src_c;
    }
    f[p] = (TW)acc;
    u[p] = (TW)0;
  });
  __syncthreads();
  int flags = 0, lin = 0, it = 0;
  bool conv = false;
  OuterCtl ctl;
  ctl.eta = sp.lin_rtol;
  for (it = 0; it < sp.max_newton; ++it) {
    // residual R = K u + r h^2 u^3 - f; CG right-hand side -R
    for_nodes_split(
        n,
        [&](int p, int i, int j) -> TW {
          if (!interior(i, j, n)) return (TW)0;
          const TW uu = u[p];
          return stiff_apply_em<TW>(em, u, p, np) + (TW)c * uu * uu * uu - f[p];
        },
        [&](int p, int i, int j, TW R) {
          if (interior(i, j, n)) m.cr[p] = (TS)(-R);
        });
    __syncthreads();
    build_diagonals<TW, TS>(g, m, u);
    bool ok = true;
    lin += pcg(g, m, ctl.eta, sp.max_lin, sp.nu, red, &ok);
    if (!ok) flags |= SAA_FLAG_CG;
    double v[2] = {0.0, 0.0};
    struct DU {
      TW d, un;
    };
    for_nodes_split(
        n,
        [&](int p, int i, int j) -> DU {
          if (!interior(i, j, n)) return DU{(TW)0, (TW)0};
          const TW d = (TW)m.cx[p];
          return DU{d, u[p] + d};
        },
        [&](int p, int i, int j, const DU& r) {
          if (interior(i, j, n)) {
            u[p] = r.un;
            v[0] += (double)r.d * (double)r.d;
            v[1] += (double)r.un * (double)r.un;
          }
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
  // QoI: q = u^T M_II u - 2 u^T (M ut)_I + ut^T M ut (u = 0 on the boundary).
  const double h2 = g.h2;
  double qa = 0.0;
  for_nodes(n, [&](int p, int i, int j) {
    if (interior(i, j, n)) {
      const double up = (double)u[p];
      const double mu = (h2 / 12.0) * (6.0 * up + (double)u[p + 1] + (double)u[p - 1] + (double)u[p + np] +
                                       (double)u[p - np] + (double)u[p + np + 1] + (double)u[p - np - 1]);
      qa += up * (mu - 2.0 * g.mt[p]);
    }
  });
  qa = block_sum1(qa, red);
  if (threadIdx.x == 0) {
    q_out[s] = qa + g.ctt;
    newton_out[s] = it;
    lin_out[s] = lin;
    flag_out[s] = flags;
  }
}

template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_state(PdeGeo g, const double* FT, const double* Z,
                                                  int64_t z_stride, const double* em_all, TW* u_all,
                                                  TW* f_all, MgBufs<TS> all, SolveParams sp, double* q_out,
                                                  int* newton_out, int* lin_out, int* flag_out, int64_t N) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  __shared__ double zs[SAA_MAX_DZ];
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  state_sample<TW, TS, LDSC>(g, FT, Z, z_stride, em_all, u_all, f_all, all, sp, q_out, newton_out, lin_out, flag_out,
                             s, red, zs);
}

// Several problems in one launch: block b belongs to the last job whose first
// block is <= b (job descriptors in device memory, read uniformly).
template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_state_multi(const StateJob<TW, TS>* jobs, int count, SolveParams sp) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  __shared__ double zs[SAA_MAX_DZ];
  int p = 0;
  for (int k = 1; k < count; ++k)
    if ((int64_t)blockIdx.x >= jobs[k].first) p = k;
  const StateJob<TW, TS>& J = jobs[p];
  const int64_t s = (int64_t)blockIdx.x - J.first;
  if (s >= J.N) return;
  state_sample<TW, TS, LDSC>(J.g, J.FT, J.Z, 0, J.em, J.u, J.f, J.b, sp, J.q, J.newton, J.lin, J.flag, s, red, zs);
}

// ---------------------------------------------------------------------------
// Adjoint: A(u) lambda = 2 (M (u - ut))_I, g = F^T lambda (Sec. 2.3).  One
// block per sample.  Only samples whose risk weight can be non-zero are
// solved (act 0: q_i > t, the CVaR weight s_eps'(q - t) > 0; act 1: all;
// act 2: 0 < q_i - t < act_w, the smoothed failure-probability weight
// s_eps''(q - t) != 0; act 3: a (q_i - act_w) + 1 > 0 with a = t > 0, the
// buffered-exceedance weight a s_eps'(a (q - tau) + 1)); the others get a
// zero g row.
// ---------------------------------------------------------------------------
// One sample's adjoint (shared by the single- and multi-problem kernels).
template <typename TW, typename TS, bool LDSC>
__device__ __forceinline__ void adjoint_sample(const PdeGeo& g, const double* FT, const double* em_all,
                                               const TW* u_all, TW* b_all, TW* lam_all, const MgBufs<TS>& all,
                                               const SolveParams& sp, const double* q, const double* tstar, int act,
                                               double act_w, double* g_out, int* lin_out, int* flag_out,
                                               int* did_out, int64_t s, double* red) {
  const int n = g.n[0], np = n + 1;
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
  const double* em = em_all + s * g.nodes;
  const TW* u = u_all + s * g.nodes;
  TW* b = b_all + s * g.nodes;
  TW* lam = lam_all + s * g.nodes;
  MgBufs<TS> m = sample_bufs(all, g, s);
  if (LDSC) {
    extern __shared__ char dyn_lds[];
    setup_lds_levels(g, m, (TS*)dyn_lds);
  }
  const double h2 = g.h2;
  for_nodes(n, [&](int p, int i, int j) {
    double v = 0.0;
    if (interior(i, j, n)) {
      const double up = (double)u[p];
      const double mu = (h2 / 12.0) * (6.0 * up + (double)u[p + 1] + (double)u[p - 1] + (double)u[p + np] +
                                       (double)u[p - np] + (double)u[p + np + 1] + (double)u[p - np - 1]);
      v = 2.0 * (mu - g.mt[p]);
    }
    b[p] = (TW)v;
  });
  __syncthreads();
  build_diagonals<TW, TS>(g, m, u);
  bool ok = true;
  int passes = 0;
  const int lin = dc_solve<TW, TS>(g, m, sp, em, u, b, lam, red, &ok, &passes);
  // g = F^T lambda from the separable factors: g_{s b + a} = c sum_j G[b][j] r_a(j)
  // with the row sums r_a(j) = sum_i G[a][i] lambda_ij.  Each wave takes whole
  // interior rows (lanes split the row, a butterfly sum gives every lane the
  // s row sums); lane s b + a accumulates its control; the waves' partials are
  // added in wave order.
  {
    const int ns = g.src_s, lane = threadIdx.x & (SAA_WAVE - 1), wid = threadIdx.x / SAA_WAVE;
    const int nw = blockDim.x / SAA_WAVE;
    const int la = lane % ns, lb = lane / ns;   // this lane's control (a, b) when lane < s^2
    double acc = 0.0;
    for (int j = 1 + wid; j < n; j += nw) {
      double r[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) r[a] = 0.0;
      for (int i = 1 + lane; i < n; i += SAA_WAVE) {
        const double l = (double)lam[j * np + i];
#pragma unroll
        for (int a = 0; a < 8; ++a)
          if (a < ns) r[a] += g.src1[a * np + i] * l;
      }
      double ra = 0.0;
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (a < ns) {
          const double t = wave_sum(r[a]);
          if (a == la) ra = t;
        }
      }
      if (lane < g.dz) acc += g.src1[lb * np + j] * ra;
    }
    red[wid * SAA_WAVE + lane] = acc;
    __syncthreads();
    if (threadIdx.x < g.dz) {
      double v = 0.0;
      for (int w = 0; w < nw; ++w) v += red[w * SAA_WAVE + threadIdx.x];
      g_out[s * g.dz + threadIdx.x] = g.src_c * v;
    }
  }
  if (threadIdx.x == 0) {
    lin_out[s] = lin;
    did_out[s] = 1;
    if (!ok) flag_out[s] |= SAA_FLAG_DC;
  }
}

// ---------------------------------------------------------------------------
// Control Jacobian du/dz = A(u)^{-1} F by d_Z linearised solves sharing the
// state's multigrid hierarchy (Sec. 3.4, eq. (projected_sensitivity)).
// Output dudz[s][k][interior index] in float64.  One block per sample.
// ---------------------------------------------------------------------------
template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_adjoint(PdeGeo g, const double* FT, const double* em_all,
                                                    const TW* u_all, TW* b_all, TW* lam_all, MgBufs<TS> all,
                                                    SolveParams sp, const double* q, const double* tstar,
                                                    int act, double act_w, double* g_out, int* lin_out,
                                                    int* flag_out, int* did_out, int64_t N) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  adjoint_sample<TW, TS, LDSC>(g, FT, em_all, u_all, b_all, lam_all, all, sp, q, tstar, act, act_w, g_out, lin_out,
                               flag_out, did_out, s, red);
}

template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_adjoint_multi(const AdjointJob<TW, TS>* jobs, int count, SolveParams sp,
                                                          int act, double act_w) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  int p = 0;
  for (int k = 1; k < count; ++k)
    if ((int64_t)blockIdx.x >= jobs[k].first) p = k;
  const AdjointJob<TW, TS>& J = jobs[p];
  const int64_t s = (int64_t)blockIdx.x - J.first;
  if (s >= J.N) return;
  adjoint_sample<TW, TS, LDSC>(J.g, J.FT, J.em, J.u, J.bvec, J.lam, J.b, sp, J.q, J.tstar, act, act_w, J.gout, J.lin,
                               J.flag, J.did, s, red);
}

template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_linearized(PdeGeo g, const double* FT, const double* em_all,
                                                       const TW* u_all, TW* b_all, TW* x_all, MgBufs<TS> all,
                                                       SolveParams sp, double* dudz, int* lin_out, int* flag_out,
                                                       int64_t N) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  const int n = g.n[0];
  const int64_t du = (int64_t)(n - 1) * (n - 1);
  const double* em = em_all + s * g.nodes;
  const TW* u = u_all + s * g.nodes;
  TW* b = b_all + s * g.nodes;
  TW* x = x_all + s * g.nodes;
  MgBufs<TS> m = sample_bufs(all, g, s);
  if (LDSC) {
    extern __shared__ char dyn_lds[];
    setup_lds_levels(g, m, (TS*)dyn_lds);
  }
  build_diagonals<TW, TS>(g, m, u);
  int lin = 0;
  bool ok_all = true;
  for (int k = 0; k < g.dz; ++k) {
    for_nodes(n, [&](int p, int i, int j) { b[p] = (TW)FT[(int64_t)k * g.nodes + p]; });
    __syncthreads();
    bool ok = true;
    int passes = 0;
    lin += dc_solve<TW, TS>(g, m, sp, em, u, b, x, red, &ok, &passes);
    ok_all = ok_all && ok;
    double* out = dudz + (s * g.dz + k) * du;
    for_nodes(n, [&](int p, int i, int j) {
      if (interior(i, j, n)) out[(int64_t)(j - 1) * (n - 1) + (i - 1)] = (double)x[p];
    });
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lin_out[s] = lin;
    if (!ok_all) flag_out[s] |= SAA_FLAG_DC;
  }
}

// Reduced control Jacobians by adjoints: J_r = Phi^T M A(u)^{-1} F = (A(u)^{-1}
// M Phi)^T F since A(u) is symmetric, so r_u solves with right-hand sides
// M phi_k replace the d_Z linearised ones (Sec. 3.4: the adjoint variant
// for d_Z >= r_U).  MPhiT: r_u x d_U (interior order); output
// JY[(s d_Z + kz) r_u + k] = f_kz^T lambda_k.  One block per sample.
template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_adjoint_jac(PdeGeo g, const double* FT, const double* em_all,
                                                        const TW* u_all, TW* b_all, TW* x_all, MgBufs<TS> all,
                                                        SolveParams sp, const double* MPhiT, int r_u, double* JY,
                                                        int* lin_out, int* flag_out, int64_t N) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  const int64_t s = blockIdx.x;
  if (s >= N) return;
  const int n = g.n[0];
  const int64_t du = (int64_t)(n - 1) * (n - 1);
  const double* em = em_all + s * g.nodes;
  const TW* u = u_all + s * g.nodes;
  TW* b = b_all + s * g.nodes;
  TW* x = x_all + s * g.nodes;
  MgBufs<TS> m = sample_bufs(all, g, s);
  if (LDSC) {
    extern __shared__ char dyn_lds[];
    setup_lds_levels(g, m, (TS*)dyn_lds);
  }
  build_diagonals<TW, TS>(g, m, u);
  int lin = 0;
  bool ok_all = true;
  for (int k = 0; k < r_u; ++k) {
    const double* rhs = MPhiT + (int64_t)k * du;
    for_nodes(n, [&](int p, int i, int j) {
      b[p] = interior(i, j, n) ? (TW)rhs[(int64_t)(j - 1) * (n - 1) + (i - 1)] : (TW)0;
    });
    __syncthreads();
    bool ok = true;
    int passes = 0;
    lin += dc_solve<TW, TS>(g, m, sp, em, u, b, x, red, &ok, &passes);
    ok_all = ok_all && ok;
    for (int k0 = 0; k0 < g.dz; k0 += 8) {   // f_kz^T lambda, eight controls per pass
      double v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = 0.0;
      for_nodes(n, [&](int p, int i, int j) {
        if (interior(i, j, n)) {
          const double l = (double)x[p];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (k0 + t < g.dz) v[t] += FT[(int64_t)(k0 + t) * g.nodes + p] * l;
        }
      });
      block_sum<8>(v, red);
      if (threadIdx.x == 0)
        for (int t = 0; t < 8 && k0 + t < g.dz; ++t) JY[(s * g.dz + k0 + t) * r_u + k] = v[t];
    }
  }
  if (threadIdx.x == 0) {
    lin_out[s] = lin;
    if (!ok_all) flag_out[s] |= SAA_FLAG_DC;
  }
}

// Copy interior node values to the dense interior-order layout (float64).
template <typename TW>
__global__ void saa_k_interior(const TW* u_all, double* out, int n, int64_t N) {
  const int64_t du = (int64_t)(n - 1) * (n - 1);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * du) return;
  const int64_t s = t / du;
  const int64_t r = t - s * du;
  const int j = (int)(r / (n - 1)) + 1, i = (int)(r % (n - 1)) + 1;
  out[t] = (double)u_all[s * (int64_t)(n + 1) * (n + 1) + (int64_t)j * (n + 1) + i];
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace saa_launch {

// Dynamic LDS for the coarse levels (6 arrays), or 0 when they stay in HBM:
// used for FP32 solver arrays when they fit next to the static reduction
// buffers in the 160 KB of a workgroup.
template <typename TS>
static size_t coarse_lds_bytes(const PdeGeo& g) {
  if (sizeof(TS) != 4 || g.L <= LF) return 0;
  const size_t b = 6 * (size_t)(g.lstride - g.off[LF]) * sizeof(TS);
  const size_t static_lds = (size_t)SAA_MAX_DZ * (BS / SAA_WAVE) * sizeof(double) + SAA_MAX_DZ * sizeof(double);
  return (b + static_lds <= 150 * 1024) ? b : 0;
}

static bool set_lds_attr(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

void sine_table(double* S, int K1, int n, hipStream_t st) {
  const int total = K1 * (n + 1);
  saa_k_sine_table<<<(total + 255) / 256, 256, 0, st>>>(S, K1, n);
}

void source_matrix(double* FT, int n, int s, double sigma, hipStream_t st) {
  const int64_t total = (int64_t)(n + 1) * (n + 1) * s * s;
  saa_k_source_matrix<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(FT, n, s, sigma);
}

void field(const double* xi, const double* S, const double* amp, double* em, int K1, int n, int64_t N,
           hipStream_t st) {
  // band of T rows: K1 * rows <= FIELD_BAND doubles (with K1 <= 64 the block
  // needs at most 48 KB of LDS)
  const int rows = std::max(1, std::min(n + 1, FIELD_BAND / K1));
  const size_t lds = sizeof(double) * ((size_t)K1 * K1 + (size_t)K1 * rows);
  saa_k_field<<<(unsigned)N, 256, lds, st>>>(xi, S, amp, em, K1, n, rows, N);
}

template <typename TS>
void hierarchy(const PdeGeo& g, const double* em, double* kap, int64_t kstride, int64_t chunk,
               const MgBufs<TS>& b, int64_t N, hipStream_t st) {
  for (int64_t s0 = 0; s0 < N; s0 += chunk) {
    const int64_t nb = (N - s0 < chunk) ? (N - s0) : chunk;
    saa_k_hierarchy<TS><<<(unsigned)nb, BS, 0, st>>>(g, em, kap, kstride, b, s0, N);
  }
}
template void hierarchy<float>(const PdeGeo&, const double*, double*, int64_t, int64_t, const MgBufs<float>&,
                               int64_t, hipStream_t);
template void hierarchy<double>(const PdeGeo&, const double*, double*, int64_t, int64_t,
                                const MgBufs<double>&, int64_t, hipStream_t);

template <typename TW, typename TS>
void state(const PdeGeo& g, const double* FT, const double* Z, int64_t z_stride, const double* em, TW* u, TW* f,
           const MgBufs<TS>& b, const SolveParams& sp, double* q, int* newton, int* lin, int* flag, int64_t N,
           hipStream_t st) {
  const size_t lds = coarse_lds_bytes<TS>(g);
  if (lds) {
    static bool attr = set_lds_attr((const void*)saa_k_state<TW, TS, true>, lds);
    (void)attr;
    saa_k_state<TW, TS, true><<<(unsigned)N, BS, lds, st>>>(g, FT, Z, z_stride, em, u, f, b, sp, q, newton, lin, flag, N);
  } else {
    saa_k_state<TW, TS, false><<<(unsigned)N, BS, 0, st>>>(g, FT, Z, z_stride, em, u, f, b, sp, q, newton, lin, flag, N);
  }
}

template <typename TW, typename TS>
void adjoint(const PdeGeo& g, const double* FT, const double* em, const TW* u, TW* bvec, TW* lam,
             const MgBufs<TS>& b, const SolveParams& sp, const double* q, const double* tstar, int act,
             double act_w, double* gout, int* lin, int* flag, int* did, int64_t N, hipStream_t st) {
  const size_t lds = coarse_lds_bytes<TS>(g);
  if (lds) {
    static bool attr = set_lds_attr((const void*)saa_k_adjoint<TW, TS, true>, lds);
    (void)attr;
    saa_k_adjoint<TW, TS, true><<<(unsigned)N, BS, lds, st>>>(g, FT, em, u, bvec, lam, b, sp, q, tstar, act, act_w,
                                                              gout, lin, flag, did, N);
  } else {
    saa_k_adjoint<TW, TS, false><<<(unsigned)N, BS, 0, st>>>(g, FT, em, u, bvec, lam, b, sp, q, tstar, act, act_w,
                                                               gout, lin, flag, did, N);
  }
}

template <typename TW, typename TS>
void linearized(const PdeGeo& g, const double* FT, const double* em, const TW* u, TW* bvec, TW* x,
                const MgBufs<TS>& b, const SolveParams& sp, double* dudz, int* lin, int* flag, int64_t N,
                hipStream_t st) {
  const size_t lds = coarse_lds_bytes<TS>(g);
  if (lds) {
    static bool attr = set_lds_attr((const void*)saa_k_linearized<TW, TS, true>, lds);
    (void)attr;
    saa_k_linearized<TW, TS, true><<<(unsigned)N, BS, lds, st>>>(g, FT, em, u, bvec, x, b, sp, dudz, lin, flag, N);
  } else {
    saa_k_linearized<TW, TS, false><<<(unsigned)N, BS, 0, st>>>(g, FT, em, u, bvec, x, b, sp, dudz, lin, flag, N);
  }
}

template <typename TW, typename TS>
void adjoint_jac(const PdeGeo& g, const double* FT, const double* em, const TW* u, TW* bvec, TW* x,
                 const MgBufs<TS>& b, const SolveParams& sp, const double* MPhiT, int r_u, double* JY, int* lin,
                 int* flag, int64_t N, hipStream_t st) {
  const size_t lds = coarse_lds_bytes<TS>(g);
  if (lds) {
    static bool attr = set_lds_attr((const void*)saa_k_adjoint_jac<TW, TS, true>, lds);
    (void)attr;
    saa_k_adjoint_jac<TW, TS, true><<<(unsigned)N, BS, lds, st>>>(g, FT, em, u, bvec, x, b, sp, MPhiT, r_u, JY, lin,
                                                                   flag, N);
  } else {
    saa_k_adjoint_jac<TW, TS, false><<<(unsigned)N, BS, 0, st>>>(g, FT, em, u, bvec, x, b, sp, MPhiT, r_u, JY, lin,
                                                                    flag, N);
  }
}

template <typename TW>
void interior_copy(const TW* u, double* out, int n, int64_t N, hipStream_t st) {
  const int64_t total = N * (int64_t)(n - 1) * (n - 1);
  saa_k_interior<TW><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(u, out, n, N);
}

template <typename TW, typename TS>
void state_multi(const StateJob<TW, TS>* jobs, int count, int64_t blocks, size_t lds, const SolveParams& sp,
                 hipStream_t st) {
  if (lds) {
    (void)set_lds_attr((const void*)saa_k_state_multi<TW, TS, true>, lds);
    saa_k_state_multi<TW, TS, true><<<(unsigned)blocks, BS, lds, st>>>(jobs, count, sp);
  } else {
    saa_k_state_multi<TW, TS, false><<<(unsigned)blocks, BS, 0, st>>>(jobs, count, sp);
  }
}

template <typename TW, typename TS>
void adjoint_multi(const AdjointJob<TW, TS>* jobs, int count, int64_t blocks, size_t lds, const SolveParams& sp,
                   int act, double act_w, hipStream_t st) {
  if (lds) {
    (void)set_lds_attr((const void*)saa_k_adjoint_multi<TW, TS, true>, lds);
    saa_k_adjoint_multi<TW, TS, true><<<(unsigned)blocks, BS, lds, st>>>(jobs, count, sp, act, act_w);
  } else {
    saa_k_adjoint_multi<TW, TS, false><<<(unsigned)blocks, BS, 0, st>>>(jobs, count, sp, act, act_w);
  }
}

template <typename TS>
size_t coarse_lds(const PdeGeo& g) {
  return coarse_lds_bytes<TS>(g);
}

#define SAA_INST(TW, TS)                                                                                         \
  template void state_multi<TW, TS>(const StateJob<TW, TS>*, int, int64_t, size_t, const SolveParams&,           \
                                    hipStream_t);                                                                \
  template void adjoint_multi<TW, TS>(const AdjointJob<TW, TS>*, int, int64_t, size_t, const SolveParams&, int,  \
                                      double, hipStream_t);                                                      \
  template void state<TW, TS>(const PdeGeo&, const double*, const double*, int64_t, const double*, TW*, TW*,     \
                              const MgBufs<TS>&, const SolveParams&, double*, int*, int*, int*, int64_t,         \
                              hipStream_t);                                                                      \
  template void adjoint<TW, TS>(const PdeGeo&, const double*, const double*, const TW*, TW*, TW*,                \
                                const MgBufs<TS>&, const SolveParams&, const double*, const double*, int,        \
                                double, double*, int*, int*, int*, int64_t, hipStream_t);                                \
  template void linearized<TW, TS>(const PdeGeo&, const double*, const double*, const TW*, TW*, TW*,             \
                                   const MgBufs<TS>&, const SolveParams&, double*, int*, int*, int64_t,          \
                                   hipStream_t);                                                                 \
  template void adjoint_jac<TW, TS>(const PdeGeo&, const double*, const double*, const TW*, TW*, TW*,            \
                                    const MgBufs<TS>&, const SolveParams&, const double*, int, double*, int*,    \
                                    int*, int64_t, hipStream_t);
SAA_INST(double, double)
SAA_INST(double, float)
SAA_INST(float, float)
#undef SAA_INST
template size_t coarse_lds<float>(const PdeGeo&);
template size_t coarse_lds<double>(const PdeGeo&);
template void interior_copy<double>(const double*, double*, int, int64_t, hipStream_t);
template void interior_copy<float>(const float*, double*, int, int64_t, hipStream_t);

}  // namespace saa_launch
