// PDE-form data structures shared by the HIP kernels and the host runtime.
#pragma once
#include <stdint.h>

#define SAA_MAX_LEVELS 12
#define SAA_MAX_DZ 64

// Multigrid level geometry of one sample.  Level 0 is the fine grid with n
// cells per side; level l has n >> l cells.  Every per-level array stores the
// full (n_l+1)^2 node grid (boundary entries stay zero), and the levels of
// one sample are stacked at offsets off[l] inside a block of `lstride`
// elements.
struct PdeGeo {
  int L;                        // number of levels (coarsest has 1 unknown)
  int n[SAA_MAX_LEVELS];        // cells per side
  int64_t off[SAA_MAX_LEVELS];  // element offset of level l inside a sample block
  int64_t lstride;              // elements per sample of level-stacked arrays
  int64_t nodes;                // (n_0 + 1)^2
  int dz;                       // number of controls
  double h2;                    // h^2 = lumped P1 weight of an interior node
  double r;                     // reaction coefficient
  const double* mt;             // (M u_target) at interior nodes, 0 on the boundary (node layout)
  double ctt;                   // u_target^T M u_target over all nodes
  // The lumped source matrix is separable: F[p][s b + a] = src_c G[a][i] G[b][j]
  // at interior node p = (i, j), with G[a][i] = exp(-(i h - (a + 1) / (s + 1))^2
  // / (2 sigma^2)) stored in src1 (s x (n_0 + 1)) and src_c = h^2 / (sigma sqrt(2 pi)).
  const double* src1;
  int src_s;
  double src_c;
};

// Per-sample multigrid / CG workspaces in the solver precision TS.
template <typename TS>
struct MgBufs {
  TS* WE;  // edge weight of (i,j)-(i+1,j), level-stacked
  TS* WN;  // edge weight of (i,j)-(i,j+1), level-stacked
  TS* KD;  // stiffness diagonal (sum of the four incident edge weights)
  TS* D;   // operator diagonal: KD + lumped reaction 3 r h^2 u^2 (restricted)
  TS* X;   // V-cycle iterate per level (level 0 = preconditioned residual z)
  TS* B;   // V-cycle right-hand side per level (level 0 unused)
  TS* T;   // V-cycle residual / reaction scratch per level
  TS* cx;  // CG solution (fine grid)
  TS* cr;  // CG residual
  TS* cp;  // CG search direction
  TS* cq;  // A p
  // LDS copies of the coarse levels (1..L-1) of WE, WN, D, X, B, T, stacked
  // like the global arrays from off[1] on; null when the coarse levels live
  // in HBM.
  TS* lWE = nullptr;
  TS* lWN = nullptr;
  TS* lD = nullptr;
  TS* lX = nullptr;
  TS* lB = nullptr;
  TS* lT = nullptr;
};

// Solver controls passed to the persistent kernels.
struct SolveParams {
  double newton_tol;  // stop when |update| <= newton_tol |iterate|
  double adj_tol;     // same for the adjoint / linearised defect corrections
  double lin_rtol;    // inner PCG relative residual
  int max_newton;
  int max_lin;
  int max_dc;
  int nu;             // red-black smoothing sweeps before and after each coarse correction
};

// Solver statistics reduced over the samples by the CVaR kernel.
struct CvarStats {
  int newton_max;
  int n_unconverged;
  int n_adjoints;
  int pad;
  long long lin_state;
  long long lin_adjoint;
  long long newton_total;
};

// Per-sample status flags.
enum { SAA_FLAG_NEWTON = 1, SAA_FLAG_CG = 2, SAA_FLAG_DC = 4, SAA_FLAG_NAN = 8 };

// One problem of a multi-size launch (several 2D contexts in one grid):
// blocks [first, first + N) of the launch solve its samples 0 .. N-1.
#define SAA_MAX_JOBS 4
template <typename TW, typename TS>
struct StateJob {
  PdeGeo g;
  const double* FT;
  const double* Z;    // the problem's control (shared by its samples)
  const double* em;
  TW* u;
  TW* f;
  MgBufs<TS> b;
  double* q;
  int* newton;
  int* lin;
  int* flag;
  int64_t N;
  int64_t first;
};

template <typename TW, typename TS>
struct AdjointJob {
  PdeGeo g;
  const double* FT;
  const double* em;
  const TW* u;
  TW* bvec;
  TW* lam;
  MgBufs<TS> b;
  const double* q;
  const double* tstar;
  double* gout;
  int* lin;
  int* flag;
  int* did;
  int64_t N;
  int64_t first;
};
