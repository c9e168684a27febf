// Data structures of the 3D PDE form (Q1 hexahedra on the unit cube) shared
// by the HIP kernels and the host runtime.
#pragma once
#include <stdint.h>

#include "pde.h"

// Multigrid geometry of one sample.  Level l has n[l] cells per side; every
// per-level array stores the full (n_l+1)^3 node grid (x fastest, boundary
// entries zero) and the levels of one sample are stacked at off[l] inside a
// block of lstride elements.  Per-element arrays use the same layout: element
// (i, j, k) (cells [i, i+1] x [j, j+1] x [k, k+1]) sits at the index of its
// lowest corner node; entries with i, j or k equal to n_l are zero.
struct Pde3Geo {
  int L;                        // number of levels
  int n[SAA_MAX_LEVELS];
  int64_t off[SAA_MAX_LEVELS];
  int64_t lstride;
  int64_t nodes;                // (n_0 + 1)^3
  int dz;                       // s^3 controls
  int s;                        // sources per dimension
  double h;                     // fine mesh size 1/n_0
  double r;                     // reaction coefficient
  double src_c;                 // h^3 / (sigma sqrt(2 pi)): lumped weight times the source prefactor
  const double* G;              // s x (n_0+1): exp(-(i h - c_a)^2 / (2 sigma^2)), c_a = (a+1)/(s+1)
  const double* mt;             // (M u_target) at interior nodes, 0 elsewhere (node layout)
  double ctt;                   // u_target^T M u_target over all nodes
};

// Per-sample multigrid / CG workspaces in the solver precision TS.
template <typename TS>
struct Mg3Bufs {
  TS* E;   // element kappa per level (fine: vertex mean of exp(m); coarse: mean of the 8 children)
  TS* KD;  // stiffness diagonal (h_l / 3) x sum of the 8 incident element kappas
  TS* D;   // operator diagonal: KD + lumped reaction (restricted on coarse levels)
  TS* X;   // V-cycle iterate per level
  TS* B;   // V-cycle right-hand side per level (level 0: second CG direction buffer)
  TS* T;   // V-cycle residual / output per level (level 0: the preconditioned residual z)
  TS* cx;  // CG solution
  TS* cr;  // CG residual
  TS* cp;  // CG direction
  TS* cq;  // A p
};

// One 3D problem of a mixed-dimension launch (state and adjoint): sample s of
// the job runs in workgroup first + s.
template <typename TW, typename TS>
struct State3Job {
  Pde3Geo g;
  const double* Z;    // the problem's control (shared by its samples)
  const double* k64;  // fine element kappas (FP64), per sample
  TW* u;
  TW* f;
  Mg3Bufs<TS> b;
  double* q;
  int* newton;
  int* lin;
  int* flag;
  int64_t N;
  int64_t first;
};

template <typename TW, typename TS>
struct Adjoint3Job {
  Pde3Geo g;
  const double* k64;
  const TW* u;
  TW* bvec;
  TW* lam;
  Mg3Bufs<TS> b;
  const double* q;
  const double* tstar;
  double* gout;
  int* lin;
  int* flag;
  int* did;
  int64_t N;
  int64_t first;
};
