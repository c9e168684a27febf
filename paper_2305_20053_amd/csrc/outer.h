// Stopping control of the outer iterations (Newton and defect correction)
// of the PDE-form kernels, shared by the 2D and 3D solvers.
#pragma once
#include <hip/hip_runtime.h>

// Control of the outer iterations (Newton and defect correction).  After an
// update delta_k of the iterate x (squared norms d2 = |delta_k|^2,
// x2 = |x|^2) the iteration has converged when
//  * |delta_k| <= tol |x|, or
//  * the error left after this update, predicted from the contraction seen
//    between the last two updates, |delta_k|^2 / |delta_{k-1}| <= tol |x|, or
//  * the updates stopped contracting below 1e-4 |x| (rounding floor of the
//    state precision).
// Otherwise the next inner solve only needs to shrink the predicted error to
// tol |x|, so its relative tolerance is 0.1 tol |x| / predicted, kept within
// [lin_rtol, 0.1].
struct OuterCtl {
  double prev2 = INFINITY;
  double eta;
};

__device__ __forceinline__ bool outer_converged(OuterCtl& c, double d2, double x2, double tol, double lin_rtol) {
  bool done = d2 <= tol * tol * x2 || (d2 <= 1e-8 * x2 && d2 > 0.0625 * c.prev2);
  double eta = lin_rtol;
  if (!done && c.prev2 < INFINITY && d2 > 0.0) {
    // predicted^2 = d2^2 / prev2
    done = d2 * d2 <= tol * tol * x2 * c.prev2;
    const double e = 0.1 * tol * sqrt(x2 * c.prev2) / d2;
    eta = fmin(0.1, fmax(lin_rtol, e));
  }
  c.prev2 = d2;
  c.eta = eta;
  return done;
}
