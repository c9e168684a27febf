"""Outer OUU solve (Sec. 2.1, eq. (ouu); Sec. 4.2 minimises over the box
Z_ad with L-BFGS-B).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The minimiser is scipy's L-BFGS-B, used as a library primitive on an oracle
objective (PDE form from oracle.saa, surrogate form from oracle.surrogate);
`projected_gradient` is the first-order optimality measure of the box
problem: P(z - grad) - z, zero exactly at a KKT point.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def projected_gradient(z, g, lb, ub):
    return np.clip(z - g, lb, ub) - z


def solve(fun_grad, z0, lb, ub, pgtol=1e-10, ftol=1e-15, maxiter=1000, memory=10):
    """argmin of fun_grad (z -> (J, grad)) over [lb, ub]; returns (z, J, nfev)."""
    lb = np.broadcast_to(np.asarray(lb, float), np.shape(z0))
    ub = np.broadcast_to(np.asarray(ub, float), np.shape(z0))
    res = minimize(fun_grad, np.clip(z0, lb, ub), jac=True, method="L-BFGS-B", bounds=list(zip(lb, ub)),
                   options=dict(gtol=pgtol, ftol=ftol, maxiter=maxiter, maxcor=memory, maxfun=10 * maxiter))
    return res.x, float(res.fun), int(res.nfev)
