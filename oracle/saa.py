"""SAA objective and gradient of the PDE form (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For fixed samples m_i (Sec. 2.2: fixed samples make the SAA problem
deterministic) each sample needs one Newton state solve and one adjoint solve
(Sec. 2.3); the per-sample (q_i, g_i) feed the smoothed-CVaR reduction of
oracle.cvar.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import cvar, fem2d, fem3d


def _fem(prob):
    """The finite-element module of a problem: Q1 on the cube or P1 on the square."""
    return fem3d if isinstance(prob, fem3d.Problem3D) else fem2d


def per_sample(prob, xi: np.ndarray, z: np.ndarray, ops=None, rtol=1e-14):
    """q (N,) and g (N, d_Z) for samples xi (N, K1, K1[, K1]) at control z."""
    fem = _fem(prob)
    ops = ops if ops is not None else fem.operators(prob)
    n_s = xi.shape[0]
    q = np.empty(n_s)
    g = np.empty((n_s, prob.d_z))
    for i in range(n_s):
        s = fem.solve_sample(ops, xi[i], z, rtol=rtol)
        q[i] = s["q"]
        g[i] = s["g"]
    return q, g


def _worker(args):
    prob, xi_chunk, z = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    return per_sample(prob, xi_chunk, z)


def per_sample_parallel(prob, xi, z, workers=None):
    """Same as per_sample, one worker process per core over samples."""
    workers = workers or os.cpu_count() or 1
    chunks = np.array_split(xi, min(workers, xi.shape[0]))
    with ProcessPoolExecutor(max_workers=len(chunks)) as ex:
        parts = list(ex.map(_worker, [(prob, c, z) for c in chunks]))
    return (np.concatenate([p[0] for p in parts]),
            np.concatenate([p[1] for p in parts]))


def objective_grad(prob, xi, z, beta=0.95, eps=1e-4, alpha=1e-3, t_mode=0, t_in=0.0,
                   workers=1):
    """J(z), grad J(z), t* and the per-sample q, g (Sec. 2.2, eq. (CVaR_saa_ouu))."""
    if workers == 1:
        q, g = per_sample(prob, xi, z)
    else:
        q, g = per_sample_parallel(prob, xi, z, workers)
    out = cvar.objective(q, g, z, beta, eps, alpha, t_mode=t_mode, t_in=t_in)
    out["q"] = q
    out["g"] = g
    return out
