"""Expectation-type risk measures and their SAA estimators (Sec. 2.1: the
framework covers any risk measure written through expectations of functions
of Q, such as moments and probabilities of failure; Sec. 2.2: SAA).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Each function takes the per-sample q_i = Q(u(m_i, z)) and g_i = dq_i/dz and
returns J = rho_hat(z) + alpha/2 |z|^2 with its gradient, written from the
definitions:
  mean       rho = E[Q]                                   (eq. (saa))
  mean_var   rho = E[Q] + kappa Var[Q]  (Var with 1/N); d Var / dz =
             (2/N) sum_i (q_i - mean q)(g_i - mean g)
  pof        rho = P[Q > tau] smoothed as E[H_eps(Q - tau)], H_eps = the
             derivative of the C^2 plus-function smoothing (a C^1 step
             rising over [0, eps]); d/dz = E[H_eps'(Q - tau) dQ/dz].
"""
from __future__ import annotations

import numpy as np

from . import cvar


def mean(q, g, z, alpha):
    return {"J": float(np.mean(q) + 0.5 * alpha * z @ z), "grad": np.mean(g, axis=0) + alpha * z,
            "t": 0.0}


def mean_var(q, g, z, kappa, alpha):
    m = np.mean(q)
    dq = q - m
    var = np.mean(dq * dq)
    dvar = 2.0 * np.mean(dq[:, None] * (g - np.mean(g, axis=0)), axis=0)
    return {"J": float(m + kappa * var + 0.5 * alpha * z @ z),
            "grad": np.mean(g, axis=0) + kappa * dvar + alpha * z, "t": float(m)}


def pof(q, g, z, tau, eps, alpha):
    x = q - tau
    return {"J": float(np.mean(cvar.dsplus(x, eps)) + 0.5 * alpha * z @ z),
            "grad": np.mean(cvar.d2splus(x, eps)[:, None] * g, axis=0) + alpha * z, "t": float(tau)}
