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
  bpoe       buffered probability of exceedance (Mafusalov and Uryasev):
             rho = min_{a >= 0} E[(a (Q - tau) + 1)^+], the plus function
             smoothed with s_eps; a* from scipy's brentq on the derivative
             in a; by the envelope theorem d/dz = E[a* s_eps'(.) dQ/dz].
"""
from __future__ import annotations

import numpy as np

from scipy.optimize import brentq

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


def bpoe(q, g, z, tau, eps, alpha):
    x = q - tau
    reg = 0.5 * alpha * z @ z
    if np.max(q) <= tau:
        return {"J": float(reg), "grad": alpha * z, "t": float("inf")}

    def dphi(a):
        return np.mean(cvar.dsplus(a * x + 1.0, eps) * x)
    if dphi(0.0) >= 0.0:
        a = 0.0
    else:
        hi = 1.0 / (np.max(q) - tau)
        while dphi(hi) <= 0.0:
            hi *= 4.0
        a = brentq(dphi, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=1000)
    y = a * x + 1.0
    return {"J": float(np.mean(cvar.splus(y, eps)) + reg),
            "grad": np.mean((a * cvar.dsplus(y, eps))[:, None] * g, axis=0) + alpha * z, "t": float(a)}
