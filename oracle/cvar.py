"""Smoothed CVaR by sample average approximation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper Sec. 2.1-2.2: the Rockafellar-Uryasev form (eq. (CVaR_ouu))
    J(z, t) = t + 1/(1-beta) E[(Q - t)^+] + P(z)
with (x)^+ replaced by the C^2 piecewise quartic (x)^+_eps, and the SAA
version eq. (CVaR_saa_ouu)
    J_hat(z, t) = t + 1/(N (1-beta)) sum_i (q_i - t)^+_eps + P(z).
Reading taken here: t is minimised out for a given z (the RU minimum), so
J(z) = J_hat(z, t*), and by the envelope theorem
    grad J(z) = sum_i w_i g_i + alpha z,  w_i = s'_eps(q_i - t*) / (N (1-beta)),
which is the chain rule of eq. (ouu_risk_gradient) with f = s_eps.
"""
from __future__ import annotations

import numpy as np


def splus(x, eps):
    """(x)^+_eps: 0 (x <= 0); x^3/eps^2 - x^4/(2 eps^3) (0 < x < eps); x - eps/2 (x >= eps)."""
    x = np.asarray(x, dtype=np.float64)
    mid = x ** 3 / eps ** 2 - x ** 4 / (2.0 * eps ** 3)
    return np.where(x <= 0.0, 0.0, np.where(x >= eps, x - 0.5 * eps, mid))


def dsplus(x, eps):
    """d/dx (x)^+_eps: 0; 3x^2/eps^2 - 2x^3/eps^3; 1."""
    x = np.asarray(x, dtype=np.float64)
    mid = 3.0 * x ** 2 / eps ** 2 - 2.0 * x ** 3 / eps ** 3
    return np.where(x <= 0.0, 0.0, np.where(x >= eps, 1.0, mid))


def d2splus(x, eps):
    """d^2/dx^2 (x)^+_eps: 0; 6x/eps^2 - 6x^2/eps^3; 0."""
    x = np.asarray(x, dtype=np.float64)
    mid = 6.0 * x / eps ** 2 - 6.0 * x ** 2 / eps ** 3
    return np.where((x <= 0.0) | (x >= eps), 0.0, mid)


def t_star(q, beta, eps):
    """Minimiser of t -> t + sum_i s_eps(q_i - t) / (N (1-beta)).

    The optimality condition is Phi(t) = sum_i s'_eps(q_i - t) = N (1-beta).
    Phi is continuous and non-increasing, Phi(min q - eps) = N and
    Phi(max q) = 0, so bisection on [min q - eps, max q] brackets a root; it
    runs until the midpoint no longer moves, then one Newton step is taken if
    it stays inside the final bracket.
    """
    q = np.asarray(q, dtype=np.float64)
    n = q.size
    target = n * (1.0 - beta)
    lo = float(q.min()) - eps
    hi = float(q.max())

    def phi(t):
        return float(np.sum(dsplus(q - t, eps)))

    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if phi(mid) > target:
            lo = mid
        else:
            hi = mid
    t = 0.5 * (lo + hi)
    slope = -float(np.sum(d2splus(q - t, eps)))
    if slope < 0.0:
        t_new = t - (phi(t) - target) / slope
        if lo <= t_new <= hi:
            t = t_new
    return t


def objective(q, g, z, beta, eps, alpha, t_mode=0, t_in=0.0):
    """SAA smoothed CVaR objective and gradient.

    q: (N,), g: (N, d_Z) per-sample dq/dz, z: (d_Z,).
    t_mode 0: t minimised out; t_mode 1: evaluate at the given t_in (joint
    (z, t) form) and also return dJ/dt = 1 - sum s'/(N (1-beta)).
    Returns dict(J, grad, t, dJdt, w).
    """
    q = np.asarray(q, dtype=np.float64)
    n = q.size
    scale = 1.0 / (n * (1.0 - beta))
    t = t_star(q, beta, eps) if t_mode == 0 else float(t_in)
    w = dsplus(q - t, eps) * scale
    J = t + scale * float(np.sum(splus(q - t, eps))) + 0.5 * alpha * float(z @ z)
    grad = w @ g + alpha * z
    dJdt = 1.0 - float(np.sum(w))
    return {"J": J, "grad": grad, "t": t, "dJdt": dJdt, "w": w}


def cvar_tail_mean(q, beta):
    """Exact CVaR of the empirical law: mean of the upper (1-beta) tail, with
    the atom at the quantile taken fractionally.  k = N (1-beta) samples."""
    qs = np.sort(np.asarray(q, dtype=np.float64))[::-1]
    k = qs.size * (1.0 - beta)
    kf = int(np.floor(k))
    total = qs[:kf].sum()
    if k > kf:
        total += (k - kf) * qs[kf]
    return total / k


def cvar_ru_bruteforce(q, beta):
    """min over t in {q_i} of t + sum (q_i - t)^+ / (N (1-beta)); the RU
    objective is piecewise linear and convex in t with kinks at the q_i."""
    q = np.asarray(q, dtype=np.float64)
    scale = 1.0 / (q.size * (1.0 - beta))
    return min(t + scale * np.maximum(q - t, 0.0).sum() for t in q)
