"""Pins of the oracle's smoothed-CVaR reduction (no GPU)."""
import json
import os

import numpy as np
import pytest

from oracle import cvar

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cvar_cases.json")


def _cases():
    with open(GOLDEN) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", _cases())
def test_brute_force_and_golden(case):
    q = np.array(case["q"], dtype=float)
    beta = case["beta"]
    assert abs(cvar.cvar_tail_mean(q, beta) - case["cvar"]) < 1e-14
    assert abs(cvar.cvar_ru_bruteforce(q, beta) - case["cvar"]) < 1e-14
    # smoothed value within the eps bound: x+ - eps/2 <= s_eps(x) <= x+
    eps = 1e-4
    out = cvar.objective(q, np.zeros((q.size, 1)), np.zeros(1), beta, eps, 0.0)
    assert case["cvar"] - eps / (2 * (1 - beta)) - 1e-14 <= out["J"] <= case["cvar"] + 1e-14


def test_splus_closed_forms():
    eps = 1e-4
    assert cvar.splus(0.0, eps) == 0.0 and cvar.dsplus(0.0, eps) == 0.0
    assert abs(cvar.splus(eps, eps) - eps / 2) < 1e-20
    assert abs(cvar.dsplus(eps, eps) - 1.0) < 1e-15
    assert cvar.d2splus(0.0, eps) == 0.0 and abs(cvar.d2splus(eps * (1 - 1e-12), eps)) < 1e-6 / eps
    # both derivatives are the derivatives of the value (central differences)
    x = np.linspace(-0.5 * eps, 1.5 * eps, 41)
    d = 1e-9 * eps
    np.testing.assert_allclose((cvar.splus(x + d, eps) - cvar.splus(x - d, eps)) / (2 * d),
                               cvar.dsplus(x, eps), atol=1e-6)
    np.testing.assert_allclose((cvar.dsplus(x + d, eps) - cvar.dsplus(x - d, eps)) / (2 * d),
                               cvar.d2splus(x, eps), atol=1e-6 / eps)
    # the quartic joins continuously with value, slope and curvature (C^2)
    for x0, v, s in [(0.0, 0.0, 0.0), (eps, eps / 2, 1.0)]:
        lo, hi = x0 - 1e-12 * eps, x0 + 1e-12 * eps
        assert abs(cvar.splus(lo, eps) - cvar.splus(hi, eps)) < 1e-15
        assert abs(cvar.dsplus(lo, eps) - cvar.dsplus(hi, eps)) < 1e-10
        assert abs(cvar.d2splus(lo, eps) - cvar.d2splus(hi, eps)) < 1e-6 / eps


def test_beta_zero_is_mean_minus_half_eps():
    q = np.random.default_rng(1).uniform(0, 1, 257)
    out = cvar.objective(q, np.zeros((q.size, 1)), np.zeros(1), 0.0, 1e-4, 0.0)
    assert abs(out["J"] - (q.mean() - 0.5e-4)) < 1e-15


@pytest.mark.parametrize("n,beta", [(64, 0.95), (256, 0.95), (1024, 0.9), (1000, 0.99)])
def test_tstar_optimality_and_weights(n, beta):
    rng = np.random.default_rng(n)
    q = 0.18 + 1e-3 * rng.standard_normal(n)
    eps = 1e-4
    t = cvar.t_star(q, beta, eps)
    target = n * (1 - beta)
    # dJ/dt = 0 at t*: sum s' = N (1 - beta), so the weights sum to one
    assert abs(np.sum(cvar.dsplus(q - t, eps)) - target) < 1e-9 * target
    out = cvar.objective(q, rng.standard_normal((n, 3)), np.zeros(3), beta, eps, 0.0)
    assert abs(out["w"].sum() - 1.0) < 1e-12
    assert np.all(out["w"] >= 0)
    # J is the minimum over t: a grid of nearby t never does better
    def jt(tt):
        return tt + np.sum(cvar.splus(q - tt, eps)) / target
    grid = t + np.linspace(-5 * eps, 5 * eps, 201)
    assert all(jt(tt) >= out["J"] - 1e-15 for tt in grid)
    # smoothed CVaR within eps/(2(1-beta)) of the exact empirical CVaR
    exact = cvar.cvar_tail_mean(q, beta)
    assert exact - eps / (2 * (1 - beta)) - 1e-14 <= out["J"] <= exact + 1e-14


def test_joint_mode_matches_minimised_mode_at_tstar():
    rng = np.random.default_rng(7)
    q = rng.uniform(0, 1, 100)
    g = rng.standard_normal((100, 4))
    z = rng.uniform(0, 1, 4)
    a = cvar.objective(q, g, z, 0.9, 1e-4, 1e-3)
    b = cvar.objective(q, g, z, 0.9, 1e-4, 1e-3, t_mode=1, t_in=a["t"])
    assert abs(a["J"] - b["J"]) < 1e-15
    np.testing.assert_allclose(a["grad"], b["grad"], rtol=1e-15, atol=1e-18)
    assert abs(b["dJdt"]) < 1e-9
    # away from t*, dJ/dt matches a central difference of J in t
    t1 = a["t"] + 3e-5
    c = cvar.objective(q, g, z, 0.9, 1e-4, 1e-3, t_mode=1, t_in=t1)
    d = 1e-8
    jp = cvar.objective(q, g, z, 0.9, 1e-4, 1e-3, t_mode=1, t_in=t1 + d)["J"]
    jm = cvar.objective(q, g, z, 0.9, 1e-4, 1e-3, t_mode=1, t_in=t1 - d)["J"]
    assert abs((jp - jm) / (2 * d) - c["dJdt"]) < 1e-6
