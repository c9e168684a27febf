"""Pins of the oracle's expectation-type risk measures (no GPU): relations
to the CVaR at beta = 0, numpy's variance, the exact failure fraction in the
eps -> 0 limit, and finite differences of J through a linear map q(z)."""
import numpy as np
import pytest

from oracle import cvar, risk


def _linear(seed, N=300, dz=6):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((N, dz))
    b = rng.standard_normal(N)
    return A, b, rng.standard_normal(dz)


def test_mean_is_cvar_at_beta_zero_shifted_by_half_eps():
    """With t* = min q - eps every sample sits on the linear branch of
    s_eps, so the smoothed CVaR_0 is E[Q] - eps/2 with the same gradient."""
    A, b, z = _linear(21)
    q, g = A @ z + b, A
    eps = 1e-3
    c = cvar.objective(q, g, z, 0.0, eps, 1e-3)
    m = risk.mean(q, g, z, 1e-3)
    assert abs(m["J"] - eps / 2 - c["J"]) <= 1e-12 * abs(c["J"])
    np.testing.assert_allclose(m["grad"], c["grad"], rtol=1e-12, atol=1e-14)


def test_mean_var_value_is_numpy_variance():
    A, b, z = _linear(22)
    q = A @ z + b
    r = risk.mean_var(q, A, z, 0.7, 0.0)
    assert abs(r["J"] - (np.mean(q) + 0.7 * np.var(q))) <= 1e-12 * abs(r["J"])


def test_pof_is_the_failure_fraction_away_from_the_threshold():
    A, b, z = _linear(23)
    q = A @ z + b
    tau = float(np.median(q)) + 1e-3
    gap = np.min(np.abs(q - tau))
    r = risk.pof(q, A, z, tau, 0.5 * gap, 0.0)
    assert r["J"] == np.mean(q > tau)
    assert np.all(r["grad"] == 0.0)


def test_bpoe_is_one_minus_beta_at_the_cvar():
    """bPOE_tau = 1 - beta where tau = CVaR_beta (Mafusalov-Uryasev), here
    with beta N integer (CVaR = mean of the top k samples) and a tiny eps."""
    A, b, z = _linear(25)
    q = A @ z + b
    for k in (7, 30, 120):
        tau = float(np.mean(np.sort(q)[-k:]))
        r = risk.bpoe(q, A, z, tau, 1e-10, 0.0)
        assert abs(r["J"] - k / len(q)) <= 1e-7, (k, r["J"])


def test_bpoe_limits():
    A, b, z = _linear(26)
    q = A @ z + b
    eps = 0.1
    r = risk.bpoe(q, A, z, float(np.mean(q)) - 0.1, eps, 0.0)      # tau below the mean: a* = 0
    assert r["t"] == 0.0 and abs(r["J"] - (1.0 - eps / 2)) <= 1e-15 and np.all(r["grad"] == 0.0)
    r = risk.bpoe(q, A, z, float(np.max(q)) + 1e-3, eps, 0.0)      # no exceedance: a* = inf, 0
    assert r["t"] == float("inf") and r["J"] == 0.0


@pytest.mark.parametrize("which", ["mean", "mean_var", "pof", "bpoe"])
def test_gradients_match_finite_differences(which):
    A, b, z = _linear(24)
    tau = float(np.median(A @ z + b))

    def J(zz):
        q = A @ zz + b
        if which == "mean":
            return risk.mean(q, A, zz, 0.3)
        if which == "mean_var":
            return risk.mean_var(q, A, zz, 0.8, 0.3)
        if which == "bpoe":
            return risk.bpoe(q, A, zz, tau + 1.0, 0.5, 0.3)
        return risk.pof(q, A, zz, tau, 2.0, 0.3)
    g = J(z)["grad"]
    h = 1e-6
    fd = np.array([(J(z + h * e)["J"] - J(z - h * e)["J"]) / (2 * h) for e in np.eye(len(z))])
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)
