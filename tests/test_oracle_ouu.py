"""Pins of the oracle's outer OUU solve (no GPU): the box-constrained
minimiser against closed forms and brute-force KKT enumeration, and first-
order optimality of a small PDE-form OUU solution under the oracle gradient
(itself pinned by finite differences in test_oracle_gradient)."""
import itertools

import numpy as np

import saa_inputs as si
from oracle import fem2d, ouu, saa as osaa


def test_separable_quadratic_is_clipped_centre():
    rng = np.random.default_rng(11)
    a = rng.uniform(0.5, 3.0, 8)
    c = rng.uniform(-3.0, 3.0, 8)
    lb, ub = -1.0, 1.5
    z, J, _ = ouu.solve(lambda z: (0.5 * np.sum(a * (z - c) ** 2), a * (z - c)), np.zeros(8), lb, ub)
    np.testing.assert_allclose(z, np.clip(c, lb, ub), atol=1e-9)


def _kkt_bruteforce(A, b, lb, ub):
    """min 1/2 z^T A z - b^T z on a box: enumerate every free / lower / upper
    assignment, solve the free block, keep the feasible KKT point."""
    n = len(b)
    for assign in itertools.product((0, 1, 2), repeat=n):
        z = np.where(np.array(assign) == 1, lb, np.where(np.array(assign) == 2, ub, 0.0))
        F = np.array(assign) == 0
        if F.any():
            z[F] = np.linalg.solve(A[np.ix_(F, F)], b[F] - A[np.ix_(F, ~F)] @ z[~F])
        if np.any(z < lb - 1e-12) or np.any(z > ub + 1e-12):
            continue
        g = A @ z - b
        ok = np.all(np.abs(g[F]) <= 1e-9) and np.all(g[np.array(assign) == 1] >= -1e-12) and \
            np.all(g[np.array(assign) == 2] <= 1e-12)
        if ok:
            return z
    raise AssertionError("no KKT point")


def test_coupled_quadratic_matches_kkt_enumeration():
    rng = np.random.default_rng(12)
    for trial in range(5):
        B = rng.standard_normal((5, 5))
        A = B @ B.T + 0.5 * np.eye(5)
        b = 3.0 * rng.standard_normal(5)
        lb, ub = -np.ones(5), np.full(5, 0.7)
        z_ref = _kkt_bruteforce(A, b, lb, ub)
        z, J, _ = ouu.solve(lambda z: (0.5 * z @ A @ z - b @ z, A @ z - b), np.zeros(5), lb, ub)
        np.testing.assert_allclose(z, z_ref, atol=1e-8)
        assert np.abs(ouu.projected_gradient(z, A @ z - b, lb, ub)).max() <= 1e-7


def test_pde_form_solution_is_a_local_minimum():
    """n = 16, 8 samples, box [-1.5, 1.5]^25: projected gradient ~ 0 and no
    feasible random perturbation lowers J."""
    prob = fem2d.Problem2D(n=16, kl_per_dim=4, target=fem2d.TARGET_SIN)
    xi = si.kl_coefficients(si.SEED_XI_SMALL, 8, 4)

    def fg(z):
        r = osaa.objective_grad(prob, xi, z)
        return r["J"], r["grad"]
    lb, ub = -1.5, 1.5
    z, J, _ = ouu.solve(fg, np.full(25, 0.5), lb, ub, pgtol=1e-9)
    g = fg(z)[1]
    assert np.abs(ouu.projected_gradient(z, g, lb, ub)).max() <= 1e-8
    assert 0 < np.sum((z <= lb) | (z >= ub)) < 25          # some bounds active, some not
    rng = np.random.default_rng(13)
    for _ in range(6):
        zp = np.clip(z + 1e-2 * rng.standard_normal(25), lb, ub)
        assert fg(zp)[0] >= J - 1e-14
