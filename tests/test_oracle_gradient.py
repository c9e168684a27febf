"""Pins of the oracle's adjoint gradient (no GPU): Taylor test of the full SAA
objective, central differences of per-sample q, and the control Jacobian
against differences of nonlinear solves."""
import numpy as np

from oracle import fem2d, saa
import saa_inputs as si


def _small(kl_amp=20.0):
    prob = fem2d.Problem2D(n=16, kl_per_dim=4, kl_amp=kl_amp)
    xi = si.kl_coefficients(11, 16, 4)
    z = si.control(12)
    return prob, xi, z


def test_taylor_second_order():
    prob, xi, z = _small()
    beta, eps, alpha = 0.8, 1e-4, 1e-3
    base = saa.objective_grad(prob, xi, z, beta, eps, alpha)
    d = np.random.default_rng(0).standard_normal(prob.d_z)
    hs = [1e-1 * 2.0 ** -k for k in range(6)]
    rem = []
    for h in hs:
        Jh = saa.objective_grad(prob, xi, z + h * d, beta, eps, alpha)["J"]
        rem.append(abs(Jh - base["J"] - h * base["grad"] @ d))
    slopes = np.diff(np.log(rem)) / np.diff(np.log(hs))
    assert np.all(slopes > 1.8), slopes


def test_per_sample_gradient_central_difference():
    prob, xi, z = _small()
    ops = fem2d.operators(prob)
    s = fem2d.solve_sample(ops, xi[0], z)
    h = 1e-5
    fd = np.empty(prob.d_z)
    for k in range(prob.d_z):
        e = np.zeros(prob.d_z)
        e[k] = h
        fd[k] = (fem2d.solve_sample(ops, xi[0], z + e, want_grad=False)["q"]
                 - fem2d.solve_sample(ops, xi[0], z - e, want_grad=False)["q"]) / (2 * h)
    np.testing.assert_allclose(s["g"], fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


def test_control_jacobian_matches_nonlinear_differences():
    prob, xi, z = _small()
    ops = fem2d.operators(prob)
    s = fem2d.solve_sample(ops, xi[1], z)
    J = fem2d.control_jacobian(ops, s)
    h = 1e-5
    for k in (0, 7, 24):
        e = np.zeros(prob.d_z)
        e[k] = h
        up = fem2d.solve_sample(ops, xi[1], z + e, want_grad=False)["u"]
        um = fem2d.solve_sample(ops, xi[1], z - e, want_grad=False)["u"]
        np.testing.assert_allclose(J[:, k], (up - um) / (2 * h), rtol=1e-7,
                                   atol=1e-7 * np.abs(J[:, k]).max())
    # chain rule: dq/dz = (dq/du)^T du/dz equals the adjoint gradient
    np.testing.assert_allclose(fem2d.qoi_gradient(ops, s["u"]) @ J, s["g"], rtol=1e-11)
