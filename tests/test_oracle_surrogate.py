"""Pins of the oracle's surrogate, POD and training pieces (no GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem2d, surrogate, training
import saa_inputs as si


@pytest.fixture(scope="module")
def small_pod():
    """States of a 16 x 16 problem at random (m, z), POD of rank 8."""
    prob = fem2d.Problem2D(n=16, kl_per_dim=4, kl_amp=20.0)
    ops = fem2d.operators(prob)
    xi = si.kl_coefficients(31, 40, 4)
    Z = si.controls(32, 40)
    samples = [fem2d.solve_sample(ops, xi[i], Z[i], want_grad=True) for i in range(40)]
    U = np.stack([s["u"] for s in samples])
    ubar, Phi, lam = training.pod(U, ops.M, 8)
    return prob, ops, xi, Z, samples, U, ubar, Phi, lam


def test_pod_orthonormal_and_truncation_identity(small_pod):
    prob, ops, xi, Z, samples, U, ubar, Phi, lam = small_pod
    np.testing.assert_allclose(Phi.T @ (ops.M @ Phi), np.eye(8), atol=1e-12)
    # sum_i ||d_i - Phi Phi^T M d_i||_M^2 = sum of the trailing eigenvalues
    D = U - ubar
    R = D - (D @ (ops.M @ Phi)) @ Phi.T
    err = np.einsum("ij,ij->", R, (ops.M @ R.T).T)
    assert abs(err - lam[8:].sum()) <= 1e-10 * lam.sum()
    assert np.all(np.diff(lam) <= 1e-15 * lam[0])


def test_reduced_qoi_equals_full_decode(small_pod):
    prob, ops, xi, Z, samples, U, ubar, Phi, lam = small_pod
    c = Phi.T @ (ops.M_full @ (fem2d.extend(ops, ubar) - ops.t_full))[ops.interior]
    c0 = fem2d.qoi(ops, ubar) - c @ c
    phi = np.random.default_rng(2).standard_normal((5, 8)) * 0.01
    q_red = surrogate.reduced_qoi(phi, c, c0)
    q_full = [fem2d.qoi(ops, surrogate.decode(Phi, ubar, p)) for p in phi]
    np.testing.assert_allclose(q_red, q_full, rtol=1e-13)


def _net(seed, r_m, d_z, r_u, width=16, depth=4):
    return si.random_mlp(seed, [r_m + d_z] + [width] * depth + [r_u])


def test_vjp_and_jvp_against_central_differences():
    r_m, d_z, r_u = 6, 3, 5
    layers = _net(3, r_m, d_z, r_u)
    rng = np.random.default_rng(4)
    model = surrogate.Surrogate(layers, r_m, d_z, rng.standard_normal(r_u), 0.3)
    xhat = rng.standard_normal((4, r_m))
    z = rng.uniform(0, 1, d_z)
    q, g = surrogate.qoi_and_grad(model, xhat, z)
    x = np.concatenate([xhat, np.broadcast_to(z, (4, d_z))], axis=1)
    phi, jphi = surrogate.jacobian_z(layers, x, r_m)
    h = 1e-6
    for k in range(d_z):
        e = np.zeros(d_z)
        e[k] = h
        qp, _ = surrogate.qoi_and_grad(model, xhat, z + e)
        qm, _ = surrogate.qoi_and_grad(model, xhat, z - e)
        np.testing.assert_allclose(g[:, k], (qp - qm) / (2 * h), rtol=1e-6, atol=1e-9)
        xp = x.copy(); xp[:, r_m + k] += h
        xm = x.copy(); xm[:, r_m + k] -= h
        fd = (surrogate.forward(layers, xp)[0] - surrogate.forward(layers, xm)[0]) / (2 * h)
        np.testing.assert_allclose(jphi[:, :, k], fd, rtol=1e-7, atol=1e-10)
    # VJP equals the JVP contracted with dq/dphi = 2 (phi + c)
    np.testing.assert_allclose(g, np.einsum("bo,bok->bk", 2 * (phi + model.c), jphi), rtol=1e-12)


def test_gelu_derivatives():
    a = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose((surrogate.gelu(a + h) - surrogate.gelu(a - h)) / (2 * h),
                               surrogate.dgelu(a), atol=1e-9)
    np.testing.assert_allclose((surrogate.dgelu(a + h) - surrogate.dgelu(a - h)) / (2 * h),
                               surrogate.d2gelu(a), atol=1e-9)
    assert surrogate.gelu(0.0) == 0.0 and abs(surrogate.dgelu(0.0) - 0.5) < 1e-16


@pytest.mark.parametrize("dino", [True, False])
def test_loss_gradient_central_differences(dino):
    r_m, d_z, r_u, bsz = 6, 3, 5, 7
    widths = [r_m + d_z, 12, 12, 12, 12, r_u]
    layers = si.random_mlp(8, widths, bias_scale=0.3)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((bsz, r_m + d_z))
    y = rng.standard_normal((bsz, r_u))
    jy = rng.standard_normal((bsz, r_u, d_z))
    val, grads = training.loss_and_grad(layers, x, y, jy, r_m, dino=dino)
    assert abs(val - training.loss(layers, x, y, jy, r_m, dino=dino)) < 1e-12 * val
    p0 = training.flatten(layers)
    gflat = training.flatten(grads)
    idx = rng.choice(p0.size, 50, replace=False)
    h = 1e-6
    for i in idx:
        pp = p0.copy(); pp[i] += h
        pm = p0.copy(); pm[i] -= h
        fd = (training.loss(training.unflatten(pp, widths), x, y, jy, r_m, dino)
              - training.loss(training.unflatten(pm, widths), x, y, jy, r_m, dino)) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gflat[i])


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g, bias-corrected moments are exactly g and g^2,
    so every step moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(10)
    g = rng.standard_normal(20)
    p = rng.standard_normal(20)
    m = np.zeros(20); v = np.zeros(20)
    p0 = p.copy()
    for step in range(1, 6):
        p, m, v = training.adam_step(p, g, m, v, step, 1e-3)
        np.testing.assert_allclose(p, p0 - step * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_prop31_gradient_error_bound(small_pod):
    """Prop. 3.1: ||dq/dz(u) - dq/dz(u_w)|| <= L ||du/dz|| ||u - u_w||_M
    + ||dq/du(u_w)||_{M^-1} ||du/dz - du_w/dz||, L = 2 for the L2 tracking QoI."""
    prob, ops, xi, Z, samples, U, ubar, Phi, lam = small_pod
    r_m, d_z, r_u = 8, prob.d_z, Phi.shape[1]
    layers = si.random_mlp(12, [r_m + d_z, 16, 16, 16, 16, r_u], bias_scale=0.01)
    Mi = spla.splu(ops.M.tocsc())
    Lh = np.linalg.cholesky(ops.M.toarray())      # M = L L^T, ||v||_M = ||L^T v||
    for i in range(3):
        s = samples[i]
        x = np.concatenate([surrogate.encode(xi[i:i + 1], r_m), Z[i:i + 1]], axis=1)
        phi, jphi = surrogate.jacobian_z(layers, x, r_m)
        uw = surrogate.decode(Phi, ubar, phi[0])
        duw = Phi @ jphi[0]
        du = fem2d.control_jacobian(ops, s)
        bw = fem2d.qoi_gradient(ops, uw)
        g_true = s["g"]
        g_w = bw @ duw
        lhs = np.linalg.norm(g_true - g_w)
        op = lambda A: np.linalg.norm(Lh.T @ A, 2)
        e = uw - s["u"]
        rhs = 2.0 * op(du) * np.sqrt(e @ (ops.M @ e)) + np.sqrt(bw @ Mi.solve(bw)) * op(du - duw)
        assert lhs <= rhs * (1 + 1e-12), (lhs, rhs)
