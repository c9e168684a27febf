"""Pins of the 3D Q1 oracle (no GPU).

Each test checks the oracle against something other than itself: the
textbook trilinear element matrices, exact quadrature identities, a
manufactured solution with its convergence order, a closed-form discrete
solution from the tensor-product structure of the Q1 matrices, discrete sine
orthogonality of the KL field, the closed-form integral of the Gaussian
sources and a Taylor test of the adjoint gradient.
"""
import math

import numpy as np
import pytest
import sympy

import saa_inputs as si
from oracle import fem2d, fem3d


def test_reference_element_matches_textbook_values():
    """Unit-cube trilinear element: stiffness 1/3 on the diagonal, 0 between
    vertices sharing an edge, -1/12 across a face diagonal and across the body
    diagonal; mass (1/6)^3 prod_d (2 if the bits agree else 1)."""
    K, M = fem3d.reference_matrices()
    for a in range(8):
        for b in range(8):
            differ = bin(a ^ b).count("1")
            kv = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}[differ]
            mv = 2.0 ** (3 - differ) / 216.0
            assert abs(K[a, b] - kv) < 1e-15, (a, b)
            assert abs(M[a, b] - mv) < 1e-15, (a, b)


def test_assembled_stencil_and_lumped_weights():
    """kappa = 1: interior row of K is 8h/3 at the centre, 0 at the six face
    neighbours, -h/6 at the twelve edge neighbours, -h/12 at the eight
    corners; lumped weights h^3."""
    n = 6
    K = fem3d.assemble_stiffness_full(n, np.ones((n + 1) ** 3)).toarray()
    h = 1.0 / n
    p = (3 * (n + 1) + 3) * (n + 1) + 3
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                q = p + (dz * (n + 1) + dy) * (n + 1) + dx
                nz = abs(dx) + abs(dy) + abs(dz)
                want = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[nz]
                assert abs(K[p, q] - want) < 1e-15
    assert np.count_nonzero(np.abs(K[p]) > 1e-15) == 21
    w = fem3d.lumped_weights_full(n)
    np.testing.assert_allclose(w[fem3d.interior_nodes(n)], h ** 3, rtol=1e-14)


def test_mass_and_stiffness_quadrature_identities():
    """Products of Q1 functions are integrated exactly: int 1 = 1,
    int x y z = 1/8, int x^2 = 1/3; int |grad (x y)|^2 = 2/3,
    int |grad x|^2 = 1 (kappa = 1)."""
    n = 5
    M = fem3d.assemble_mass_full(n)
    K = fem3d.assemble_stiffness_full(n, np.ones((n + 1) ** 3))
    xyz = fem3d.node_coords(n)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    one = np.ones(len(x))
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    assert abs(x @ (M @ (y * z)) - 0.125) < 1e-14
    assert abs(x @ (M @ x) - 1.0 / 3.0) < 1e-14
    assert abs((x * y) @ (K @ (x * y)) - 2.0 / 3.0) < 1e-13
    assert abs(x @ (K @ x) - 1.0) < 1e-13
    assert np.max(np.abs(K @ one)) < 1e-13          # constants lie in the kernel


def _mms():
    x, y, z = sympy.symbols("x y z")
    u = sympy.sin(sympy.pi * x) * sympy.sin(sympy.pi * y) * sympy.sin(sympy.pi * z)
    m = sympy.Rational(3, 10) * sympy.sin(sympy.pi * x) * sympy.sin(2 * sympy.pi * y) * sympy.sin(sympy.pi * z)
    k = sympy.exp(m)
    f = -sum(sympy.diff(k * sympy.diff(u, v), v) for v in (x, y, z)) + u ** 3
    return tuple(sympy.lambdify((x, y, z), e, "numpy") for e in (f, u, m))


def test_mms_second_order_convergence():
    f_ex, u_ex, m_ex = _mms()
    errs = []
    for n in (6, 12, 24):
        prob = fem3d.Problem3D(n=n, kl_per_dim=2)
        ops = fem3d.operators(prob)
        xyz = fem3d.node_coords(n)
        K = fem3d.stiffness(ops, m_ex(xyz[:, 0], xyz[:, 1], xyz[:, 2]))
        xi = xyz[ops.interior]
        f = ops.w * f_ex(xi[:, 0], xi[:, 1], xi[:, 2])
        u, _, _ = fem2d.newton_solve(K, ops.w, 1.0, f)
        e = fem3d.extend(ops, u - u_ex(xi[:, 0], xi[:, 1], xi[:, 2]))
        errs.append(np.sqrt(e @ (ops.M_full @ e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.15), rates


@pytest.mark.parametrize("n", [4, 10])
def test_discrete_sine_closed_form(n):
    """kappa = 1, r = 0, lumped source h^3 s with s = sin sin sin: s is an
    eigenvector of K = sum_d K1 (x) M1 (x) M1 with 1D stiffness eigenvalue
    (4/h) sin^2(pi h/2) and 1D mass eigenvalue (h/3)(2 + cos pi h), so
    u = h^3 s / (3 (4/h) sin^2(pi h/2) ((h/3)(2 + cos pi h))^2)."""
    prob = fem3d.Problem3D(n=n, reaction=0.0, kl_per_dim=2)
    ops = fem3d.operators(prob)
    xyz = fem3d.node_coords(n)[ops.interior]
    s = np.sin(np.pi * xyz[:, 0]) * np.sin(np.pi * xyz[:, 1]) * np.sin(np.pi * xyz[:, 2])
    K = fem3d.stiffness(ops, np.zeros(prob.n_nodes))
    u, _, _ = fem2d.newton_solve(K, ops.w, 0.0, ops.w * s)
    h = 1.0 / n
    lam = 3.0 * (4.0 / h) * np.sin(np.pi * h / 2) ** 2 * ((h / 3.0) * (2.0 + np.cos(np.pi * h))) ** 2
    exact = h ** 3 * s / lam
    assert np.max(np.abs(u - exact)) <= 1e-13 * np.max(np.abs(exact))


def test_kl_field_sine_orthogonality():
    """sum over interior nodes of m sin(j pi x) sin(k pi y) sin(l pi z)
    = (n/2)^3 a_jkl xi_jkl for 1 <= j, k, l < n."""
    prob = fem3d.Problem3D(n=8, kl_per_dim=5, kl_amp=3.0)
    xi = si.kl_coefficients(77, 1, 5, dim=3)[0]
    m = fem3d.field_nodal(xi, prob)
    xyz = fem3d.node_coords(prob.n)
    a = fem3d.kl_amplitudes(prob)
    for (j, k, l) in [(1, 1, 1), (2, 5, 3), (5, 5, 5), (4, 1, 2)]:
        basis = (np.sin(j * np.pi * xyz[:, 0]) * np.sin(k * np.pi * xyz[:, 1]) * np.sin(l * np.pi * xyz[:, 2]))
        got = m @ basis / (prob.n / 2) ** 3
        assert abs(got - a[j - 1, k - 1, l - 1] * xi[j - 1, k - 1, l - 1]) < 1e-14
    # a value the amplitude law fixes: a_111 = (3 pi^2 + 25)^(-1.5) times kl_amp
    assert abs(a[0, 0, 0] - 3.0 * (3 * np.pi ** 2 + 25.0) ** -1.5) < 1e-16


def test_source_integrals_match_closed_form():
    """Lumped quadrature over all nodes (boundary nodes with their partial
    weights) of each source equals int_cube f_k = (sigma sqrt(2 pi))^{-1}
    prod_d sigma sqrt(pi/2) [erf((1 - c_d)/(sigma sqrt 2)) + erf(c_d/(sigma sqrt 2))]
    up to O(h^2); the largest load of source k sits at the node nearest its
    lattice centre ((a+1)/(s+1), (b+1)/(s+1), (c+1)/(s+1)), k = a + s b + s^2 c."""
    prob = fem3d.Problem3D(n=40, kl_per_dim=2)
    ops = fem3d.operators(prob)
    xyz = fem3d.node_coords(prob.n)
    w = fem3d.lumped_weights_full(prob.n)
    fk = fem3d.source_functions(prob, xyz)
    s = prob.src_sigma
    cs = (np.arange(prob.n_src_per_dim) + 1.0) / (prob.n_src_per_dim + 1.0)
    for k in [0, 5, 21, 63]:
        a, b, c = k % 4, (k // 4) % 4, k // 16
        exact = 1.0 / (s * math.sqrt(2 * math.pi))
        for cd in (cs[a], cs[b], cs[c]):
            exact *= s * math.sqrt(math.pi / 2) * (math.erf((1 - cd) / (s * math.sqrt(2))) +
                                                   math.erf(cd / (s * math.sqrt(2))))
        # Euler-Maclaurin: the trapezoid error is (h^2/12) [f'] at the faces,
        # about 3.6e-4 relative per face 2.5 sigma from a centre at n = 40
        assert abs(w @ fk[:, k] - exact) < 2e-3 * exact, k
        if k == 0:   # and it falls as h^2
            p2 = fem3d.Problem3D(n=20, kl_per_dim=2)
            x2 = fem3d.node_coords(20)
            e2 = abs(fem3d.lumped_weights_full(20) @ fem3d.source_functions(p2, x2)[:, 0] - exact)
            assert 3.5 < e2 / abs(w @ fk[:, k] - exact) < 4.5
        peak = xyz[ops.interior][np.argmax(ops.F[:, k])]
        assert np.max(np.abs(peak - np.array([cs[a], cs[b], cs[c]]))) <= 0.5 / prob.n, k


def test_qoi_of_zero_state_is_target_norm():
    """q(0) = int u_target^2: exactly 0.25 for the constant 0.5; 1/8 for the
    product of sines (second order in h)."""
    p0 = fem3d.Problem3D(n=6, kl_per_dim=2)
    o0 = fem3d.operators(p0)
    assert abs(fem3d.qoi(o0, np.zeros(len(o0.interior))) - 0.25) < 1e-14
    errs = []
    for n in (8, 16):
        p = fem3d.Problem3D(n=n, kl_per_dim=2, target=fem3d.TARGET_SIN)
        o = fem3d.operators(p)
        errs.append(abs(fem3d.qoi(o, np.zeros(len(o.interior))) - 0.125))
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_adjoint_gradient_taylor():
    """dq/dz from the adjoint against central differences of q(z) along a
    random direction (second-order agreement as the step shrinks)."""
    prob = fem3d.Problem3D(n=8, n_src_per_dim=2, kl_per_dim=3, kl_amp=20.0, target=fem3d.TARGET_SIN)
    ops = fem3d.operators(prob)
    xi = si.kl_coefficients(78, 1, 3, dim=3)[0]
    z = si.control(79, prob.d_z, lo=-2.0, hi=4.0)
    s = fem3d.solve_sample(ops, xi, z)
    dz = np.random.default_rng(80).standard_normal(prob.d_z)
    errs = []
    for h in (1e-1, 5e-2):
        qp = fem3d.solve_sample(ops, xi, z + h * dz, want_grad=False)["q"]
        qm = fem3d.solve_sample(ops, xi, z - h * dz, want_grad=False)["q"]
        errs.append(abs((qp - qm) / (2 * h) - s["g"] @ dz))
    assert errs[1] < 0.3 * errs[0] or errs[1] < 1e-11 * abs(s["g"] @ dz)
    assert errs[1] < 1e-4 * abs(s["g"] @ dz)


def test_cg_stand_in_matches_lu():
    """The CG stand-in for the LU factors (used for the stored 48^3 values)
    gives the same q and dq/dz as the direct solves."""
    prob = fem3d.Problem3D(n=8, n_src_per_dim=2, kl_per_dim=3, kl_amp=20.0)
    ops = fem3d.operators(prob)
    xi = si.kl_coefficients(81, 1, 3, dim=3)[0]
    z = si.control(82, prob.d_z)
    a = fem3d.solve_sample(ops, xi, z)
    b = fem3d.solve_sample(ops, xi, z, linear="cg")
    assert abs(a["q"] - b["q"]) <= 1e-13 * abs(a["q"])
    assert np.linalg.norm(a["g"] - b["g"]) <= 1e-11 * np.linalg.norm(a["g"])


def test_control_jacobian_matches_nonlinear_differences():
    """du/dz from the d_Z linearised solves (Sec. 3.4) against central
    differences of the nonlinear state in z (second-order differences with
    h = 1e-5 leave an error of order h^2 u''' ~ 1e-10), and the chain rule
    (dq/du)^T du/dz against the adjoint gradient."""
    prob = fem3d.Problem3D(n=6, n_src_per_dim=4, kl_per_dim=3, kl_amp=20.0, target=fem3d.TARGET_SIN)
    ops = fem3d.operators(prob)
    xi = si.kl_coefficients(83, 1, 3, dim=3)[0]
    z = si.control(84, prob.d_z, lo=-2.0, hi=4.0)
    s = fem3d.solve_sample(ops, xi, z)
    J = fem3d.control_jacobian(ops, s)
    assert J.shape == (len(ops.interior), prob.d_z)
    h = 1e-5
    for k in (0, 21, 63):
        e = np.zeros(prob.d_z)
        e[k] = h
        up = fem3d.solve_sample(ops, xi, z + e, want_grad=False)["u"]
        um = fem3d.solve_sample(ops, xi, z - e, want_grad=False)["u"]
        np.testing.assert_allclose(J[:, k], (up - um) / (2 * h), rtol=1e-6, atol=1e-7 * np.abs(J[:, k]).max())
    np.testing.assert_allclose(fem3d.qoi_gradient(ops, s["u"]) @ J, s["g"], rtol=1e-11)
