"""Pins of the oracle's finite-element state solve (no GPU).

Each test checks the oracle against something other than itself: a
manufactured solution with a known convergence order, a closed-form discrete
solution, exact quadrature identities, Newton's quadratic rate, convexity.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import sympy

from oracle import fem2d


def _mms_source():
    """f = -div(e^m grad u) + r u^3 for u = sin(pi x) sin(pi y),
    m = 0.3 sin(pi x) sin(2 pi y), r = 1, derived symbolically."""
    x, y = sympy.symbols("x y")
    u = sympy.sin(sympy.pi * x) * sympy.sin(sympy.pi * y)
    m = sympy.Rational(3, 10) * sympy.sin(sympy.pi * x) * sympy.sin(2 * sympy.pi * y)
    k = sympy.exp(m)
    f = -(sympy.diff(k * sympy.diff(u, x), x) + sympy.diff(k * sympy.diff(u, y), y)) + u ** 3
    return (sympy.lambdify((x, y), f, "numpy"), sympy.lambdify((x, y), u, "numpy"),
            sympy.lambdify((x, y), m, "numpy"))


def test_mms_second_order_convergence():
    f_ex, u_ex, m_ex = _mms_source()
    errs = []
    ns = [8, 16, 32, 64]
    for n in ns:
        prob = fem2d.Problem2D(n=n)
        ops = fem2d.operators(prob)
        xy = fem2d.node_coords(n)
        K = fem2d.stiffness(ops, m_ex(xy[:, 0], xy[:, 1]))
        xi = xy[ops.interior]
        f = ops.w * f_ex(xi[:, 0], xi[:, 1])
        u, _, _ = fem2d.newton_solve(K, ops.w, 1.0, f)
        e = fem2d.extend(ops, u - u_ex(xi[:, 0], xi[:, 1]))
        errs.append(np.sqrt(e @ (ops.M_full @ e)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.1), rates


@pytest.mark.parametrize("n", [8, 32])
def test_discrete_sine_closed_form(n):
    """kappa = 1, r = 0, source w_p sin(pi x) sin(pi y): the discrete solution
    is h^2 sin sin / (8 sin^2(pi h / 2)) (eigenvector of the 5-point Laplacian)."""
    prob = fem2d.Problem2D(n=n, reaction=0.0)
    ops = fem2d.operators(prob)
    xy = fem2d.node_coords(n)[ops.interior]
    s = np.sin(np.pi * xy[:, 0]) * np.sin(np.pi * xy[:, 1])
    K = fem2d.stiffness(ops, np.zeros(prob.n_nodes))
    u, _, _ = fem2d.newton_solve(K, ops.w, 0.0, ops.w * s)
    h = 1.0 / n
    exact = h * h * s / (8.0 * np.sin(np.pi * h / 2) ** 2)
    assert np.max(np.abs(u - exact)) <= 1e-14 * np.max(np.abs(exact)) * 10
    np.testing.assert_allclose(ops.w, h * h, rtol=1e-14)


def test_stiffness_is_five_point_edge_stencil():
    """For per-triangle coefficients the P1 stiffness on this mesh couples only
    E/W/N/S neighbours, with edge weight -(kappa_T1 + kappa_T2)/2 of the two
    triangles sharing the edge; the diagonal couplings vanish exactly."""
    n = 6
    rng = np.random.default_rng(0)
    coef = np.exp(0.5 * rng.standard_normal((n + 1) ** 2))
    K = fem2d.assemble_stiffness_full(n, coef).toarray()
    P = lambda i, j: j * (n + 1) + i
    kap = lambda a, b, c: (coef[a] + coef[b] + coef[c]) / 3.0
    for j in range(n + 1):
        for i in range(n + 1):
            p = P(i, j)
            nz = set(np.nonzero(np.abs(K[p]) > 1e-15)[0])
            allowed = {p}
            if i < n:
                allowed.add(P(i + 1, j))
            if i > 0:
                allowed.add(P(i - 1, j))
            if j < n:
                allowed.add(P(i, j + 1))
            if j > 0:
                allowed.add(P(i, j - 1))
            assert nz <= allowed
            if i < n:   # east edge (i,j)-(i+1,j): T_lo(i,j) below-right, T_up(i,j-1) below
                ws = []
                if j < n:
                    ws.append(kap(P(i, j), P(i + 1, j), P(i + 1, j + 1)))
                if j > 0:
                    ws.append(kap(P(i, j - 1), P(i + 1, j), P(i, j)))
                assert abs(K[p, P(i + 1, j)] + sum(ws) / 2) < 1e-14
            if j < n:   # north edge (i,j)-(i,j+1): T_up(i,j), T_lo(i-1,j)
                ws = []
                if i < n:
                    ws.append(kap(P(i, j), P(i + 1, j + 1), P(i, j + 1)))
                if i > 0:
                    ws.append(kap(P(i - 1, j), P(i, j), P(i, j + 1)))
                assert abs(K[p, P(i, j + 1)] + sum(ws) / 2) < 1e-14
    np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-13)   # constants in the kernel


def test_mass_matrix_exact_moments():
    """Consistent P1 mass integrates products of P1 functions exactly:
    int 1 = 1, int x^2 = 1/3, int x y = 1/4, int (x+2y)^2 = 1/3 + 1 + 4/3."""
    n = 7
    M = fem2d.assemble_mass_full(n)
    xy = fem2d.node_coords(n)
    one = np.ones(len(xy))
    x, y = xy[:, 0], xy[:, 1]
    assert abs(one @ M @ one - 1.0) < 1e-14
    assert abs(x @ M @ x - 1.0 / 3.0) < 1e-14
    assert abs(x @ M @ y - 0.25) < 1e-14
    v = x + 2 * y
    assert abs(v @ M @ v - (1 / 3 + 1.0 + 4 / 3)) < 1e-13
    assert np.all(np.linalg.eigvalsh(M.toarray()) > 0)


def test_lumped_weights_and_source_mass():
    """sum_p w_p = area; sum_p w_p f_k(x_p) -> int f_k = sigma sqrt(2 pi) for a
    source well inside the domain (2D Gaussian mass 2 pi sigma^2 times the
    prefactor)."""
    prob = fem2d.Problem2D(n=256)
    w = fem2d.lumped_weights_full(prob.n)
    assert abs(w.sum() - 1.0) < 1e-12
    xy = fem2d.node_coords(prob.n)
    f = fem2d.source_functions(prob, xy)
    mass = w @ f
    centre = 12                           # source at (1/2, 1/2): 10 sigma from the boundary
    np.testing.assert_allclose(mass[centre], prob.src_sigma * np.sqrt(2 * np.pi), rtol=1e-9)
    # sources 3.3 sigma from an edge lose at most their tail beyond that edge
    assert np.all(mass <= prob.src_sigma * np.sqrt(2 * np.pi) * (1 + 1e-9))
    assert np.all(mass >= prob.src_sigma * np.sqrt(2 * np.pi) * (1 - 2e-3))


def test_newton_quadratic_convergence_and_energy_minimum():
    prob = fem2d.Problem2D(n=32, kl_amp=30.0)
    ops = fem2d.operators(prob)
    rng = np.random.default_rng(3)
    xi = rng.standard_normal((8, 8))
    z = 4.0 * rng.uniform(0, 1, 25)          # larger control: stronger nonlinearity
    hist = []
    s = fem2d.solve_sample(ops, xi, z, history=hist)
    assert 2 <= s["newton_iters"] <= 6
    r = np.array(hist)
    # quadratic: log r_{k+1} ~ 2 log r_k (checked while above rounding level)
    for k in range(len(r) - 2):
        if r[k + 1] > 1e-12:
            assert r[k + 1] <= 10.0 * r[k] ** 2 / r[0], (k, r)
    K, w, f = s["K"], ops.w, ops.F @ z
    e0 = fem2d.energy(s["u"], K, w, prob.reaction, f)
    for _ in range(5):
        d = 1e-3 * rng.standard_normal(len(s["u"]))
        assert fem2d.energy(s["u"] + d, K, w, prob.reaction, f) > e0
    assert np.all(np.abs((K - K.T).data) < 1e-15) if (K - K.T).nnz else True


def test_kl_field_recovered_by_sine_orthogonality():
    """The nodal field of a KL draw determines its xi (discrete sine
    orthogonality), which pins the mode ordering and amplitudes."""
    from oracle import surrogate
    prob = fem2d.Problem2D(n=32, kl_per_dim=8)
    xi = np.random.default_rng(5).standard_normal((8, 8))
    m = fem2d.field_nodal(xi, prob)
    r_m = 64
    rec = surrogate.encode_from_nodal(m, prob.n, fem2d.kl_amplitudes(prob), r_m)
    np.testing.assert_allclose(rec, surrogate.encode(xi[None], r_m)[0], rtol=0, atol=1e-12)
    a = fem2d.kl_amplitudes(prob)
    assert abs(a[0, 0] - (2 * np.pi ** 2 + 25) ** -1.25) < 1e-18


@pytest.mark.parametrize("target,exact", [(fem2d.TARGET_SIN, 0.25), (fem2d.TARGET_QUAD, 8.0 / 15.0),
                                          (fem2d.TARGET_CONST, 0.25)])
def test_tracking_qoi_of_zero_state_converges_to_target_norm(target, exact):
    """Q(0) = int u_target^2 over the unit square (Sec. 4.2 targets):
    int sin^2(2 pi x) sin^2(2 pi y) = 1/4, int 16 y^2 (1 - y)^2 = 8/15, and a
    constant 0.5 gives 1/4 exactly.  The mass norm of the nodal interpolant
    converges at second order; dQ/du(0) = -2 (M u_target)_I, whose sum over
    the interior plus the boundary rows is -2 int u_target."""
    errs = []
    for n in (16, 32, 64):
        ops = fem2d.operators(fem2d.Problem2D(n=n, target=target, u_target=0.5))
        q = fem2d.qoi(ops, np.zeros(ops.prob.n_unknowns))
        errs.append(abs(q - exact))
        g = fem2d.qoi_gradient(ops, np.zeros(ops.prob.n_unknowns))
        full = -2.0 * (ops.M_full @ ops.t_full)
        np.testing.assert_allclose(g, full[ops.interior], rtol=1e-14, atol=1e-16)
        integral = {fem2d.TARGET_SIN: 0.0, fem2d.TARGET_QUAD: 2.0 / 3.0, fem2d.TARGET_CONST: 0.5}[target]
        assert abs(-0.5 * full.sum() - integral) <= 4.0 / n ** 2
    if target == fem2d.TARGET_CONST:
        assert max(errs) <= 1e-14
    else:
        assert errs[2] <= 2e-3
        assert 3.5 <= errs[0] / errs[1] <= 4.5 and 3.5 <= errs[1] / errs[2] <= 4.5, errs
