"""P1 finite elements for the 2D semilinear elliptic state equation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

State equation (paper Sec. 4.2, eq. (elliptic_pde), Dirichlet u = 0):

    -div(exp(m) grad u) + r u^3 = sum_k z_k f_k      on (0,1)^2,

with Gaussian sources f_k(x) = (sigma sqrt(2 pi))^{-1} exp(-|x-x_k|^2/(2 sigma^2))
(Sec. 4.2, source definition) and a log-coefficient m drawn from a sine
Karhunen-Loeve expansion (the KLE input basis of Sec. 3.3).  The QoI is the
tracking functional Q(u) = int (u - u_target)^2 dx (Sec. 4.2) with one of the
two target states of Sec. 4.2, sin(2 pi x) sin(2 pi y) or 4 y (1 - y), or a
constant, interpolated at the nodes.  Newton on the
discrete residual uses sparse LU, the adjoint reuses the last factors
(Sec. 2.3, eq. (ouu_qoi_gradient)).

Discretisation readings (the paper defers them to FEniCS defaults):
  * mesh: nodes (i h, j h), 0 <= i, j <= n, flat index j (n+1) + i; every
    cell is split along its (i,j)-(i+1,j+1) diagonal;
  * kappa_T = mean of exp(m) at the three vertices of T;
  * the reaction term and the source are lumped: weights w_p = sum |T|/3;
  * the QoI uses the consistent P1 mass matrix over all nodes.

Everything is written from element loops over triangles; no stencil formula
appears here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


TARGET_CONST, TARGET_SIN, TARGET_QUAD = 0, 1, 2


def target_state(prob, xy: np.ndarray) -> np.ndarray:
    """u_target at the points xy (Sec. 4.2): sin(2 pi x1) sin(2 pi x2),
    4 x2 (1 - x2), or the constant u_target."""
    x, y = xy[:, 0], xy[:, 1]
    if prob.target == TARGET_SIN:
        return np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    if prob.target == TARGET_QUAD:
        return 4.0 * y * (1.0 - y)
    return np.full(len(xy), prob.u_target)


@dataclass(frozen=True)
class Problem2D:
    n: int = 32                  # cells per side
    n_src_per_dim: int = 5       # sources on an n_src x n_src interior lattice
    src_sigma: float = 0.05      # source width sigma
    kl_per_dim: int = 8          # K1 sine modes per dimension
    kl_shift: float = 25.0       # a_jk = amp (pi^2 (j^2+k^2) + shift)^(-exp)
    kl_exp: float = 1.25
    kl_amp: float = 1.0
    reaction: float = 1.0        # r
    u_target: float = 0.5        # the target when target == TARGET_CONST
    target: int = 0              # TARGET_CONST, TARGET_SIN or TARGET_QUAD

    @property
    def h(self) -> float:
        return 1.0 / self.n

    @property
    def d_z(self) -> int:
        return self.n_src_per_dim ** 2

    @property
    def n_nodes(self) -> int:
        return (self.n + 1) ** 2

    @property
    def n_unknowns(self) -> int:
        return (self.n - 1) ** 2


# ----------------------------------------------------------------------------
# Mesh
# ----------------------------------------------------------------------------

def node_coords(n: int) -> np.ndarray:
    """(n+1)^2 x 2 node coordinates, flat index j (n+1) + i (x fastest)."""
    t = np.arange(n + 1) / n
    x, y = np.meshgrid(t, t, indexing="xy")      # x varies along axis 1
    return np.stack([x.ravel(), y.ravel()], axis=1)


def interior_nodes(n: int) -> np.ndarray:
    """Flat indices of the (n-1)^2 interior nodes, in flat-index order."""
    i, j = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="xy")
    return (j * (n + 1) + i).ravel()


def triangles(n: int) -> np.ndarray:
    """2 n^2 x 3 vertex indices; cell (i,j) -> T_lo, T_up (counter-clockwise)."""
    tris = []
    for j in range(n):
        for i in range(n):
            p00 = j * (n + 1) + i
            p10 = p00 + 1
            p11 = p00 + n + 2
            p01 = p00 + n + 1
            tris.append((p00, p10, p11))   # lower-right triangle
            tris.append((p00, p11, p01))   # upper-left triangle
    return np.array(tris, dtype=np.int64)


def element_gradients(coords: np.ndarray, tris: np.ndarray):
    """Areas |T| and gradients of the three barycentric functions of each T.

    For vertices v_a, solve [1 x y] c = e_a; grad lambda_a = (c_1, c_2).
    Returns (area (nT,), grads (nT, 3, 2)).
    """
    v = coords[tris]                                   # nT x 3 x 2
    mat = np.concatenate([np.ones(v.shape[:2] + (1,)), v], axis=2)   # nT x 3 x 3
    inv = np.linalg.inv(mat)                           # columns: coefficients
    grads = np.transpose(inv[:, 1:, :], (0, 2, 1))     # nT x 3 x 2
    area = 0.5 * np.abs(np.linalg.det(mat))
    return area, grads


# ----------------------------------------------------------------------------
# Random field (sine KL expansion)
# ----------------------------------------------------------------------------

def kl_amplitudes(prob: Problem2D) -> np.ndarray:
    """a_jk = amp (pi^2 (j^2 + k^2) + shift)^(-exp), j, k = 1..K1 (K1 x K1)."""
    j = np.arange(1, prob.kl_per_dim + 1)
    jj, kk = np.meshgrid(j, j, indexing="ij")
    return prob.kl_amp * (np.pi ** 2 * (jj ** 2 + kk ** 2) + prob.kl_shift) ** (-prob.kl_exp)


def field_nodal(xi: np.ndarray, prob: Problem2D) -> np.ndarray:
    """m(x_p) = sum_jk a_jk xi_jk sin(j pi x_p) sin(k pi y_p) at all nodes.

    xi: (K1, K1) with j (x-frequency) first.  Returns (n+1)^2 values.
    """
    a = kl_amplitudes(prob)
    xy = node_coords(prob.n)
    modes = np.arange(1, prob.kl_per_dim + 1)
    sx = np.sin(np.pi * np.outer(xy[:, 0], modes))     # nodes x K1 (j)
    sy = np.sin(np.pi * np.outer(xy[:, 1], modes))     # nodes x K1 (k)
    m = np.zeros(len(xy))
    for j in range(prob.kl_per_dim):
        for k in range(prob.kl_per_dim):
            m += a[j, k] * xi[j, k] * sx[:, j] * sy[:, k]
    return m


# ----------------------------------------------------------------------------
# Assembly by element loops
# ----------------------------------------------------------------------------

def _scatter(n_nodes, tris, local):
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    return sp.coo_matrix((local.ravel(), (rows, cols)), shape=(n_nodes, n_nodes)).tocsr()


def assemble_stiffness_full(n: int, coef_nodal: np.ndarray) -> sp.csr_matrix:
    """K_pq = sum_T kappa_T |T| grad phi_p . grad phi_q over all nodes, with
    kappa_T the mean of the nodal coefficient over the vertices of T."""
    coords = node_coords(n)
    tris = triangles(n)
    area, grads = element_gradients(coords, tris)
    kappa = coef_nodal[tris].mean(axis=1)
    local = (kappa * area)[:, None, None] * np.einsum("tad,tbd->tab", grads, grads)
    return _scatter(len(coords), tris, local)


def assemble_mass_full(n: int) -> sp.csr_matrix:
    """Consistent P1 mass: local |T|/12 [[2,1,1],[1,2,1],[1,1,2]]."""
    coords = node_coords(n)
    tris = triangles(n)
    area, _ = element_gradients(coords, tris)
    ref = (np.ones((3, 3)) + np.eye(3)) / 12.0
    local = area[:, None, None] * ref[None, :, :]
    return _scatter(len(coords), tris, local)


def lumped_weights_full(n: int) -> np.ndarray:
    """w_p = sum_{T containing p} |T| / 3 at every node."""
    coords = node_coords(n)
    tris = triangles(n)
    area, _ = element_gradients(coords, tris)
    w = np.zeros(len(coords))
    np.add.at(w, tris.ravel(), np.repeat(area / 3.0, 3))
    return w


def source_centres(prob: Problem2D) -> np.ndarray:
    """Interior lattice ((a+1)/(s+1), (b+1)/(s+1)), source k = s b + a."""
    s = prob.n_src_per_dim
    c = (np.arange(s) + 1.0) / (s + 1.0)
    a, b = np.meshgrid(np.arange(s), np.arange(s), indexing="xy")
    return np.stack([c[a.ravel()], c[b.ravel()]], axis=1)


def source_functions(prob: Problem2D, xy: np.ndarray) -> np.ndarray:
    """f_k(x) = (sigma sqrt(2 pi))^{-1} exp(-|x - x_k|^2 / (2 sigma^2)); (len(xy), d_Z)."""
    c = source_centres(prob)
    s = prob.src_sigma
    d2 = ((xy[:, None, :] - c[None, :, :]) ** 2).sum(axis=2)
    return np.exp(-d2 / (2 * s * s)) / (s * np.sqrt(2 * np.pi))


@dataclass
class Operators2D:
    """Sample-independent discrete operators, restricted to interior nodes."""
    prob: Problem2D
    interior: np.ndarray          # flat indices of unknowns
    M_full: sp.csr_matrix         # consistent mass, all nodes
    M: sp.csr_matrix              # consistent mass, interior block
    w: np.ndarray                 # lumped weights, interior
    F: np.ndarray                 # lumped source matrix, interior x d_Z
    t_full: np.ndarray = field(repr=False, default=None)   # target over all nodes


def operators(prob: Problem2D) -> Operators2D:
    n = prob.n
    interior = interior_nodes(n)
    M_full = assemble_mass_full(n)
    w_full = lumped_weights_full(n)
    xy = node_coords(n)
    F_full = w_full[:, None] * source_functions(prob, xy)
    t_full = target_state(prob, xy)
    return Operators2D(prob=prob, interior=interior, M_full=M_full,
                       M=M_full[interior][:, interior].tocsr(),
                       w=w_full[interior], F=F_full[interior], t_full=t_full)


def stiffness(ops: Operators2D, m_nodal: np.ndarray) -> sp.csr_matrix:
    K_full = assemble_stiffness_full(ops.prob.n, np.exp(m_nodal))
    return K_full[ops.interior][:, ops.interior].tocsr()


# ----------------------------------------------------------------------------
# Nonlinear solve, QoI, adjoint
# ----------------------------------------------------------------------------

def residual(u, K, w, r, f):
    """R(u) = K u + r w u^3 - f (gradient of the convex energy below)."""
    return K @ u + r * w * u ** 3 - f


def energy(u, K, w, r, f):
    """E(u) = 1/2 u^T K u + r/4 sum w u^4 - f^T u."""
    return 0.5 * u @ (K @ u) + 0.25 * r * np.sum(w * u ** 4) - f @ u


def jacobian(u, K, w, r):
    """dR/du = K + 3 r diag(w u^2) (symmetric positive definite)."""
    return (K + sp.diags(3.0 * r * w * u ** 2)).tocsc()


class CGSolver:
    """Solves with one SPD matrix by Jacobi-preconditioned conjugate
    gradients (scipy's textbook CG) to a relative residual of `rtol`; a
    stand-in for the LU factors where a direct factorisation of a large 3D
    Jacobian is too slow.  Same .solve interface as the LU object."""

    def __init__(self, A, rtol=1e-14):
        self.A = A.tocsr()
        self.M = sp.diags(1.0 / self.A.diagonal())
        self.rtol = rtol

    def solve(self, b):
        b = np.asarray(b, dtype=np.float64)
        if b.ndim == 2:
            return np.stack([self.solve(b[:, k]) for k in range(b.shape[1])], axis=1)
        x, info = spla.cg(self.A, b, rtol=self.rtol, atol=0.0, maxiter=20000, M=self.M)
        if info != 0:
            raise RuntimeError(f"CG did not converge (info {info})")
        return x


def _factor(J, linear):
    return spla.splu(J) if linear == "lu" else CGSolver(J)


def newton_solve(K, w, r, f, rtol=1e-14, max_iter=20, history=None, linear="lu"):
    """Newton from u = 0 with sparse LU (linear="cg": the CG stand-in above).

    Stops when ||R|| <= rtol max(1, ||f||), or after a step whose size is at
    the float64 rounding level of u (||du|| <= 1e-13 ||u||: the remaining
    error is then quadratically small).  A backtracking safeguard on the
    energy is kept, though the convex problem never needs it in practice.
    Returns (u, LU of the Jacobian at the returned u, Newton steps taken).
    """
    u = np.zeros_like(f)
    scale = max(1.0, np.linalg.norm(f))
    steps = 0
    while True:
        R = residual(u, K, w, r, f)
        nr = np.linalg.norm(R)
        if history is not None:
            history.append(nr)
        if nr <= rtol * scale:
            break
        if steps == max_iter:
            raise RuntimeError(f"Newton did not converge: ||R|| = {nr:.3e}")
        lu = _factor(jacobian(u, K, w, r), linear)
        du = -lu.solve(R)
        e0 = energy(u, K, w, r, f)
        step = 1.0
        while energy(u + step * du, K, w, r, f) > e0 + 1e-12 * abs(e0) and step > 1e-4:
            step *= 0.5
        u = u + step * du
        steps += 1
        if np.linalg.norm(step * du) <= 1e-13 * np.linalg.norm(u):
            if history is not None:
                history.append(np.linalg.norm(residual(u, K, w, r, f)))
            break
    lu = _factor(jacobian(u, K, w, r), linear)
    return u, lu, steps


def extend(ops: Operators2D, u_int: np.ndarray) -> np.ndarray:
    """Interior vector -> all nodes, with the Dirichlet value 0 on the boundary."""
    u = np.zeros(ops.prob.n_nodes)
    u[ops.interior] = u_int
    return u


def qoi(ops: Operators2D, u_int: np.ndarray) -> float:
    """q = (u - u_target)^T M_full (u - u_target) = int (u - u_target)^2 dx (exact for P1)."""
    d = extend(ops, u_int) - ops.t_full
    return float(d @ (ops.M_full @ d))


def qoi_gradient(ops: Operators2D, u_int: np.ndarray) -> np.ndarray:
    """dq/du on the unknowns: 2 (M_full (u - u_target)) restricted to the interior."""
    d = extend(ops, u_int) - ops.t_full
    return 2.0 * (ops.M_full @ d)[ops.interior]


def solve_sample(ops: Operators2D, xi_i: np.ndarray, z: np.ndarray, want_grad=True,
                 rtol=1e-14, history=None):
    """One sample: state u, q and dq/dz = F^T lambda with A(u) lambda = dq/du.

    Sign: R(u(z), z) = 0 with dR/dz = -F gives du/dz = A^{-1} F, so
    dq/dz = F^T A^{-T} dq/du and A = A^T (Sec. 2.3, adjoint gradient).
    """
    prob = ops.prob
    K = stiffness(ops, field_nodal(xi_i, prob))
    f = ops.F @ z
    u, lu, iters = newton_solve(K, ops.w, prob.reaction, f, rtol=rtol, history=history)
    q = qoi(ops, u)
    out = {"u": u, "q": q, "newton_iters": iters, "K": K, "lu": lu}
    if want_grad:
        lam = lu.solve(qoi_gradient(ops, u))
        out["lam"] = lam
        out["g"] = ops.F.T @ lam
    return out


def control_jacobian(ops: Operators2D, sample: dict) -> np.ndarray:
    """du/dz = A(u)^{-1} F: the d_Z linearised solves reusing one factorisation
    (Sec. 3.4, eq. (projected_sensitivity), d_Z < r_U case)."""
    return sample["lu"].solve(ops.F)
