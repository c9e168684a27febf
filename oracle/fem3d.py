"""Q1 finite elements for the 3D semilinear elliptic state equation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The same state equation as the 2D problem (paper Sec. 4.2, eq.
(elliptic_pde), Dirichlet u = 0), posed on the unit cube:

    -div(exp(m) grad u) + r u^3 = sum_k z_k f_k      on (0,1)^3,

with Gaussian sources f_k(x) = (sigma sqrt(2 pi))^{-1} exp(-|x-x_k|^2/(2 sigma^2))
(the 2D prefactor kept, width 0.08) on an s x s x s interior lattice, and a
log-coefficient m from a sine Karhunen-Loeve expansion with amplitudes
a_jkl = amp (pi^2 (j^2 + k^2 + l^2) + shift)^(-exp).  The QoI is the tracking
functional Q(u) = int (u - u_target)^2 dx (Sec. 4.2).

Discretisation readings (the paper gives no 3D discretisation):
  * mesh: nodes (i h, j h, k h), 0 <= i, j, k <= n, flat index
    (k (n+1) + j) (n+1) + i; trilinear (Q1) hexahedra;
  * kappa_e = mean of exp(m) at the eight vertices of the element;
  * reaction and source lumped: w_p = sum_e |e| / 8;
  * the QoI uses the consistent Q1 mass matrix over all nodes;
  * targets: the constant u_target, sin(2 pi x) sin(2 pi y) sin(2 pi z), or
    4 y (1 - y), interpolated at the nodes.

Element matrices come from 2 x 2 x 2 Gauss quadrature of the trilinear shape
functions (exact for both matrices); no stencil formula appears here.  The
Newton solver, residual and Jacobian are the dimension-independent ones of
the 2D oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import fem2d

TARGET_CONST, TARGET_SIN, TARGET_QUAD = 0, 1, 2


@dataclass(frozen=True)
class Problem3D:
    n: int = 48                  # cells per side
    n_src_per_dim: int = 4       # sources on an s x s x s interior lattice
    src_sigma: float = 0.08
    kl_per_dim: int = 10         # K1 sine modes per dimension
    kl_shift: float = 25.0
    kl_exp: float = 1.5
    kl_amp: float = 1.0
    reaction: float = 1.0
    u_target: float = 0.5
    target: int = 0

    @property
    def h(self) -> float:
        return 1.0 / self.n

    @property
    def d_z(self) -> int:
        return self.n_src_per_dim ** 3

    @property
    def n_nodes(self) -> int:
        return (self.n + 1) ** 3

    @property
    def n_unknowns(self) -> int:
        return (self.n - 1) ** 3


def target_state(prob, xyz: np.ndarray) -> np.ndarray:
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    if prob.target == TARGET_SIN:
        return np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)
    if prob.target == TARGET_QUAD:
        return 4.0 * y * (1.0 - y)
    return np.full(len(xyz), prob.u_target)


# ----------------------------------------------------------------------------
# Mesh and reference element
# ----------------------------------------------------------------------------

def node_coords(n: int) -> np.ndarray:
    """(n+1)^3 x 3 coordinates, flat index (k (n+1) + j) (n+1) + i."""
    t = np.arange(n + 1) / n
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def interior_nodes(n: int) -> np.ndarray:
    k, j, i = np.meshgrid(np.arange(1, n), np.arange(1, n), np.arange(1, n), indexing="ij")
    return ((k * (n + 1) + j) * (n + 1) + i).ravel()


def hexahedra(n: int) -> np.ndarray:
    """n^3 x 8 vertex indices; local vertex v = a + 2 b + 4 c sits at offset (a, b, c)."""
    np1 = n + 1
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = ((k * np1 + j) * np1 + i).ravel()
    offs = [c * np1 * np1 + b * np1 + a for c in (0, 1) for b in (0, 1) for a in (0, 1)]
    return base[:, None] + np.array(offs)[None, :]


def reference_matrices():
    """Stiffness and mass of the trilinear element on the unit cube, by
    2-point Gauss quadrature per direction (exact for these integrands).

    Shape function of local vertex v = a + 2b + 4c:
    N_v(x) = prod_d (x_d if bit_d else 1 - x_d).
    """
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    for gx in g:
        for gy in g:
            for gz in g:
                pt = (gx, gy, gz)
                N = np.zeros(8)
                dN = np.zeros((8, 3))
                for v in range(8):
                    bits = (v & 1, (v >> 1) & 1, (v >> 2) & 1)
                    f1 = [pt[d] if bits[d] else 1.0 - pt[d] for d in range(3)]
                    df = [1.0 if bits[d] else -1.0 for d in range(3)]
                    N[v] = f1[0] * f1[1] * f1[2]
                    dN[v, 0] = df[0] * f1[1] * f1[2]
                    dN[v, 1] = f1[0] * df[1] * f1[2]
                    dN[v, 2] = f1[0] * f1[1] * df[2]
                w = 1.0 / 8.0          # each Gauss weight is 1/2 on [0, 1]
                K += w * dN @ dN.T
                M += w * np.outer(N, N)
    return K, M


def _scatter(n_nodes, hexes, local):
    rows = np.repeat(hexes, 8, axis=1).ravel()
    cols = np.tile(hexes, (1, 8)).ravel()
    return sp.coo_matrix((local.ravel(), (rows, cols)), shape=(n_nodes, n_nodes)).tocsr()


def assemble_stiffness_full(n: int, coef_nodal: np.ndarray) -> sp.csr_matrix:
    """K_pq = sum_e kappa_e int_e grad phi_p . grad phi_q; an element of side
    h scales the unit-cube matrix by h (gradients 1/h each, volume h^3)."""
    hexes = hexahedra(n)
    Kref, _ = reference_matrices()
    kappa = coef_nodal[hexes].mean(axis=1)
    local = (kappa / n)[:, None, None] * Kref[None, :, :]
    return _scatter((n + 1) ** 3, hexes, local)


def assemble_mass_full(n: int) -> sp.csr_matrix:
    hexes = hexahedra(n)
    _, Mref = reference_matrices()
    local = np.broadcast_to(Mref / n ** 3, (len(hexes), 8, 8))
    return _scatter((n + 1) ** 3, hexes, local)


def lumped_weights_full(n: int) -> np.ndarray:
    hexes = hexahedra(n)
    w = np.zeros((n + 1) ** 3)
    np.add.at(w, hexes.ravel(), 1.0 / (8.0 * n ** 3))
    return w


# ----------------------------------------------------------------------------
# Random field and sources
# ----------------------------------------------------------------------------

def kl_amplitudes(prob: Problem3D) -> np.ndarray:
    j = np.arange(1, prob.kl_per_dim + 1)
    jj, kk, ll = np.meshgrid(j, j, j, indexing="ij")
    return prob.kl_amp * (np.pi ** 2 * (jj ** 2 + kk ** 2 + ll ** 2) + prob.kl_shift) ** (-prob.kl_exp)


def field_nodal(xi: np.ndarray, prob: Problem3D) -> np.ndarray:
    """m(x_p) = sum_jkl a_jkl xi_jkl sin(j pi x) sin(k pi y) sin(l pi z);
    xi: (K1, K1, K1) with j the x-frequency."""
    a = kl_amplitudes(prob) * xi
    t = np.arange(prob.n + 1) / prob.n
    S = np.sin(np.pi * np.outer(np.arange(1, prob.kl_per_dim + 1), t))   # K1 x (n+1)
    # m[z, y, x] = sum_jkl a[j, k, l] S[j, x] S[k, y] S[l, z]
    m = np.einsum("jkl,jx,ky,lz->zyx", a, S, S, S)
    return m.ravel()


def source_centres(prob: Problem3D) -> np.ndarray:
    """((a+1)/(s+1), (b+1)/(s+1), (c+1)/(s+1)), source k = a + s b + s^2 c."""
    s = prob.n_src_per_dim
    c = (np.arange(s) + 1.0) / (s + 1.0)
    cc, bb, aa = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
    return np.stack([c[aa.ravel()], c[bb.ravel()], c[cc.ravel()]], axis=1)


def source_functions(prob: Problem3D, xyz: np.ndarray) -> np.ndarray:
    c = source_centres(prob)
    s = prob.src_sigma
    d2 = ((xyz[:, None, :] - c[None, :, :]) ** 2).sum(axis=2)
    return np.exp(-d2 / (2 * s * s)) / (s * np.sqrt(2 * np.pi))


@dataclass
class Operators3D:
    prob: Problem3D
    interior: np.ndarray
    M_full: sp.csr_matrix
    M: sp.csr_matrix
    w: np.ndarray
    F: np.ndarray
    t_full: np.ndarray = field(repr=False, default=None)


def operators(prob: Problem3D) -> Operators3D:
    n = prob.n
    interior = interior_nodes(n)
    M_full = assemble_mass_full(n)
    w_full = lumped_weights_full(n)
    xyz = node_coords(n)
    F_full = w_full[:, None] * source_functions(prob, xyz)
    return Operators3D(prob=prob, interior=interior, M_full=M_full,
                       M=M_full[interior][:, interior].tocsr(), w=w_full[interior],
                       F=F_full[interior], t_full=target_state(prob, xyz))


def stiffness(ops: Operators3D, m_nodal: np.ndarray) -> sp.csr_matrix:
    K_full = assemble_stiffness_full(ops.prob.n, np.exp(m_nodal))
    return K_full[ops.interior][:, ops.interior].tocsr()


# ----------------------------------------------------------------------------
# State, QoI, adjoint (the 2D oracle's Newton solver on these operators)
# ----------------------------------------------------------------------------

def extend(ops: Operators3D, u_int: np.ndarray) -> np.ndarray:
    u = np.zeros(ops.prob.n_nodes)
    u[ops.interior] = u_int
    return u


def qoi(ops: Operators3D, u_int: np.ndarray) -> float:
    d = extend(ops, u_int) - ops.t_full
    return float(d @ (ops.M_full @ d))


def qoi_gradient(ops: Operators3D, u_int: np.ndarray) -> np.ndarray:
    d = extend(ops, u_int) - ops.t_full
    return 2.0 * (ops.M_full @ d)[ops.interior]


def solve_sample(ops: Operators3D, xi_i: np.ndarray, z: np.ndarray, want_grad=True, rtol=1e-14, linear="lu"):
    """State u, q and dq/dz = F^T lambda with A(u) lambda = dq/du (Sec. 2.3).
    linear="cg" replaces the LU factors by tight CG solves (large grids)."""
    prob = ops.prob
    K = stiffness(ops, field_nodal(xi_i, prob))
    f = ops.F @ z
    u, lu, iters = fem2d.newton_solve(K, ops.w, prob.reaction, f, rtol=rtol, linear=linear)
    out = {"u": u, "q": qoi(ops, u), "newton_iters": iters, "lu": lu}
    if want_grad:
        lam = lu.solve(qoi_gradient(ops, u))
        out["lam"] = lam
        out["g"] = ops.F.T @ lam
    return out


def control_jacobian(ops: Operators3D, sample: dict) -> np.ndarray:
    """du/dz = A(u)^{-1} F (d_U x d_Z): the d_Z linearised solves with the
    factors of the converged state (Sec. 3.4, eq. (projected_sensitivity))."""
    return sample["lu"].solve(ops.F)
