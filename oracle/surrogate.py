"""MR-DINO surrogate evaluated in float64 (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Architecture, paper Sec. 3.3 eq. (rbnet):
    u_w(m, z) = Phi phi_w(m_r, z) + b,   m_r = Psi^T m,
with Psi the leading KL modes of the input field (Sec. 3.3, PCA/KLE basis)
and Phi an M-orthonormal POD basis of the state, b = mean state.

Readings:
  * encoder: the field is an explicit sine KL sum, so the KL coordinates are
    the xi themselves; the r_m leading modes are those of largest amplitude
    a_jk, i.e. smallest j^2 + k^2, ties broken by lexicographic (j, k).
    Whitened coordinates (xi, unit variance) are used.
  * phi_w: dense MLP with GELU (erf form) on every hidden layer and a linear
    output layer; input [m_r; z].
  * QoI: for the quadratic tracking Q the reduced evaluation of Sec. 3.3
    (Q(u_w) = phi^T W_r phi for b = 0) becomes, with the bias and target,
    q = ||phi + c||^2 + c0, c = Phi^T (M (b - u_target))_I,
    c0 = ||b - u_target||_M^2 - ||c||^2  (exact when Phi^T M Phi = I).
  * dq/dz by reverse mode (VJP) of the network (Sec. 3.1,
    eq. (neural_operator_gradient)); dphi/dz by forward mode (JVP).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erf


def kl_order(kl_per_dim: int, dim: int = 2) -> list[tuple]:
    """Mode multi-indices (1-based) sorted by |k|^2, ties lexicographic."""
    rng = range(1, kl_per_dim + 1)
    if dim == 2:
        idx = [(j, k) for j in rng for k in rng]
    else:
        idx = [(j, k, l) for j in rng for k in rng for l in rng]
    return sorted(idx, key=lambda t: (sum(v * v for v in t), t))


def encode(xi: np.ndarray, r_m: int) -> np.ndarray:
    """(N, K1, K1[, K1]) KL coefficients -> (N, r_m) leading whitened coordinates."""
    dim = xi.ndim - 1
    order = kl_order(xi.shape[1], dim)[:r_m]
    cols = [xi[(slice(None),) + tuple(v - 1 for v in t)] for t in order]
    return np.stack(cols, axis=1)


def encode_from_nodal(m_nodal: np.ndarray, n: int, amplitudes: np.ndarray, r_m: int) -> np.ndarray:
    """Recover the leading xi from nodal values of m on the (n+1)^2 grid by
    discrete sine orthogonality: for 1 <= j, k < n,
    sum_{interior p} sin(j pi x_p) sin(k' pi x_p) = (n/2) delta_{jk'}, so
    xi_jk = (4/n^2) sum_p m(x_p) sin(j pi x_p) sin(k pi y_p) / a_jk."""
    K1 = amplitudes.shape[0]
    order = kl_order(K1, 2)[:r_m]
    t = np.arange(n + 1) / n
    grid = m_nodal.reshape(n + 1, n + 1)          # [y, x]
    out = np.empty(r_m)
    for c, (j, k) in enumerate(order):
        s = (grid * np.outer(np.sin(k * np.pi * t), np.sin(j * np.pi * t))).sum()
        out[c] = 4.0 / n ** 2 * s / amplitudes[j - 1, k - 1]
    return out


# ----------------------------------------------------------------------------
# GELU and its derivatives
# ----------------------------------------------------------------------------

def _npdf(a):
    return np.exp(-0.5 * a * a) / np.sqrt(2.0 * np.pi)


def gelu(a):
    """a Phi_N(a) = a/2 (1 + erf(a / sqrt 2))."""
    return 0.5 * a * (1.0 + erf(a / np.sqrt(2.0)))


def dgelu(a):
    """Phi_N(a) + a phi_N(a)."""
    return 0.5 * (1.0 + erf(a / np.sqrt(2.0))) + a * _npdf(a)


def d2gelu(a):
    """phi_N(a) (2 - a^2)."""
    return _npdf(a) * (2.0 - a * a)


# ----------------------------------------------------------------------------
# Network
# ----------------------------------------------------------------------------

@dataclass
class Surrogate:
    layers: list          # [(W_l (out x in), b_l)], hidden layers GELU, last linear
    r_m: int
    d_z: int
    c: np.ndarray         # (r_u,)
    c0: float


def forward(layers, x):
    """x: (B, r_m + d_Z). Returns phi (B, r_u) and the pre-activations a_l and
    activations h_l (h_0 = x) of the hidden layers."""
    h = [x]
    a = []
    for W, b in layers[:-1]:
        a.append(h[-1] @ W.T + b)
        h.append(gelu(a[-1]))
    W, b = layers[-1]
    return h[-1] @ W.T + b, a, h


def reduced_qoi(phi, c, c0):
    return np.sum((phi + c) ** 2, axis=1) + c0


def qoi_and_grad(model: Surrogate, xhat: np.ndarray, z: np.ndarray):
    """q (B,) and dq/dz (B, d_Z) at x = [xhat; z] (reverse mode)."""
    bsz = xhat.shape[0]
    x = np.concatenate([xhat, np.broadcast_to(z, (bsz, model.d_z))], axis=1)
    phi, a, h = forward(model.layers, x)
    q = reduced_qoi(phi, model.c, model.c0)
    delta = 2.0 * (phi + model.c)                 # dq/dphi
    W, _ = model.layers[-1]
    gh = delta @ W
    for l in range(len(model.layers) - 2, -1, -1):
        ga = dgelu(a[l]) * gh
        W, _ = model.layers[l]
        gh = ga @ W
    return q, gh[:, model.r_m:]


def jacobian_z(layers, x, r_m):
    """dphi/dz (B, r_u, d_Z) by forward mode: tangents J_0 = [0; I]."""
    phi, a, h = forward(layers, x)
    W1, _ = layers[0]
    JA = np.broadcast_to(W1[:, r_m:], (x.shape[0],) + W1[:, r_m:].shape)
    JH = dgelu(a[0])[:, :, None] * JA
    for l in range(1, len(layers) - 1):
        W, _ = layers[l]
        JA = np.einsum("oi,bik->bok", W, JH)
        JH = dgelu(a[l])[:, :, None] * JA
    W, _ = layers[-1]
    return phi, np.einsum("oi,bik->bok", W, JH)


def decode(Phi, ubar, phi):
    """u_w = Phi phi + b on the unknowns (Sec. 3.3, eq. (rbnet))."""
    return phi @ Phi.T + ubar
