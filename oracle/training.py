"""Reduced bases and derivative-informed training (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Weighted POD (Sec. 3.3): eigenvectors of E[(u - ubar)(u - ubar)^T] in the
  M inner product, computed by the method of snapshots: G = D^T M D with
  D = [u_1 - ubar, ...], G V = V Lambda, Phi = D V_r Lambda_r^{-1/2}, so that
  Phi^T M Phi = I.  Columns of V are signed so that their entry of largest
  magnitude is positive.
* DINO loss in the reduced output space (Sec. 3.4,
  eq. (reduced_basis_derivative_equivalence)), averaged over the batch:
    L = 1/B sum_b ||phi_b - y_b||^2 + ||dphi_b/dz - Jy_b||_F^2,
  with y = Phi^T M (u - ubar) and Jy = Phi^T M du/dz; dropping the second
  term gives the L2-only (MR-NO) loss of eq. (no_exp_risk_min).
* Its gradient with respect to every weight and bias, derived by hand
  through the forward-mode tangent recurrence (needs GELU'').
* Adam (the optimiser named in Sec. 4.2.1).
"""
from __future__ import annotations

import numpy as np

from .surrogate import d2gelu, dgelu, forward, gelu


def pod(U: np.ndarray, M, r: int):
    """U: (N_s, d) snapshots (rows), M: (d, d) SPD.  Returns (ubar, Phi (d, r),
    eigenvalues of G in decreasing order (all N_s))."""
    ubar = U.mean(axis=0)
    D = (U - ubar).T                                  # d x N_s
    G = D.T @ (M @ D)
    G = 0.5 * (G + G.T)
    lam, V = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    Vr = V[:, :r].copy()
    piv = np.argmax(np.abs(Vr), axis=0)
    Vr *= np.sign(Vr[piv, np.arange(r)])
    Phi = D @ Vr / np.sqrt(lam[:r])
    return ubar, Phi, lam


def project(Phi, M, ubar, U):
    """y_i = Phi^T M (u_i - ubar) for rows of U."""
    return (U - ubar) @ (M @ Phi)


def loss(layers, x, y, jy, r_m, dino=True):
    """Batch-mean DINO (or L2-only) loss."""
    phi, a, h = forward(layers, x)
    bsz = x.shape[0]
    val = np.sum((phi - y) ** 2)
    if dino:
        W1, _ = layers[0]
        JH = dgelu(a[0])[:, :, None] * W1[None, :, r_m:]
        for l in range(1, len(layers) - 1):
            JH = dgelu(a[l])[:, :, None] * np.einsum("oi,bik->bok", layers[l][0], JH)
        jphi = np.einsum("oi,bik->bok", layers[-1][0], JH)
        val += np.sum((jphi - jy) ** 2)
    return val / bsz


def loss_and_grad(layers, x, y, jy, r_m, dino=True):
    """Loss and its gradient [(dW_l, db_l)] by a hand-derived backward pass.

    Forward: a_l = W_l h_{l-1} + b_l, h_l = s(a_l) (l < L), phi = W_L h_{L-1} + b_L.
    Tangents: JA_1 = W_1[:, r_m:], JH_l = s'(a_l) * JA_l, JA_l = W_l JH_{l-1},
    Jphi = W_L JH_{L-1}.
    Backward, with adjoints gH_l = dL/dh_l, gJH_l = dL/dJH_l:
      gJA_l = s'(a_l) * gJH_l
      gA_l  = s'(a_l) * gH_l + s''(a_l) * sum_k gJH_l[:, k] JA_l[:, k]
      dW_l  = gA_l h_{l-1}^T + gJA_l JH_{l-1}^T     (l >= 2)
      dW_1  = gA_1 x^T,  dW_1[:, r_m:] += sum_b gJA_1
      gH_{l-1} = W_l^T gA_l,  gJH_{l-1} = W_l^T gJA_l.
    """
    L = len(layers)
    bsz = x.shape[0]
    phi, a, h = forward(layers, x)
    JA, JH = [], []
    if dino:
        W1, _ = layers[0]
        JA.append(np.broadcast_to(W1[:, r_m:], (bsz,) + W1[:, r_m:].shape))
        JH.append(dgelu(a[0])[:, :, None] * JA[0])
        for l in range(1, L - 1):
            JA.append(np.einsum("oi,bik->bok", layers[l][0], JH[-1]))
            JH.append(dgelu(a[l])[:, :, None] * JA[-1])
        jphi = np.einsum("oi,bik->bok", layers[-1][0], JH[-1])
    e = phi - y
    val = np.sum(e ** 2)
    if dino:
        ej = jphi - jy
        val += np.sum(ej ** 2)
    val /= bsz

    grads = [None] * L
    g_out = 2.0 * e / bsz
    WL = layers[-1][0]
    dW = g_out.T @ h[-1]
    if dino:
        gj_out = 2.0 * ej / bsz
        dW = dW + np.einsum("bok,bik->oi", gj_out, JH[-1])
        gJH = np.einsum("bok,oi->bik", gj_out, WL)
    grads[-1] = (dW, g_out.sum(axis=0))
    gH = g_out @ WL
    for l in range(L - 2, -1, -1):
        s1 = dgelu(a[l])
        gA = s1 * gH
        if dino:
            gJA = s1[:, :, None] * gJH
            gA = gA + d2gelu(a[l]) * np.sum(gJH * JA[l], axis=2)
        W = layers[l][0]
        dW = gA.T @ h[l]
        if dino:
            if l >= 1:
                dW = dW + np.einsum("bok,bik->oi", gJA, JH[l - 1])
            else:
                dW = dW.copy()
                dW[:, r_m:] += gJA.sum(axis=0)
        grads[l] = (dW, gA.sum(axis=0))
        if l > 0:
            gH = gA @ W
            if dino:
                gJH = np.einsum("bok,oi->bik", gJA, W)
    return val, grads


def flatten(layers) -> np.ndarray:
    """Pack [(W_l, b_l)] as W_1 (row-major), b_1, W_2, b_2, ..."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def unflatten(vec: np.ndarray, widths: list[int]):
    layers, off = [], 0
    for fi, fo in zip(widths[:-1], widths[1:]):
        W = vec[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = vec[off:off + fo]
        off += fo
        layers.append((W, b))
    return layers


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the flat parameter vector (step counts from 1).
    Returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


__all__ = ["pod", "project", "loss", "loss_and_grad", "flatten", "unflatten",
           "adam_step", "gelu"]
