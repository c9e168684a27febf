"""The library's host symmetric eigensolver (POD Gram matrices) against
numpy's LAPACK eigh and exact invariants (no GPU)."""
import numpy as np
import pytest

import paper_2305_20053_amd as saa


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (300, 4)])
def test_random_symmetric(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A + A.T
    w, V = saa.sym_eig(A)
    ref = np.linalg.eigvalsh(A)[::-1]
    np.testing.assert_allclose(w, ref, atol=1e-12 * max(1.0, np.abs(ref).max()))
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-12 * n)
    np.testing.assert_allclose(A @ V, V * w, atol=1e-11 * max(1.0, np.abs(ref).max()))


def test_gram_matrix_with_clustered_spectrum():
    """Gram matrices of snapshots: positive semidefinite, rapidly decaying
    spectrum, rank deficiency (zero eigenvalues)."""
    rng = np.random.default_rng(7)
    basis = np.linalg.qr(rng.standard_normal((400, 30)))[0]
    coef = rng.standard_normal((30, 120)) * (10.0 ** -np.arange(30) / 3)[:, None]
    D = basis @ coef
    G = D.T @ D
    w, V = saa.sym_eig(G)
    ref = np.linalg.eigvalsh(G)[::-1]
    np.testing.assert_allclose(w, ref, atol=1e-13 * ref[0])
    assert np.all(np.diff(w) <= 1e-14 * w[0])
    np.testing.assert_allclose(V.T @ V, np.eye(120), atol=1e-11)
    # well-separated leading eigenvectors (gap >= 1e-6 |G|) match up to sign
    _, Vr = np.linalg.eigh(G)
    Vr = Vr[:, ::-1]
    for c in range(5):
        assert abs(abs(V[:, c] @ Vr[:, c]) - 1.0) < 1e-9


def test_diagonal_and_repeated():
    A = np.diag([3.0, 1.0, 3.0, -2.0])
    w, V = saa.sym_eig(A)
    np.testing.assert_allclose(w, [3.0, 3.0, 1.0, -2.0], atol=1e-15)
    np.testing.assert_allclose(np.abs(V.T @ V), np.eye(4), atol=1e-14)


def test_rejects_bad_input():
    lib = saa.lib()
    assert lib.saa_sym_eig(0, None, None, None) == saa.SAA_E_INVALID
    A = np.array([[np.nan]])
    w = np.zeros(1); V = np.zeros((1, 1))
    assert lib.saa_sym_eig(1, A.ctypes.data, w.ctypes.data, V.ctypes.data) == saa.SAA_E_INVALID
