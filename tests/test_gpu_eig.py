"""The library's GPU symmetric eigensolver (parallel cyclic Jacobi, used for
the POD Gram matrix, Sec. 3.3) against numpy's LAPACK eigh and exact
invariants: eigenvalues, residuals A V = V diag(w), orthonormality; odd n
(a padded dummy index), a rank-deficient Gram matrix with a rapidly
decaying spectrum, repeated eigenvalues."""
import numpy as np
import pytest
import torch

import paper_2305_20053_amd as saa

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (301, 4)])
def test_random_symmetric(gpu_lib, n, seed):
    print(f"case eig n={n}", flush=True)
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A + A.T
    w, V, sweeps = saa.sym_eig_gpu(torch.from_numpy(A).cuda())
    V = V.cpu().numpy()
    ref = np.linalg.eigvalsh(A)[::-1]
    scale = max(1.0, np.abs(ref).max())
    np.testing.assert_allclose(w, ref, atol=1e-12 * scale * max(1, n / 64))
    np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-12 * max(n, 8))
    np.testing.assert_allclose(A @ V, V * w, atol=1e-11 * scale * max(1, n / 64))
    assert sweeps <= 15


def test_gram_matrix_with_clustered_spectrum(gpu_lib):
    rng = np.random.default_rng(7)
    basis = np.linalg.qr(rng.standard_normal((400, 30)))[0]
    coef = rng.standard_normal((30, 120)) * (10.0 ** -np.arange(30) / 3)[:, None]
    D = basis @ coef
    G = D.T @ D
    w, V, _ = saa.sym_eig_gpu(torch.from_numpy(G).cuda())
    V = V.cpu().numpy()
    ref = np.linalg.eigvalsh(G)[::-1]
    np.testing.assert_allclose(w, ref, atol=1e-13 * ref[0])
    np.testing.assert_allclose(V.T @ V, np.eye(120), atol=1e-11)
    _, Vr = np.linalg.eigh(G)
    Vr = Vr[:, ::-1]
    for c in range(5):                      # well-separated leading eigenvectors, up to sign
        assert abs(abs(V[:, c] @ Vr[:, c]) - 1.0) < 1e-9
    # agrees with the host solver
    wh, _ = saa.sym_eig(G)
    np.testing.assert_allclose(w, wh, atol=1e-13 * ref[0])


def test_diagonal_and_repeated(gpu_lib):
    A = np.diag([3.0, 1.0, 3.0, -2.0])
    w, V, sweeps = saa.sym_eig_gpu(torch.from_numpy(A).cuda())
    np.testing.assert_allclose(w, [3.0, 3.0, 1.0, -2.0], atol=1e-15)
    np.testing.assert_allclose(np.abs(V.cpu().numpy().T @ V.cpu().numpy()), np.eye(4), atol=1e-14)
    assert sweeps == 0


def test_rejects_bad_input(gpu_lib):
    lib = saa.lib()
    w = np.zeros(2)
    assert lib.saa_sym_eig_gpu(0, None, w.ctypes.data, None, None, None) == saa.SAA_E_INVALID
