"""The host routine for the eigensolver's projected problems (Krylov-Schur
restart, Stage-2 Rayleigh-Ritz): A = Q diag(w) Q^T on matrices of the shapes
those problems take (random, tridiagonal with an arrow row as after a thick
restart, clustered and exactly repeated eigenvalues), on both sides of the
switch from Jacobi (order <= 64) to tridiagonal QR.  Eigenvalues are compared
with LAPACK's (numpy); eigenvectors by residual and orthogonality, since the
basis of a repeated eigenvalue is not unique.  Host only, no GPU."""
import numpy as np
import pytest


def _check(a, tol=1e-13):
    from paper_2507_18282_amd import sym_eig
    n = a.shape[0]
    w, q = sym_eig(a)
    ref = np.linalg.eigvalsh(a)
    scale = max(1.0, float(np.abs(ref).max()))
    assert np.max(np.abs(np.sort(w) - ref)) <= tol * scale * max(1, n) ** 0.5
    assert np.max(np.abs(a @ q - q * w)) <= tol * scale * max(1, n) ** 0.5
    assert np.max(np.abs(q.T @ q - np.eye(n))) <= tol * max(1, n) ** 0.5


@pytest.mark.parametrize("n", [1, 2, 3, 10, 64, 65, 130, 400])
def test_random_symmetric(n):
    rng = np.random.default_rng(n)
    g = rng.standard_normal((n, n))
    _check(0.5 * (g + g.T))


@pytest.mark.parametrize("n", [40, 200])
def test_arrow_tridiagonal_clustered(n):
    # Ritz values after a thick restart: a diagonal block with an arrow row,
    # followed by a tridiagonal tail; eigenvalues clustered near 1
    rng = np.random.default_rng(7)
    a = np.zeros((n, n))
    keep = n // 2
    a[np.arange(keep), np.arange(keep)] = 1.0 - 1e-6 * rng.random(keep)
    a[keep, :keep] = a[:keep, keep] = 1e-4 * rng.standard_normal(keep)
    d = rng.random(n - keep)
    a[np.arange(keep, n), np.arange(keep, n)] = d
    e = 0.1 * rng.standard_normal(n - keep - 1)
    a[np.arange(keep, n - 1), np.arange(keep + 1, n)] = e
    a[np.arange(keep + 1, n), np.arange(keep, n - 1)] = e
    _check(a)


@pytest.mark.parametrize("n", [30, 150])
def test_repeated_eigenvalues(n):
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat(np.arange(n // 3 + 1, dtype=float), 3)[:n]
    _check((q * lam) @ q.T)


def test_diagonal_and_zero():
    _check(np.diag(np.arange(100.0)[::-1]))
    from paper_2507_18282_amd import sym_eig
    w, q = sym_eig(np.zeros((70, 70)))
    assert np.all(w == 0.0) and np.allclose(q.T @ q, np.eye(70))


def test_rejects_bad_order():
    from paper_2507_18282_amd import sym_eig
    with pytest.raises(Exception):
        sym_eig(np.zeros((0, 0)))
