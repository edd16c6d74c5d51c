"""Pins of the oracle's discrete operators against closed forms and
independent loop code (paper, Section 3: D_h and its eigenvalues)."""
import numpy as np
import pytest

from oracle import operators as ops
from tests._loops import lap_loops


@pytest.mark.parametrize("n", [5, 16, 63, 128])
def test_eigenvalues_match_paper_formula(n):
    # assembled D_h has exactly the eigenvalues of Section 3 (distinct, negative)
    ev = np.sort(np.linalg.eigvalsh(ops.laplacian_1d(n).toarray()))
    lam = np.sort(ops.eigenvalues_paper(n))
    assert np.all(lam < 0) and len(np.unique(np.round(lam, 6))) == n
    assert np.max(np.abs(ev - lam)) <= 1e-12 * np.max(np.abs(lam))


@pytest.mark.parametrize("n", [8, 64, 128])
def test_sine_matrix_diagonalises(n):
    S = ops.sine_matrix(n)
    assert np.max(np.abs(S @ S - np.eye(n))) < 1e-13
    D = ops.laplacian_1d(n).toarray()
    lam = ops.eigenvalues_paper(n)
    assert np.max(np.abs(S @ D @ S - np.diag(lam))) <= 1e-12 * np.max(np.abs(lam))


def test_2d_kronecker_sum_eigenpairs():
    n = 7
    L = ops.laplacian(n, 2).toarray()
    S = ops.sine_matrix(n)
    lam = ops.eigenvalues_paper(n)
    rng = np.random.default_rng(1)
    for _ in range(5):
        p, q = rng.integers(0, n, size=2)
        mode = np.outer(S[:, p], S[:, q])    # [iy, ix]
        out = (L @ mode.reshape(-1)).reshape(n, n)
        assert np.allclose(out, (lam[p] + lam[q]) * mode, rtol=0, atol=1e-10 * abs(lam[p] + lam[q]))


@pytest.mark.parametrize("dim,n", [(1, 9), (2, 6)])
def test_laplacian_matches_loop_stencil(dim, n):
    rng = np.random.default_rng(2)
    u = rng.standard_normal((n,) * dim)
    a = (ops.laplacian(n, dim) @ u.reshape(-1)).reshape(u.shape)
    b = lap_loops(u)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_norm_h():
    n = 31
    x = (np.arange(1, n + 1)) / (n + 1)
    u = np.sin(np.pi * x)
    # h sum sin^2 = 1/2 exactly on this grid
    assert abs(ops.norm_h(u, 1) ** 2 - 0.5) < 1e-14
