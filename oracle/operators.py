"""Discrete operators (paper, Section 3: the matrix D_h and its eigenvalues;
Section 3 closing remark, item 2: natural extension to 2D).

Grid: n interior points per dimension on (0,1), h = 1/(n+1); the unknowns are
the interior values only (Section 2.1: u(jh) for the interior nodes), the
boundary values are zero.  2D arrays are row-major, index [iy, ix].
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp


def mesh_h(n: int) -> float:
    return 1.0 / (n + 1)


@functools.lru_cache(maxsize=None)
def laplacian_1d(n: int) -> sp.csr_matrix:
    """D_h = (1/h^2) tridiag(1, -2, 1) of size n (Section 3, the D_h matrix)."""
    h = mesh_h(n)
    e = np.ones(n)
    return (sp.diags([e[:-1], -2.0 * e, e[:-1]], [-1, 0, 1]) / (h * h)).tocsr()


@functools.lru_cache(maxsize=None)
def laplacian(n: int, dim: int) -> sp.csr_matrix:
    """Dirichlet Laplacian on n^dim interior points.

    1D: D_h.  2D: the Kronecker sum D_h (x) I + I (x) D_h acting on the
    row-major flattening (x fastest), the natural 2D extension.
    """
    d1 = laplacian_1d(n)
    if dim == 1:
        return d1
    if dim == 2:
        eye = sp.identity(n, format="csr")
        return (sp.kron(eye, d1) + sp.kron(d1, eye)).tocsr()
    raise ValueError("dim must be 1 or 2")


def eigenvalues_paper(n: int) -> np.ndarray:
    """lambda_p = (2/h^2)(cos(p pi/(N_x - 1)) - 1), p = 1..N_x-2 (Section 3),
    with N_x - 1 = n + 1 intervals."""
    h = mesh_h(n)
    p = np.arange(1, n + 1)
    return (2.0 / (h * h)) * (np.cos(p * np.pi / (n + 1)) - 1.0)


def sine_matrix(n: int) -> np.ndarray:
    """Orthonormal eigenvectors of D_h: S[j,k] = sqrt(2/(n+1)) sin(j k pi/(n+1))."""
    j = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))


def norm_h(v: np.ndarray, dim: int) -> float:
    """Discrete L2(Omega) norm sqrt(h^d sum v^2) (the L2 norm used in Section 4)."""
    n = v.shape[0]
    return float(np.sqrt(mesh_h(n) ** dim * np.sum(np.asarray(v, dtype=np.float64) ** 2)))
