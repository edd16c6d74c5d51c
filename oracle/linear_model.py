"""The linearised propagators and convergence bound of Section 3.

With diag(W^n)^2 ~ I the fine and coarse steps of (2.4) and (2.5) become
linear maps (Section 3, operator forms of F and G):
    P_i     = (I - i dT D_h + eps^2 dT D_h^2)^{-1} (I - i dT D_h),
    P_{J_i} = [ (I - i dT/J D_h + eps^2 dT/J D_h^2)^{-1} (I - i dT/J D_h) ]^J.
Theorems 3.7/3.9/3.11 bound the Parareal error by
    max_j ||E_j^{k}|| <= alpha^k min{ ((1-beta^{N-1})/(1-beta))^k, binom(N-1, k) } max_j ||E_j^0||
with alpha = ||P_J - P|| and beta = ||P|| (2-norms); Lemma 3.5 gives the
min{...} factor as the bound on the infinity norm of T(beta)^k.
"""
from __future__ import annotations

import math

import numpy as np

from .operators import laplacian


def propagator_matrix(n: int, dim: int, tau: float, eps: float, i: float,
                      power: int = 1) -> np.ndarray:
    """[(I - i tau L + eps^2 tau L^2)^{-1} (I - i tau L)]^power, dense."""
    L = laplacian(n, dim).toarray()
    eye = np.eye(L.shape[0])
    step = np.linalg.solve(eye - i * tau * L + eps * eps * tau * (L @ L), eye - i * tau * L)
    return np.linalg.matrix_power(step, power)


def alpha_beta(n: int, dim: int, dT: float, J: int, eps: float, i_fine: float,
               i_coarse: float) -> tuple:
    PJ = propagator_matrix(n, dim, dT / J, eps, i_fine, J)
    P = propagator_matrix(n, dim, dT, eps, i_coarse, 1)
    return float(np.linalg.norm(PJ - P, 2)), float(np.linalg.norm(P, 2))


def toeplitz_T(beta: float, N: int) -> np.ndarray:
    """T(beta) of Lemma 3.4: strictly lower triangular Toeplitz, first column
    (0, 1, beta, beta^2, ...)."""
    T = np.zeros((N, N))
    for i in range(1, N):
        for j in range(0, i):
            T[i, j] = beta ** (i - j - 1)
    return T


def bound_factor(alpha: float, beta: float, N: int, k: int) -> float:
    """alpha^k min{((1 - beta^{N-1})/(1 - beta))^k, binom(N-1, k)}."""
    geo = ((1.0 - beta ** (N - 1)) / (1.0 - beta)) ** k
    return alpha ** k * min(geo, math.comb(N - 1, k))
