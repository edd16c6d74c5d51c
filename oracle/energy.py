"""Discrete Ginzburg-Landau energy (Section 1, (1.2)):

    E(u) = int F(u) + (eps^2/2) |grad u|^2,  F(u) = (u^2 - 1)^2 / 4.

Discretised on the interior points as
    E_h(u) = h^d sum_i F(u_i) + (eps^2/2) h^d sum_i u_i (-L u)_i,
where the second sum equals the sum of squared forward differences over all
grid edges including those to the zero boundary values (summation by parts).
The paper gives no discrete energy; this is the reading used throughout.
(The convex part of F is printed as u^4/4 + 1 before (2.3); the constant
must be 1/4 for the split to add up to F, which only shifts E.)
"""
from __future__ import annotations

import numpy as np

from .operators import laplacian, mesh_h


def energy(u: np.ndarray, eps: float) -> float:
    n, dim = u.shape[0], u.ndim
    h = mesh_h(n)
    x = u.reshape(-1)
    L = laplacian(n, dim)
    bulk = 0.25 * (x * x - 1.0) ** 2
    grad = x * (-(L @ x))
    return float(h ** dim * np.sum(bulk) + 0.5 * eps * eps * h ** dim * np.sum(grad))
