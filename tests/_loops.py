"""Independent pure-Python loop forms of the paper's difference operators,
used only to pin the oracle (tiny grids).  Zero boundary values are explicit
ghost reads; nothing here is shared with the oracle's sparse assembly."""
import numpy as np


def lap_loops(u):
    """Pure-loop 3-point (1D) or 5-point (2D) Dirichlet Laplacian."""
    n = u.shape[0]
    h2 = (1.0 / (n + 1)) ** 2
    out = np.zeros_like(u)
    if u.ndim == 1:
        for i in range(n):
            l = u[i - 1] if i > 0 else 0.0
            r = u[i + 1] if i < n - 1 else 0.0
            out[i] = (l - 2.0 * u[i] + r) / h2
        return out
    for i in range(n):
        for j in range(n):
            c = u[i, j]
            s = 0.0
            s += u[i - 1, j] if i > 0 else 0.0
            s += u[i + 1, j] if i < n - 1 else 0.0
            s += u[i, j - 1] if j > 0 else 0.0
            s += u[i, j + 1] if j < n - 1 else 0.0
            out[i, j] = (s - 4.0 * c) / h2
    return out


def grad_sq_loops(u):
    """Sum of squared forward differences over every grid edge, boundary
    edges (to the zero values) included, divided by h^2."""
    n = u.shape[0]
    h = 1.0 / (n + 1)
    if u.ndim == 1:
        z = [0.0] + list(u) + [0.0]
        return sum((z[i + 1] - z[i]) ** 2 for i in range(n + 1)) / h ** 2
    z = np.zeros((n + 2, n + 2))
    z[1:-1, 1:-1] = u
    tot = 0.0
    for i in range(n + 2):
        for j in range(n + 1):
            tot += (z[i, j + 1] - z[i, j]) ** 2
    for i in range(n + 1):
        for j in range(n + 2):
            tot += (z[i + 1, j] - z[i, j]) ** 2
    return tot / h ** 2
