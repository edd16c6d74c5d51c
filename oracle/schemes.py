"""One time step of each scheme of Section 2.1, written as the linear or
nonlinear algebraic system the paper states, solved with sparse LU.

f(u) = u^3 - u is F'(u) for F(u) = (u^2 - 1)^2 / 4 (Section 1, after (1.2)).
L denotes the Dirichlet Laplacian D_h (or its 2D Kronecker sum).

Readings of the paper taken here (each listed in the design notes):
  * (2.5): the implicit convex term is written without D_h in the text; the
    operator form of Section 3 (the P_2 propagators) has it, so the step is
    (I + tau eps^2 L^2 - 2 tau L) v = u + tau L (u^3 - 3u).  With a general
    stabilisation constant s this is
    (I + tau eps^2 L^2 - s tau L) v = u + tau L (f(u) - s u)   ("stab" step).
  * (2.3) is solved by Newton's method in the form the paper derives for H(Y)
    (Section 3, NPA-II): (I + eps^2 tau L^2 - 3 tau L diag(Y_m^2)) Y_{m+1}
    = Yhat - 2 tau L Y_m^3, Yhat = (I - tau L) u, from Y_0 = u, stopped when
    ||Y_{m+1} - Y_m||_h <= tol, returning Y_{m+1}.
  * the fully implicit backward-Euler variant replaces Y^3 by f(Y) = Y^3 - Y
    inside L and keeps Yhat = u; its Newton form is
    (I + eps^2 tau L^2 - tau L diag(3 Y_m^2 - 1)) Y_{m+1} = u - 2 tau L Y_m^3.
  * ``f_zero`` (a test hook) sets f == 0: both the cubic and the -u parts vanish.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import laplacian, mesh_h


def f(u: np.ndarray) -> np.ndarray:
    """f(u) = F'(u) = u^3 - u (Section 1)."""
    return u * u * u - u


class NoConvergence(RuntimeError):
    pass


@functools.lru_cache(maxsize=64)
def _stab_factor(n: int, dim: int, tau: float, eps: float, s: float):
    L = laplacian(n, dim)
    eye = sp.identity(n ** dim, format="csc")
    M = (eye + (tau * eps * eps) * (L @ L) - (s * tau) * L).tocsc()
    return spla.splu(M)


def step_stab(u: np.ndarray, tau: float, eps: float, s: float = 2.0,
              f_zero: bool = False) -> np.ndarray:
    """Linear stabilised semi-implicit step; s = 2 is scheme (2.5).

    (I + tau eps^2 L^2 - s tau L) v = u + tau L (f(u) - s u).
    """
    n, dim = u.shape[0], u.ndim
    L = laplacian(n, dim)
    x = u.reshape(-1)
    fx = np.zeros_like(x) if f_zero else f(x)
    rhs = x + tau * (L @ (fx - s * x))
    v = _stab_factor(n, dim, float(tau), float(eps), float(s)).solve(rhs)
    return v.reshape(u.shape)


def step_approx2(u: np.ndarray, tau: float, eps: float,
                 f_zero: bool = False) -> np.ndarray:
    """Linearised Eyre step (2.4): (u^n)^3 -> (u^n)^2 u^{n+1},

    (I - tau L diag(u^2) + eps^2 tau L^2) v = (I - tau L) u.
    """
    n, dim = u.shape[0], u.ndim
    L = laplacian(n, dim)
    x = u.reshape(-1)
    eye = sp.identity(n ** dim, format="csc")
    if f_zero:
        M = (eye + (eps * eps * tau) * (L @ L)).tocsc()
        rhs = x.copy()
    else:
        M = (eye - tau * (L @ sp.diags(x * x)) + (eps * eps * tau) * (L @ L)).tocsc()
        rhs = x - tau * (L @ x)
    return spla.spsolve(M, rhs).reshape(u.shape)


def step_newton(u: np.ndarray, tau: float, eps: float, variant: str = "eyre",
                tol: float = 1e-10, maxit: int = 20, f_zero: bool = False,
                history: list | None = None) -> np.ndarray:
    """Implicit step solved by Newton's method.

    variant "eyre": scheme (2.3), H(Y) = Y + eps^2 tau L^2 Y - tau L Y^3 - (I - tau L) u.
    variant "be":   H(Y) = Y + eps^2 tau L^2 Y - tau L (Y^3 - Y) - u.
    Stops when ||Y_{m+1} - Y_m||_h <= tol and returns Y_{m+1}; ``history``
    (optional) receives the step norms.
    """
    n, dim = u.shape[0], u.ndim
    h = mesh_h(n)
    L = laplacian(n, dim)
    eye = sp.identity(n ** dim, format="csc")
    L2 = (L @ L).tocsc()
    x = u.reshape(-1)
    if f_zero:
        # f == 0: H(Y) = Y + eps^2 tau L^2 Y - u, a single linear solve.
        y = spla.spsolve((eye + (eps * eps * tau) * L2).tocsc(), x)
        return y.reshape(u.shape)
    if variant == "eyre":
        yhat = x - tau * (L @ x)
        lin = 3.0
        shift = 0.0
    elif variant == "be":
        yhat = x.copy()
        lin = 3.0
        shift = -1.0
    else:
        raise ValueError(variant)
    y = x.copy()
    for _ in range(maxit):
        q = lin * y * y + shift
        Jm = (eye + (eps * eps * tau) * L2 - tau * (L @ sp.diags(q))).tocsc()
        rhs = yhat - 2.0 * tau * (L @ (y * y * y))
        y_new = spla.spsolve(Jm, rhs)
        d = float(np.sqrt(h ** dim * np.sum((y_new - y) ** 2)))
        if history is not None:
            history.append(d)
        y = y_new
        if d <= tol:
            return y.reshape(u.shape)
    raise NoConvergence(f"Newton did not reach {tol} in {maxit} iterations")


def newton_residual(y: np.ndarray, u: np.ndarray, tau: float, eps: float,
                    variant: str = "eyre") -> np.ndarray:
    """H(Y) of the implicit step (for checks)."""
    n, dim = u.shape[0], u.ndim
    L = laplacian(n, dim)
    Y = y.reshape(-1)
    x = u.reshape(-1)
    LY = L @ Y
    if variant == "eyre":
        return (Y + eps * eps * tau * (L @ LY) - tau * (L @ (Y ** 3)) - (x - tau * (L @ x))).reshape(u.shape)
    return (Y + eps * eps * tau * (L @ LY) - tau * (L @ (Y ** 3 - Y)) - x).reshape(u.shape)
