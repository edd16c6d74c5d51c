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

``step_stab_dst`` and ``step_newton_pcg`` are faster routes to the same steps
(sine-basis solves), pinned to the sparse-LU routes by the CPU tests.
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


# ------------------------------------------------------------------ fast routes
# The same steps solved in the sine eigenbasis of L (Section 3: L = S diag(lam) S
# with S the orthonormal sine matrix, S = S^T = S^{-1}); the transforms are dense
# products with S.  They reach the results of the sparse-LU routes above up to
# rounding (CPU tests pin them to those) and make full-length runs at 256^2
# affordable: a sparse LU solve there costs 0.15 s (linear step) to 8 s (Newton
# step), a pair of dense transforms about 2 ms.

@functools.lru_cache(maxsize=16)
def _sine_basis(n: int, dim: int):
    from .operators import eigenvalues_paper, sine_matrix
    S = sine_matrix(n)
    lam = eigenvalues_paper(n)
    Lam = lam if dim == 1 else lam[:, None] + lam[None, :]
    return S, Lam


def _to_sine(x: np.ndarray, S: np.ndarray, transform: str = "dense") -> np.ndarray:
    """Sine-basis coefficients of a grid function (1D: S x; 2D: S X S).
    transform "dense": products with S; "fft": scipy's orthonormal DST-I (the
    same map, computed through an FFT, so rounded differently)."""
    if transform == "fft":
        import scipy.fft
        return scipy.fft.dstn(x, type=1, norm="ortho", workers=8)
    return S @ x if x.ndim == 1 else S @ x @ S


def step_stab_dst(u: np.ndarray, tau: float, eps: float, s: float = 2.0,
                  f_zero: bool = False, transform: str = "dense") -> np.ndarray:
    """step_stab solved in the sine basis: I + tau eps^2 L^2 - s tau L has the
    eigenvalues sigma = 1 + tau eps^2 Lam^2 - s tau Lam on the sine modes, so
    v = S^{-1}((S r) / sigma) with the same right-hand side r."""
    n, dim = u.shape[0], u.ndim
    L = laplacian(n, dim)
    S, Lam = _sine_basis(n, dim)
    x = u.reshape(-1)
    fx = np.zeros_like(x) if f_zero else f(x)
    rhs = (x + tau * (L @ (fx - s * x))).reshape(u.shape)
    sigma = 1.0 + tau * eps * eps * Lam * Lam - s * tau * Lam
    return _to_sine(_to_sine(rhs, S, transform) / sigma, S, transform)


def pcg(apply_K, apply_Minv, b: np.ndarray, x0: np.ndarray, rtol: float, maxit: int):
    """Textbook preconditioned conjugate gradients for an SPD operator K,
    from x0, stopped when the preconditioned residual is small:
    r.M^{-1}r <= rtol^2 b.M^{-1}b (recursive residual r).  With M close to K
    this bounds the error in the K-norm; the plain ||r|| <= rtol ||b|| would
    leave errors some 50 rtol here, where K spans several orders of magnitude."""
    x = x0.copy()
    r = b - apply_K(x)
    z = apply_Minv(r)
    rz = float(np.vdot(r, z))
    stop = rtol * rtol * float(np.vdot(b, apply_Minv(b)))
    if rz <= stop:
        return x, 0
    p = z.copy()
    for it in range(1, maxit + 1):
        Kp = apply_K(p)
        alpha = rz / float(np.vdot(p, Kp))
        x += alpha * p
        r -= alpha * Kp
        z = apply_Minv(r)
        rz_new = float(np.vdot(r, z))
        if rz_new <= stop:
            return x, it
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise NoConvergence(f"PCG did not reach {rtol} in {maxit} iterations")


def step_newton_pcg(u: np.ndarray, tau: float, eps: float, variant: str = "eyre",
                    tol: float = 1e-10, maxit: int = 20, cg_rtol: float = 1e-14,
                    cg_maxit: int = 1000, s_pc: float = 3.0, f_zero: bool = False,
                    history: list | None = None, transform: str = "dense") -> np.ndarray:
    """step_newton with each Newton system J y = rhs solved by PCG.

    Same iteration and stop as step_newton: J = I + eps^2 tau L^2 - tau L diag(q),
    q = 3 Y_m^2 (Eyre) or 3 Y_m^2 - 1 (backward Euler), rhs as there.  With the
    SPD A = -L, J = I + eps^2 tau A^2 + tau A diag(q), and A^{-1} J = A^{-1} +
    eps^2 tau A + tau diag(q) is symmetric positive definite (for the backward
    Euler form when tau < 4 eps^2).  So A^{-1} J y = A^{-1} rhs is solved by PCG
    from Y_m, preconditioned by A^{-1} + eps^2 tau A + tau s_pc I, which is
    diagonal on the sine modes (mu = -Lam)."""
    n, dim = u.shape[0], u.ndim
    h = mesh_h(n)
    L = laplacian(n, dim)
    S, Lam = _sine_basis(n, dim)
    mu = -Lam
    shp = u.shape
    x = u.reshape(-1)
    tr = lambda v: _to_sine(v, S, transform)
    Ainv = lambda v: tr(tr(v.reshape(shp)) / mu).reshape(-1)
    if f_zero:
        return step_stab_dst(u, tau, eps, 0.0, f_zero=True)
    if variant == "eyre":
        yhat = x - tau * (L @ x)
        shift = 0.0
    elif variant == "be":
        yhat = x.copy()
        shift = -1.0
    else:
        raise ValueError(variant)
    pre = 1.0 / mu + eps * eps * tau * mu + tau * s_pc
    Minv = lambda v: tr(tr(v.reshape(shp)) / pre).reshape(-1)
    y = x.copy()
    for _ in range(maxit):
        q = 3.0 * y * y + shift
        K = lambda v, q=q: Ainv(v) - eps * eps * tau * (L @ v) + tau * q * v
        rhs = yhat - 2.0 * tau * (L @ (y * y * y))
        y_new, _ = pcg(K, Minv, Ainv(rhs), y, cg_rtol, cg_maxit)
        d = float(np.sqrt(h ** dim * np.sum((y_new - y) ** 2)))
        if history is not None:
            history.append(d)
        y = y_new
        if d <= tol:
            return y.reshape(shp)
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
