"""Fine and coarse propagators (Section 2: F advances one slice of length
dT = T/N with J steps of dt = dT/J; G advances it with coarse steps).

Pairings of Section 2.1: PA-I is F = G = (2.4); PA-II is F = G = (2.5);
PA-III is F = (2.5), G = (2.4); NPA-I is F = (2.3), G = (2.4); NPA-II is
F = G = (2.3).  ``m_coarse`` coarse sub-steps of dT/m are allowed (the paper
uses one).
"""
from __future__ import annotations

import numpy as np

from . import schemes


def fine(prob, u: np.ndarray, steps: int | None = None, route: str = "lu",
         dd_iters: list | None = None) -> np.ndarray:
    """F(T_{n+1}, T_n, u): J steps of the fine scheme with tau = dT/J.
    route "lu": the sparse-LU solves; "sine": the same steps solved in the
    sine basis (faster, equal up to rounding); "mixed": scheme (2.4) solved in
    the mixed form of Section 4 (u and v = -eps^2 L u + u_n^2 u - u_n) by a
    dense solve, a second route to the same step.  With the Neumann-Neumann
    fine step, ``dd_iters`` receives each step's iteration count."""
    J = prob.j_fine if steps is None else steps
    tau = prob.dt
    v = np.array(u, dtype=np.float64, copy=True)
    fast = route == "sine"
    if route not in ("lu", "sine", "mixed") or (route == "mixed" and prob.fine_kind != "approx2"):
        raise ValueError(route)
    for _ in range(J):
        if prob.fine_kind == "linear":
            step = schemes.step_stab_dst if fast else schemes.step_stab
            v = step(v, tau, prob.eps, prob.s_fine, prob.f_zero)
        elif prob.fine_kind == "nonlinear":
            step = schemes.step_newton_pcg if fast else schemes.step_newton
            v = step(v, tau, prob.eps, prob.nl_variant, prob.newton_tol, prob.newton_max,
                     f_zero=prob.f_zero)
        elif prob.fine_kind == "approx2":
            # PA-I: scheme (2.4) as the fine step
            if route == "mixed":
                from . import dd
                v = dd.step_approx2_dd(v, tau, prob.eps, n_sub=1)[0]
            else:
                v = schemes.step_approx2(v, tau, prob.eps, prob.f_zero)
        elif prob.fine_kind == "approx2_dd":
            # PA-I with the Neumann-Neumann solve of (2.4) (Section 4, 1D)
            from . import dd
            if prob.f_zero:
                raise ValueError("the Neumann-Neumann step has no f == 0 form")
            v, it = dd.step_approx2_dd(v, tau, prob.eps, prob.dd_subdomains, prob.dd_theta,
                                       prob.dd_tol, prob.dd_max)
            if dd_iters is not None:
                dd_iters.append(it)
        else:
            raise ValueError(prob.fine_kind)
    return v


def coarse(prob, u: np.ndarray, kind: str | None = None, nn_params=None) -> np.ndarray:
    """G(T_{n+1}, T_n, u): m_coarse steps of tau = dT/m_coarse of scheme (2.4)
    ("approx2"), of the stabilised step ("stab"), of scheme (2.3) by Newton
    ("eyre", NPA-II), or the learned surrogate."""
    kind = prob.coarse_kind if kind is None else kind
    v = np.array(u, dtype=np.float64, copy=True)
    if kind == "neural":
        from . import nn
        base = coarse(prob, v, kind="approx2") if getattr(prob, "nn_base", 0) else None
        return nn.surrogate_step(nn_params, v, base)
    m = prob.m_coarse
    tau = prob.dT / m
    for _ in range(m):
        if kind == "approx2":
            v = schemes.step_approx2(v, tau, prob.eps, prob.f_zero)
        elif kind == "stab":
            v = schemes.step_stab(v, tau, prob.eps, prob.s_fine, prob.f_zero)
        elif kind == "eyre":
            v = schemes.step_newton(v, tau, prob.eps, "eyre", prob.newton_tol, prob.newton_max,
                                    prob.f_zero)
        else:
            raise ValueError(kind)
    return v


def fine_sequential(prob, u0: np.ndarray) -> list:
    """The serial fine solution at every T_n: [u0, F(u0), F(F(u0)), ...]."""
    out = [np.array(u0, dtype=np.float64, copy=True)]
    for _ in range(prob.n_slices):
        out.append(fine(prob, out[-1]))
    return out
