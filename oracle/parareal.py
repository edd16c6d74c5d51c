"""The Parareal predictor-corrector iteration (2.2) of Section 2.

    U_0^{k+1} = u0,
    U_{n+1}^{k+1} = G(U_n^{k+1}) + F(U_n^k) - G(U_n^k),

started from the coarse prediction U_{n+1}^0 = G(U_n^0) (Section 2).  The
fine values F(U_n^k) of one iteration are independent over n (the paper's
"N processors"); the coarse sweep is sequential in n.

Readings taken here:
  * the correction is evaluated as F_n + (g - G_old_n): the paper fixes no
    rounding order, and this order makes a converged slice reproduce the
    sequential fine value bit for bit (g == G_old_n gives an exact zero).
  * the update norm is delta^{k+1} = max_n ||U_n^{k+1} - U_n^k||_h (the
    L^inf(0,T; L^2) norm of Section 4 evaluated at the T_n); the iteration
    stops when delta < tol or after N iterations (finite termination,
    Theorem 3.7 proof).
  * a learned coarse propagator falls back to the plain one once the update
    norm stops contracting (delta^{k+1} >= delta^k, or not finite); G_old is
    then recomputed with the plain propagator at the current iterate.
  * the plain propagator also judges the learned one's error: before each
    correction, r^k = mean over the swept slices n >= k of
    ||G(U_n^k) - F(U_n^k)|| / ||G_plain(U_n^k) - F(U_n^k)|| (G(U_n^k) is
    G_old_n), and two consecutive iterations with r > 1 (the learned G
    further from F than the plain one) trigger the same fallback.  Slices
    where G_plain(U_n^k) equals F(U_n^k) are left out of the mean.
"""
from __future__ import annotations

from typing import Callable, Optional

import numpy as np


def parareal(u0: np.ndarray, n_slices: int, F: Callable, G: Callable,
             norm: Callable, tol: float = 0.0, kmax: Optional[int] = None,
             skip_converged: bool = False, fallback_G: Optional[Callable] = None,
             keep_iterates: bool = True) -> dict:
    """Run (2.2).  Returns a dict with the iterates ``U`` (list over k of lists
    over n = 0..N), the update norms ``delta`` and the iteration count ``k``.

    ``skip_converged`` reuses F(U_n^k) for n < k, which by finite termination
    equals F(U_n^{k-1}) exactly; it changes no value, only the work done.
    """
    N = n_slices
    kmax = N if kmax is None else kmax
    U = [np.array(u0, dtype=np.float64, copy=True)]
    for n in range(N):
        U.append(G(U[n]))
    G_old = [U[n + 1].copy() for n in range(N)]
    out = {"U": [list(U)] if keep_iterates else [], "delta": [], "k": 0,
           "fallback_at": None, "judge": []}
    Fk = [None] * N
    G_cur = G
    prev_delta = np.inf
    k = 0
    while k < kmax:
        for n in range(N):
            if skip_converged and n < k and Fk[n] is not None:
                continue
            Fk[n] = F(U[n])
        if fallback_G is not None and G_cur is not fallback_G:
            out["judge"].append(judge_ratio(U, Fk, G_old, fallback_G, norm, k))
        new = [U[0]]
        for n in range(N):
            g = G_cur(new[n])
            new.append(Fk[n] + (g - G_old[n]))
            G_old[n] = g
        delta = max(norm(new[n] - U[n]) for n in range(1, N + 1))
        U = new
        k += 1
        out["delta"].append(delta)
        if keep_iterates:
            out["U"].append(list(U))
        if delta < tol:
            break
        judged_worse = len(out["judge"]) >= 2 and min(out["judge"][-2:]) > 1.0
        if (fallback_G is not None and G_cur is not fallback_G
                and (not np.isfinite(delta) or delta >= prev_delta or judged_worse)):
            G_cur = fallback_G
            G_old = [fallback_G(U[n]) for n in range(N)]
            out["fallback_at"] = k
        prev_delta = delta
    out["k"] = k
    out["final"] = U
    return out


def judge_ratio(U, Fk, G_old, G_plain, norm, k) -> float:
    """Mean over n = k..N-1 of ||G_old_n - F_n|| / ||G_plain(U_n) - F_n||, the
    slices with a zero denominator left out (nan if none remain)."""
    r = []
    for n in range(k, len(Fk)):
        den = norm(G_plain(U[n]) - Fk[n])
        if den > 0:
            r.append(norm(G_old[n] - Fk[n]) / den)
    return float(np.mean(r)) if r else float("nan")
