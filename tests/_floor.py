"""The FP64 noise floor of a long fine solve: the same sequence of linear
fine steps computed by a second, equally correct route (dense sine-matrix
transforms instead of the oracle's sparse LU).  Long runs of the spinodal
dynamics amplify rounding differences, so two correct FP64 codes drift
apart by ~1e-11 over thousands of steps; full-run GPU parity is judged
against this measured floor (per-step and per-slice parity stay at 1e-11)."""
import numpy as np

from oracle import operators


def dense_route_sequence(p, u0):
    n = p.n
    S = operators.sine_matrix(n)
    lam = operators.eigenvalues_paper(n)
    Lam = lam if p.dim == 1 else lam[:, None] + lam[None, :]
    tau = p.dt
    sig = 1 + tau * p.eps ** 2 * Lam ** 2 - p.s_fine * tau * Lam
    L = operators.laplacian(n, p.dim)

    def step(u):
        r = u + tau * (L @ (u ** 3 - (1 + p.s_fine) * u).reshape(-1)).reshape(u.shape)
        if p.dim == 1:
            return S @ ((S @ r) / sig)
        return S @ (((S @ r @ S) / sig)) @ S

    out = [np.array(u0, dtype=np.float64)]
    u = out[0].copy()
    for _ in range(p.n_slices):
        for _ in range(p.j_fine):
            u = step(u)
        out.append(u.copy())
    return out
