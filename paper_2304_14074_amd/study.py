"""Parameter studies of Section 4 run on the GPU path, beside the
convergence bounds of Section 3.

For each of the five pairings of Section 2.1 (PA-I: F = G = (2.4); PA-II:
F = G = (2.5); PA-III: F = (2.5), G = (2.4); NPA-I: F = (2.3), G = (2.4);
NPA-II: F = G = (2.3)), and PA-I with the Neumann-Neumann solve of the fine
step (Section 4, "PA-I-NN"), a case runs the Parareal iteration (2.2) and records,
per iteration k, the update norm and the error against the fine solution,
E^k = max_n ||U(T_n) - U_n^k||_h (the L^inf(0,T; L^2) norm of Section 4 at the
T_n), until E^k < 1e-6 (the paper's stop) or k = N.  U(T_n) is the serial
fine solve on the GPU.  Beside the errors:
  * linear pairings: the bound alpha^k min{((1 - beta^{N-1})/(1 - beta))^k,
    binom(N-1, k)} E^0 of Theorems 3.7 / 3.9 / 3.11, with alpha and beta from
    ch_linear_bound;
  * nonlinear pairings: the same form with alpha = C1 dT^2 (Theorem 3.13 and
    its NPA-II counterpart) and beta = ||P_1||; C1 is estimated from the run
    (the smallest C1 for which the bound holds at every k), as the paper
    estimates it numerically.
The paper states no initial data, so every number here is parity-unpinned
against its figures (seeded u0 = amp * Uniform(-1, 1)).
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import chlib

# fine kind, coarse kind, (i_fine, i_coarse) of the linearised model or None
PAIRINGS = {
    "PA-I": ("approx2", "approx2", (1.0, 1.0)),
    "PA-II": ("linear", "stab", (2.0, 2.0)),
    "PA-III": ("linear", "approx2", (2.0, 1.0)),
    "NPA-I": ("nonlinear", "approx2", None),
    "NPA-II": ("nonlinear", "eyre", None),
    # the fine step (2.4) solved by Neumann-Neumann (8 subdomains, theta = 1/4)
    "PA-I-NN": ("approx2_dd", "approx2", (1.0, 1.0)),
}


@dataclasses.dataclass
class Case:
    """One run: a pairing on a grid with the paper's parameters."""
    pairing: str
    dim: int = 1
    n: int = 63              # h = 1/(n+1): n = 63 is the paper's h = 1/64
    eps: float = 0.0725
    T: float = 1.0
    N: int = 20
    J: int = 200
    amp: float = 0.1
    seed: int = 0            # u0 = amp * Uniform(-1, 1) from this seed; None: smooth

    def problem(self):
        fine, coarse, _ = PAIRINGS[self.pairing]
        return _Problem(dim=self.dim, n=self.n, eps=self.eps, T=self.T, n_slices=self.N,
                        j_fine=self.J, fine_kind=fine, coarse_kind=coarse)


@dataclasses.dataclass
class _Problem:
    dim: int
    n: int
    eps: float
    T: float
    n_slices: int
    j_fine: int
    fine_kind: str
    coarse_kind: str
    m_coarse: int = 1
    s_fine: float = 2.0
    newton_tol: float = 1e-10

    @property
    def dT(self):
        return self.T / self.n_slices


def initial_state(c: Case) -> np.ndarray:
    """Seeded noise amp * Uniform(-1, 1) (spinodal decomposition from a
    nearly uniform mixture), or with seed None the smooth profile
    amp * sin(2 pi x) (times sin(pi y) in 2D), which meets u = Lap u = 0 on
    the boundary."""
    if c.seed is not None:
        rng = np.random.default_rng(c.seed)
        return c.amp * rng.uniform(-1.0, 1.0, size=(c.n,) * c.dim)
    x = np.arange(1, c.n + 1) / (c.n + 1)
    u = c.amp * np.sin(2 * np.pi * x)
    return u if c.dim == 1 else np.outer(np.sin(np.pi * x), u)


def _u0_text(c: Case) -> str:
    if c.seed is not None:
        return f"{c.amp} * Uniform(-1,1), seed {c.seed}"
    return f"{c.amp} * sin(2 pi x)" + (" sin(pi y)" if c.dim == 2 else "")


def serial_fine(prob, u0: np.ndarray):
    """U(T_0..T_N) of the serial fine solve on the GPU, and its wall time."""
    one = chlib.Context([dataclasses.replace(prob, n_slices=1, T=prob.dT)])
    P = prob.n ** prob.dim
    traj = torch.empty((prob.n_slices + 1, P), dtype=torch.float64, device="cuda")
    traj[0] = torch.from_numpy(np.ascontiguousarray(u0).reshape(-1)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(prob.n_slices):
        one.ch_fine_propagate(traj[k], traj[k + 1])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    one.ch_check_status()
    return traj, secs


def bound_factor(a: float, beta: float, N: int, k: int) -> float:
    """a^k min{((1 - beta^{N-1})/(1 - beta))^k, binom(N-1, k)}."""
    geo = (1.0 - beta ** (N - 1)) / (1.0 - beta) if beta != 1.0 else float(N - 1)
    return a ** k * min(geo ** k, float(math.comb(N - 1, k)))


def run_case(c: Case, err_tol: float = 1e-6) -> dict:
    prob = c.problem()
    u0 = initial_state(c)
    N, P = c.N, c.n ** c.dim
    traj, serial_s = serial_fine(prob, u0)
    ctx = chlib.Context([prob])
    st = ctx.new_state()
    st["U"][:P] = traj[0]
    dist = torch.empty(N, dtype=torch.float64, device="cuda")

    def error():
        ctx.ch_slice_distance(st["U"][P:(N + 1) * P], traj[1:].reshape(-1), dist)
        return float(dist.max().item())

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ch_parareal_iterate(st, 0.0)
    errs, deltas = [error()], []
    K, secs_to_tol, diverged = None, None, False
    while len(deltas) < N:
        ctx.ch_parareal_iterate(st, 0.0)
        deltas.append(float(st["delta"][0].item()))
        errs.append(error())
        if not (math.isfinite(deltas[-1]) and math.isfinite(errs[-1])):
            diverged = True       # e.g. PA-II's coarse step at small eps
            break
        if errs[-1] < err_tol:
            K = len(deltas)
            secs_to_tol = time.perf_counter() - t0
            break
    try:
        ctx.ch_check_status(st)
    except chlib.CHError as e:
        if not (diverged and e.status == chlib.CH_ERR_NOCONV):
            raise
    errs = [e if math.isfinite(e) else None for e in errs]
    deltas = [d if math.isfinite(d) else None for d in deltas]
    out = {"pairing": c.pairing, "dim": c.dim, "n": c.n, "h": 1.0 / (c.n + 1), "eps": c.eps,
           "T": c.T, "N": N, "J": c.J, "dT": prob.dT, "u0": _u0_text(c),
           "iterations_to_1e-6": K, "diverged": diverged, "errors": errs, "update_norms": deltas,
           "serial_fine_s": serial_s, "parareal_to_1e-6_s": secs_to_tol,
           "ideal_speedup_N_over_K": (N / K) if K else None,
           "speedup_vs_serial_on_gpu": (serial_s / secs_to_tol) if secs_to_tol else None}
    if diverged:
        return out
    fine, coarse, lin = PAIRINGS[c.pairing]
    e0 = errs[0]
    if lin is not None:
        a, b = chlib.ch_linear_bound(c.dim, c.n, c.eps, prob.dT, c.J, lin[0], lin[1])
        out.update({"alpha": a, "beta": b,
                    "bound": [e0] + [bound_factor(a, b, N, k) * e0 for k in range(1, len(errs))]})
        out["within_bound"] = all(e <= bb * (1 + 1e-9) + 1e-15
                                  for e, bb in zip(errs, out["bound"]))
    else:
        _, b = chlib.ch_linear_bound(c.dim, c.n, c.eps, prob.dT, c.J, 1.0, 1.0)
        # smallest C1 with errs[k] <= (C1 dT^2)^k min{...} e0 for every k >= 1
        c1 = 0.0
        for k in range(1, len(errs)):
            f = bound_factor(1.0, b, N, k)
            if errs[k] > 0 and e0 > 0:
                c1 = max(c1, (errs[k] / (f * e0)) ** (1.0 / k) / prob.dT ** 2)
        out.update({"beta": b, "C1_fitted": c1,
                    "bound": [e0] + [bound_factor(c1 * prob.dT ** 2, b, N, k) * e0
                                     for k in range(1, len(errs))]})
    return out


def paper_cases() -> list:
    """The 1D experiments of Section 4 (h = 1/64, J = 200, eps = 0.0725) and
    the 2D ones (h = 1/33 here: the kernels' 2D grids are 32, 64, 128, 256),
    from seeded noise; the bound comparisons also from a smooth profile."""
    cases = []
    # bound comparisons: T = 1, N = 20 (PA-I also at eps = 0.725)
    for p in PAIRINGS:
        cases.append(Case(p))
        cases.append(Case(p, amp=0.9, seed=None))
    cases.append(Case("PA-I", eps=0.725))
    # dT sweep (PA-I): N = 20, dT = T/N
    for T in (0.5, 2.0, 5.0):
        cases.append(Case("PA-I", T=T))
    # mesh sweep (PA-I, T = 1, dt = 1/200 per unit slice length)
    for n in (31, 127):
        cases.append(Case("PA-I", n=n))
    # T, N sweep (dT = 0.05): T = 8 is the paper's N/K = 40 case
    for p in ("PA-I", "PA-III", "NPA-I"):
        for T in (2.0, 8.0):
            cases.append(Case(p, T=T, N=int(round(20 * T))))
    # eps sweep: T = 1, N = 50
    for p in ("PA-I", "PA-II", "PA-III", "NPA-I", "NPA-II"):
        for eps in (0.03, 0.0725, 0.2):
            cases.append(Case(p, N=50, eps=eps))
    # NPA-I N sweep at T = 50, J = 150 (the paper's 80x at N = 400)
    for N in (100, 400):
        cases.append(Case("NPA-I", T=50.0, N=N, J=150))
    # 2D: T = 1, N = 20, J = 200
    for p in ("PA-I", "PA-II", "PA-III", "NPA-I"):
        cases.append(Case(p, dim=2, n=32))
    # Neumann-Neumann fine solver in PA-I (h = 1/128, N0 = 8, theta = 1/4):
    # T, N sweep at J = 200 (dT = 0.05) and a dT sweep at T = 1, J = 150
    for T in (1.0, 2.0, 8.0):
        cases.append(Case("PA-I-NN", n=127, T=T, N=int(round(20 * T))))
    for N in (10, 40):
        cases.append(Case("PA-I-NN", n=127, N=N, J=150))
    return cases


def run_study(cases=None, log=None) -> list:
    res = []
    for c in cases or paper_cases():
        t0 = time.perf_counter()
        r = run_case(c)
        r["case_seconds"] = time.perf_counter() - t0
        if log:
            ab = (f"alpha={r['alpha']:.3f} beta={r['beta']:.4f}" if "alpha" in r else
                  f"beta={r.get('beta', float('nan')):.4f} C1={r.get('C1_fitted', float('nan')):.3g}")
            log(f"{c.pairing} dim={c.dim} n={c.n} eps={c.eps} T={c.T} N={c.N} J={c.J} "
                f"u0={r['u0']}: K={r['iterations_to_1e-6']} diverged={r['diverged']} {ab} "
                f"within_bound={r.get('within_bound')} ({r['case_seconds']:.1f} s)")
        res.append(r)
    return res
