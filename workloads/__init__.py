"""Seeded synthetic inputs and problem presets for the Cahn-Hilliard Parareal workloads.

This module is shared by the CPU oracle, the tests and the benchmark.  It holds
no arithmetic of the numerical method: only random initial states drawn from
``numpy.random.default_rng`` (PCG64, float64, C order over the interior grid
points) and the parameter sets of the workloads.

The paper (Section 4) never states its initial data; the distributions below
are the ones the workloads prescribe.  Time-step bookkeeping: the slice length
is dT = T / N and the number of fine steps per slice is J = ceil(dT / dt_nominal),
so that dt = dT / J divides the slice exactly (the paper's Section 2 writes
dt = dT / J).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np


@dataclasses.dataclass
class Problem:
    """Parameters of one Cahn-Hilliard instance and its Parareal splitting."""

    dim: int = 2              # 1 or 2 space dimensions
    n: int = 128              # interior points per dimension, h = 1/(n+1)
    eps: float = 0.02         # interface width epsilon
    T: float = 2.0            # final time
    n_slices: int = 64        # Parareal slices N
    j_fine: int = 1563        # fine steps per slice J
    m_coarse: int = 1         # coarse sub-steps per slice
    s_fine: float = 2.0       # stabilisation constant of the linear fine step
    fine_kind: str = "linear"       # "linear" (2.5), "nonlinear" (2.3), "approx2" (2.4) or
                                    # "approx2_dd" ((2.4) by Neumann-Neumann, 1D)
    nl_variant: str = "eyre"        # "eyre" (convex splitting) or "be" (fully implicit)
    coarse_kind: str = "approx2"    # "approx2" (2.4), "stab", "neural" or "eyre" (2.3)
    precision: str = "fp64"         # "fp64" or "split_bf16"
    newton_tol: float = 1e-10
    newton_max: int = 20
    krylov_rtol: float = 0.0       # CG target of the (2.4) solves; 0: the library's default
    nl_krylov_rtol: float = 1e-9    # CG target inside Newton
    krylov_max: int = 200
    f_zero: bool = False     # test hook: f(u) == 0
    nn_base: int = 0         # learned G: 0 = u + net(u), 1 = G_plain(u) + net(u)
    dd_subdomains: int = 8   # Neumann-Neumann fine step: equal subdomains N0
    dd_theta: float = 0.25   # relaxation of the trace update
    dd_tol: float = 1e-10    # stop: max trace change per iteration
    dd_max: int = 100        # iteration cap per step

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def dT(self) -> float:
        return self.T / self.n_slices

    @property
    def dt(self) -> float:
        return self.dT / self.j_fine

    @property
    def npts(self) -> int:
        return self.n ** self.dim


def fine_steps(T: float, n_slices: int, dt_nominal: float) -> int:
    """J = ceil(dT / dt_nominal), guarded against round-off just above an integer."""
    q = (T / n_slices) / dt_nominal
    return int(math.ceil(q - 1e-9))


def u0_uniform(n: int, dim: int, amp: float, seed: int) -> np.ndarray:
    """amp * Uniform(-1, 1) on the interior grid, drawn in C order."""
    rng = np.random.default_rng(seed)
    return amp * rng.uniform(-1.0, 1.0, size=(n,) * dim)


def u0_gauss(n: int, dim: int, mean: float, std: float, seed: int) -> np.ndarray:
    """mean + std * N(0, 1) on the interior grid, drawn in C order."""
    rng = np.random.default_rng(seed)
    return mean + std * rng.standard_normal(size=(n,) * dim)


# ---------------------------------------------------------------- presets
def small_1d() -> Problem:
    """1D, 128 interior points, eps=0.03, T=0.5, N=16, fine dt=1e-4 (J=313), s=2."""
    return Problem(dim=1, n=128, eps=0.03, T=0.5, n_slices=16,
                   j_fine=fine_steps(0.5, 16, 1e-4), m_coarse=1)


def small_1d_u0(seed: int = 0) -> np.ndarray:
    return u0_uniform(128, 1, 0.1, seed)


def linear_2d_128() -> Problem:
    """2D 128x128, eps=0.02, T=2, N=64, fine dt=2e-5 (J=1563), linear fine step."""
    return Problem(dim=2, n=128, eps=0.02, T=2.0, n_slices=64,
                   j_fine=fine_steps(2.0, 64, 2e-5), m_coarse=1)


def linear_2d_128_u0(seed: int = 0) -> np.ndarray:
    return u0_uniform(128, 2, 0.05, seed)


def nonlinear_2d_256() -> Problem:
    """2D 256x256, eps=0.015, T=4, N=128, fine dt=1e-5 (J=3125), implicit fine step."""
    return Problem(dim=2, n=256, eps=0.015, T=4.0, n_slices=128,
                   j_fine=fine_steps(4.0, 128, 1e-5), m_coarse=1,
                   fine_kind="nonlinear")


def nonlinear_2d_256_u0(seed: int = 0) -> np.ndarray:
    return u0_gauss(256, 2, 0.25, 0.05, seed)


def batched_instances(count: int = 256, seed: int = 4) -> List[Problem]:
    """Uneven independent instances: n in {64,128,256}, eps ~ U(0.01,0.04),
    N in {32,64,128}, dT = 1/32 (T = N/32), fine dt = 2e-5, linear fine step."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice([64, 128, 256]))
        eps = float(rng.uniform(0.01, 0.04))
        N = int(rng.choice([32, 64, 128]))
        T = N / 32.0
        out.append(Problem(dim=2, n=n, eps=eps, T=T, n_slices=N,
                           j_fine=fine_steps(T, N, 2e-5), m_coarse=1))
    return out


def batched_u0(p: Problem, index: int) -> np.ndarray:
    return u0_uniform(p.n, p.dim, 0.05, 1000 + index)
