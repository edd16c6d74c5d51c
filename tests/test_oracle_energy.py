"""Pins of the discrete energy (Section 1, (1.2))."""
import math

import numpy as np

from oracle import energy, operators as ops
from tests._loops import grad_sq_loops


def test_energy_of_a_sine_mode_closed_form():
    # u_i = a sin(p pi x_i): h sum sin^2 = 1/2, h sum sin^4 = 3/8 (2p, 4p != 0 mod n+1)
    n, p, a, eps = 40, 3, 0.7, 0.05
    x = np.arange(1, n + 1) / (n + 1)
    u = a * np.sin(p * math.pi * x)
    h = 1 / (n + 1)
    lam = 2 / h ** 2 * (math.cos(p * math.pi / (n + 1)) - 1)
    ref = n * h / 4 - a ** 2 / 4 + 3 * a ** 4 / 32 - eps ** 2 * lam * a ** 2 / 4
    assert abs(energy.energy(u, eps) - ref) < 1e-13


def test_gradient_part_is_edge_sum():
    rng = np.random.default_rng(0)
    for dim, n in [(1, 11), (2, 7)]:
        u = rng.standard_normal((n,) * dim)
        eps = 0.3
        h = 1 / (n + 1)
        bulk = h ** dim * np.sum(0.25 * (u ** 2 - 1) ** 2)
        ref = bulk + 0.5 * eps ** 2 * h ** dim * grad_sq_loops(u)
        assert abs(energy.energy(u, eps) - ref) < 1e-12 * abs(ref)


def test_continuum_limit_2d():
    # E(sin(pi x) sin(pi y)) = 41/256 + (eps^2/2)(pi^2/2); E_h converges at first order
    eps = 0.1
    exact = 41 / 256 + 0.5 * eps ** 2 * math.pi ** 2 / 2
    errs = []
    for n in (63, 127):
        x = np.arange(1, n + 1) / (n + 1)
        u = np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
        errs.append(abs(energy.energy(u, eps) - exact))
    assert errs[1] < 0.6 * errs[0] and errs[1] < 5e-3
