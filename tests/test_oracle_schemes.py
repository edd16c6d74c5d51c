"""Pins of the oracle's time steps (Section 2.1, schemes (2.3)-(2.5)).

Each scheme's result is checked against the scheme's own defining equation
evaluated with independent loop stencils, against closed-form mode decay for
f == 0, against a library nonlinear solver, and against energy decay."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from oracle import energy, operators as ops, schemes
from tests._loops import lap_loops


def _u0(n, dim, amp=0.5, seed=3):
    return amp * np.random.default_rng(seed).uniform(-1, 1, (n,) * dim)


@pytest.mark.parametrize("dim,n", [(1, 12), (2, 6)])
def test_stab_step_satisfies_scheme_2_5(dim, n):
    # (2.5) with D_h restored: v - u = tau L(u^3) - 3 tau L u - eps^2 tau L^2 v + 2 tau L v
    u = _u0(n, dim)
    tau, eps = 3e-4, 0.05
    v = schemes.step_stab(u, tau, eps, 2.0)
    res = v - u - (tau * lap_loops(u ** 3) - 3 * tau * lap_loops(u)
                   - eps ** 2 * tau * lap_loops(lap_loops(v)) + 2 * tau * lap_loops(v))
    assert np.max(np.abs(res)) < 1e-12


@pytest.mark.parametrize("dim,n", [(1, 12), (2, 6)])
def test_approx2_step_satisfies_scheme_2_4(dim, n):
    # (2.4): v - u = tau L(u^2 v) - tau L u - eps^2 tau L^2 v
    u = _u0(n, dim)
    tau, eps = 1e-3, 0.05
    v = schemes.step_approx2(u, tau, eps)
    res = v - u - (tau * lap_loops(u ** 2 * v) - tau * lap_loops(u) - eps ** 2 * tau * lap_loops(lap_loops(v)))
    assert np.max(np.abs(res)) < 1e-11


@pytest.mark.parametrize("dim,n", [(1, 12), (2, 6)])
def test_eyre_step_satisfies_scheme_2_3(dim, n):
    # (2.3): v - u = tau L(v^3) - tau L u - eps^2 tau L^2 v
    u = _u0(n, dim, amp=0.9)
    tau, eps = 1e-3, 0.05
    v = schemes.step_newton(u, tau, eps, "eyre", tol=1e-13)
    res = v - u - (tau * lap_loops(v ** 3) - tau * lap_loops(u) - eps ** 2 * tau * lap_loops(lap_loops(v)))
    assert np.max(np.abs(res)) < 1e-10


def test_be_step_satisfies_backward_euler():
    # v - u = tau L(f(v)) - eps^2 tau L^2 v
    u = _u0(12, 1, amp=0.9)
    tau, eps = 2e-4, 0.05
    v = schemes.step_newton(u, tau, eps, "be", tol=1e-13)
    res = v - u - (tau * lap_loops(v ** 3 - v) - eps ** 2 * tau * lap_loops(lap_loops(v)))
    assert np.max(np.abs(res)) < 1e-10


@pytest.mark.parametrize("variant", ["eyre", "be"])
def test_newton_agrees_with_library_root_finder(variant):
    n, tau, eps = 24, 5e-4, 0.06
    u = _u0(n, 1, amp=0.8, seed=7)
    L = ops.laplacian(n, 1).toarray()
    if variant == "eyre":
        H = lambda y: y + eps ** 2 * tau * L @ L @ y - tau * L @ y ** 3 - (u - tau * L @ u)
    else:
        H = lambda y: y + eps ** 2 * tau * L @ L @ y - tau * L @ (y ** 3 - y) - u
    ref = so.root(H, u.copy(), method="hybr", tol=1e-14).x
    v = schemes.step_newton(u, tau, eps, variant, tol=1e-12)
    assert np.max(np.abs(v - ref)) < 1e-10


def test_newton_converges_quadratically():
    u = _u0(32, 1, amp=0.9, seed=5)
    hist = []
    schemes.step_newton(u, 2e-3, 0.04, "eyre", tol=1e-14, history=hist)
    assert len(hist) >= 3
    # once in the asymptotic regime: d_{m+1} <= C d_m^2 with a modest C
    for a, b in zip(hist[1:-1], hist[2:]):
        if a < 1e-3 and b > 1e-15:
            assert b <= 50.0 * a * a


@pytest.mark.parametrize("dim,n,p,q", [(1, 31, 3, None), (2, 47, 1, 2)])
def test_f_zero_mode_decay_closed_form(dim, n, p, q):
    # With f == 0 a sine mode is an eigenvector: amplitude ratio per step
    # rho = (1 - s tau Lam) / (1 + tau eps^2 Lam^2 - s tau Lam), Lam the eigenvalue of L.
    tau, eps, s, m = 1e-4, 0.03, 2.0, 25
    x = np.arange(1, n + 1) / (n + 1)
    lam = lambda k: 2 * (n + 1) ** 2 * (math.cos(k * math.pi / (n + 1)) - 1)
    if dim == 1:
        u = np.sin(p * math.pi * x); Lam = lam(p)
    else:
        u = np.outer(np.sin(p * math.pi * x), np.sin(q * math.pi * x)); Lam = lam(p) + lam(q)
    rho = (1 - s * tau * Lam) / (1 + tau * eps ** 2 * Lam ** 2 - s * tau * Lam)
    v = u.copy()
    for _ in range(m):
        v = schemes.step_stab(v, tau, eps, s, f_zero=True)
    assert np.max(np.abs(v - rho ** m * u)) <= 1e-12 * np.max(np.abs(u))
    # and the continuum biharmonic decay exp(-eps^2 pi^4 (p^2+q^2)^2 t) to O(dt + h^2)
    k2 = p * p + (q * q if q else 0)
    expo = -eps ** 2 * math.pi ** 4 * k2 ** 2 * m * tau
    assert abs(m * math.log(rho) - expo) < 0.05 * abs(expo)


def test_f_zero_newton_equals_unstabilised_linear_step():
    u = _u0(10, 2, seed=9)
    a = schemes.step_newton(u, 1e-3, 0.05, "eyre", f_zero=True)
    b = schemes.step_stab(u, 1e-3, 0.05, 0.0, f_zero=True)
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("scheme", ["stab", "approx2", "eyre"])
def test_energy_non_increasing(scheme):
    # unconditional gradient stability of (2.3)-(2.5) (Section 2.1)
    n, eps, tau = 24, 0.05, 2e-4
    u = _u0(n, 2, amp=0.3, seed=11)
    E = [energy.energy(u, eps)]
    for _ in range(40):
        if scheme == "stab":
            u = schemes.step_stab(u, tau, eps, 2.0)
        elif scheme == "approx2":
            u = schemes.step_approx2(u, tau, eps)
        else:
            u = schemes.step_newton(u, tau, eps, "eyre")
        E.append(energy.energy(u, eps))
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-14 * np.abs(E[:-1]))
    assert E[-1] < E[0]


@pytest.mark.parametrize("variant,dim,n", [("eyre", 1, 12), ("eyre", 2, 6), ("be", 1, 12), ("be", 2, 6)])
def test_newton_residual_is_the_scheme_defect(variant, dim, n):
    # H(Y) at an arbitrary Y against the scheme written with loop stencils,
    # and H vanishes (to the Newton stop) at the step's result
    u = _u0(n, dim, amp=0.8, seed=13)
    y = _u0(n, dim, amp=0.8, seed=14)
    tau, eps = 4e-4, 0.05
    L = lap_loops
    if variant == "eyre":
        want = y + eps ** 2 * tau * L(L(y)) - tau * L(y ** 3) - (u - tau * L(u))
    else:
        want = y + eps ** 2 * tau * L(L(y)) - tau * L(y ** 3 - y) - u
    got = schemes.newton_residual(y, u, tau, eps, variant)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    v = schemes.step_newton(u, tau, eps, variant, tol=1e-13)
    assert np.max(np.abs(schemes.newton_residual(v, u, tau, eps, variant))) < 1e-9


# ---- the sine-basis routes reach the sparse-LU results up to rounding
@pytest.mark.parametrize("dim,n", [(1, 31), (2, 24), (2, 64)])
def test_sine_route_linear_step_equals_lu(dim, n):
    u = _u0(n, dim, amp=0.7, seed=21)
    for tau, eps, s in ((2e-5, 0.02, 2.0), (1e-3, 0.05, 0.0), (3e-4, 0.03, 3.0)):
        a = schemes.step_stab(u, tau, eps, s)
        b = schemes.step_stab_dst(u, tau, eps, s)
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a), (tau, eps, s)


def test_sine_route_mode_decay_closed_form():
    n, tau, eps, s, m = 40, 1e-4, 0.03, 2.0, 20
    x = np.arange(1, n + 1) / (n + 1)
    u = np.outer(np.sin(3 * math.pi * x), np.sin(5 * math.pi * x))
    lam = lambda k: 2 * (n + 1) ** 2 * (math.cos(k * math.pi / (n + 1)) - 1)
    Lam = lam(3) + lam(5)
    rho = (1 - s * tau * Lam) / (1 + tau * eps ** 2 * Lam ** 2 - s * tau * Lam)
    v = u.copy()
    for _ in range(m):
        v = schemes.step_stab_dst(v, tau, eps, s, f_zero=True)
    assert np.max(np.abs(v - rho ** m * u)) <= 1e-12 * np.max(np.abs(u))


@pytest.mark.parametrize("variant,n", [("eyre", 24), ("eyre", 48), ("be", 24), ("be", 48)])
def test_pcg_route_newton_step_equals_lu(variant, n):
    rng = np.random.default_rng(n)
    u = 0.25 + 0.05 * rng.standard_normal((n, n))
    for tau, eps in ((1e-5, 0.015), (2e-4, 0.05)):
        a = schemes.step_newton(u, tau, eps, variant)
        b = schemes.step_newton_pcg(u, tau, eps, variant)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a), (tau, eps)


def test_pcg_solves_a_dense_spd_system():
    # the textbook PCG against numpy's dense solve on a random SPD matrix
    rng = np.random.default_rng(2)
    B = rng.standard_normal((30, 30))
    K = B @ B.T + 30 * np.eye(30)
    b = rng.standard_normal(30)
    dinv = 1.0 / np.diag(K)
    x, it = schemes.pcg(lambda v: K @ v, lambda v: dinv * v, b, np.zeros(30), 1e-14, 200)
    ref = np.linalg.solve(K, b)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref) and it > 0
