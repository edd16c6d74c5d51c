"""Pins of the oracle's Parareal iteration (2.2).

* a closed form: for linear propagators acting on one eigenmode the
  iteration is a scalar recurrence whose solution is the truncated binomial
  expansion of the fine power, sum_{j<=k} binom(n,j) (phi-gam)^j gam^{n-j};
* finite termination (proof of Theorem 3.7): U_n^k equals the sequential fine
  value bit for bit for n <= k, and k = N reproduces the whole fine solve;
* G = F converges in one iteration;
* the error bound of Theorems 3.7/3.9/3.11 on the linearised model.
"""
import math

import numpy as np
import pytest

from oracle import linear_model as lm, operators as ops, parareal, propagators
import workloads


def _norm1(v):
    return ops.norm_h(v, v.ndim)


def test_linear_mode_closed_form():
    n, N, dT, J, eps = 15, 7, 0.05, 12, 0.08
    PJ = lm.propagator_matrix(n, 1, dT / J, eps, 2.0, J)   # fine (2.5) form
    P = lm.propagator_matrix(n, 1, dT, eps, 1.0, 1)        # coarse (2.4) form
    S = ops.sine_matrix(n)
    p = 2
    u0 = S[:, p].copy()
    phi = float(u0 @ PJ @ u0)
    gam = float(u0 @ P @ u0)
    out = parareal.parareal(u0, N, lambda u: PJ @ u, lambda u: P @ u, _norm1, tol=0.0)
    for k, Uk in enumerate(out["U"]):
        for nn in range(N + 1):
            c = sum(math.comb(nn, j) * (phi - gam) ** j * gam ** (nn - j) for j in range(0, min(k, nn) + 1))
            assert np.max(np.abs(Uk[nn] - c * u0)) < 1e-13, (k, nn)


def _small_problem(kind="linear"):
    p = workloads.Problem(dim=1, n=32, eps=0.05, T=0.12, n_slices=6, j_fine=20,
                          m_coarse=1, fine_kind=kind)
    u0 = workloads.u0_uniform(32, 1, 0.3, 0)
    return p, u0


@pytest.mark.parametrize("kind", ["linear", "nonlinear"])
def test_finite_termination_bitwise(kind):
    prob, u0 = _small_problem(kind)
    seq = propagators.fine_sequential(prob, u0)
    out = parareal.parareal(u0, prob.n_slices, lambda u: propagators.fine(prob, u),
                            lambda u: propagators.coarse(prob, u), _norm1, tol=0.0)
    assert out["k"] == prob.n_slices
    for k, Uk in enumerate(out["U"]):
        for nn in range(0, min(k, prob.n_slices) + 1):
            assert np.array_equal(Uk[nn], seq[nn]), (k, nn)
    for nn in range(prob.n_slices + 1):
        assert np.array_equal(out["final"][nn], seq[nn])


def test_skip_converged_changes_nothing():
    prob, u0 = _small_problem()
    kw = dict(norm=_norm1, tol=0.0)
    Ff = lambda u: propagators.fine(prob, u)
    Gf = lambda u: propagators.coarse(prob, u)
    a = parareal.parareal(u0, prob.n_slices, Ff, Gf, **kw)
    b = parareal.parareal(u0, prob.n_slices, Ff, Gf, skip_converged=True, **kw)
    for Ua, Ub in zip(a["U"], b["U"]):
        for x, y in zip(Ua, Ub):
            assert np.array_equal(x, y)
    assert a["delta"] == b["delta"]


def test_g_equal_f_converges_in_one_iteration():
    prob, u0 = _small_problem()
    Ff = lambda u: propagators.fine(prob, u)
    out = parareal.parareal(u0, prob.n_slices, Ff, Ff, _norm1, tol=1e-300)
    assert out["delta"][0] == 0.0 and out["k"] == 1
    seq = propagators.fine_sequential(prob, u0)
    for nn in range(prob.n_slices + 1):
        assert np.array_equal(out["final"][nn], seq[nn])


def test_fallback_from_bad_coarse_still_reaches_fine_solution():
    prob, u0 = _small_problem()
    Ff = lambda u: propagators.fine(prob, u)
    Gp = lambda u: propagators.coarse(prob, u)
    bad = lambda u: 2.0 * propagators.coarse(prob, u)   # a corrupted surrogate
    out = parareal.parareal(u0, prob.n_slices, Ff, bad, _norm1, tol=1e-12, fallback_G=Gp)
    assert out["fallback_at"] == 2          # delta^2 >= delta^1 triggers it
    assert out["delta"][2] < out["delta"][1]  # and the plain G contracts again
    seq = propagators.fine_sequential(prob, u0)
    err = max(_norm1(out["final"][i] - seq[i]) for i in range(prob.n_slices + 1))
    assert err < 1e-10


@pytest.mark.parametrize("i_fine,i_coarse", [(1, 1), (2, 2), (2, 1)])
def test_linearised_error_bound(i_fine, i_coarse):
    # PA-I, PA-II, PA-III on the linearised model (Theorems 3.7, 3.9, 3.11)
    n, N, dT, J, eps = 15, 10, 0.02, 20, 0.1
    PJ = lm.propagator_matrix(n, 1, dT / J, eps, i_fine, J)
    P = lm.propagator_matrix(n, 1, dT, eps, i_coarse, 1)
    alpha, beta = lm.alpha_beta(n, 1, dT, J, eps, i_fine, i_coarse)
    assert 0 < beta < 1  # Lemma 3.1
    u0 = np.random.default_rng(4).uniform(-1, 1, n)
    exact = [u0]
    for _ in range(N):
        exact.append(PJ @ exact[-1])
    out = parareal.parareal(u0, N, lambda u: PJ @ u, lambda u: P @ u,
                            lambda v: float(np.linalg.norm(v)), tol=0.0)
    e0 = max(np.linalg.norm(out["U"][0][j] - exact[j]) for j in range(1, N + 1))
    for k in range(1, N + 1):
        ek = max(np.linalg.norm(out["U"][k][j] - exact[j]) for j in range(1, N + 1))
        assert ek <= lm.bound_factor(alpha, beta, N, k) * e0 * (1 + 1e-9) + 1e-14


def test_toeplitz_power_first_column_lemma_3_4():
    beta, N = 0.7, 9
    T = lm.toeplitz_T(beta, N)
    for k in range(1, N):
        Tk = np.linalg.matrix_power(T, k)
        for i in range(1, N + 1):   # 1-based row index of Lemma 3.4
            ref = 0.0 if i <= k else math.comb(i - 2, k - 1) * beta ** (i - 1 - k)
            assert abs(Tk[i - 1, 0] - ref) < 1e-13
        # Lemma 3.5
        assert np.max(np.sum(np.abs(Tk), axis=1)) <= min(((1 - beta ** (N - 1)) / (1 - beta)) ** k, math.comb(N - 1, k)) + 1e-12


def test_judge_ratio_closed_form_on_a_linear_mode():
    # on one sine mode F, G and G_plain are scalars phi, gam, gp, so every
    # slice's ratio is |gam - phi| / |gp - phi| and so is their mean
    n, N, dT, J, eps = 15, 7, 0.05, 12, 0.08
    PJ = lm.propagator_matrix(n, 1, dT / J, eps, 2.0, J)   # fine (2.5) form
    P = lm.propagator_matrix(n, 1, dT, eps, 1.0, 1)        # plain coarse (2.4) form
    S = ops.sine_matrix(n)
    u0 = S[:, 2].copy()
    phi, gp = float(u0 @ PJ @ u0), float(u0 @ P @ u0)
    for scale in (0.9, 1.3):
        gam = scale * gp
        out = parareal.parareal(u0, N, lambda u: PJ @ u, lambda u: scale * (P @ u), _norm1,
                                tol=0.0, kmax=2, fallback_G=lambda u: P @ u)
        want = abs(gam - phi) / abs(gp - phi)
        assert abs(out["judge"][0] - want) < 1e-12 * want, (scale, out["judge"][0], want)


def test_judge_triggers_fallback_while_delta_contracts():
    # a surrogate 10% too large: the update norm still contracts, but the plain
    # propagator judges it worse in two consecutive iterations -> fallback
    prob, u0 = _small_problem()
    Ff = lambda u: propagators.fine(prob, u)
    Gp = lambda u: propagators.coarse(prob, u)
    biased = lambda u: 1.1 * propagators.coarse(prob, u)
    plain_rule = parareal.parareal(u0, prob.n_slices, Ff, biased, _norm1, tol=1e-12)
    d = plain_rule["delta"]
    assert all(d[i + 1] < d[i] for i in range(3))          # delta alone would not switch
    out = parareal.parareal(u0, prob.n_slices, Ff, biased, _norm1, tol=1e-12, fallback_G=Gp)
    assert out["judge"][0] > 1.0 and out["judge"][1] > 1.0
    assert out["fallback_at"] == 2
    seq = propagators.fine_sequential(prob, u0)
    err = max(_norm1(out["final"][i] - seq[i]) for i in range(prob.n_slices + 1))
    assert err < 1e-10


def test_judge_ratio_zero_for_an_exact_coarse_propagator():
    prob, u0 = _small_problem()
    Ff = lambda u: propagators.fine(prob, u)
    Gp = lambda u: propagators.coarse(prob, u)
    out = parareal.parareal(u0, prob.n_slices, Ff, Ff, _norm1, tol=1e-12, fallback_G=Gp)
    assert out["judge"][0] == 0.0 and out["fallback_at"] is None


def _symbol(lam, tau, eps, i):
    # eigenvalue of (I - i tau D + eps^2 tau D^2)^{-1} (I - i tau D) on the
    # sine mode whose D_h eigenvalue is lam (Section 3)
    return (1.0 - i * tau * lam) / (1.0 - i * tau * lam + eps * eps * tau * lam * lam)


@pytest.mark.parametrize("dim,n,i_fine,i_coarse", [(1, 15, 2.0, 1.0), (1, 20, 1.0, 1.0),
                                                   (2, 6, 2.0, 2.0), (2, 7, 2.0, 1.0)])
def test_alpha_beta_from_the_sine_eigenvalues(dim, n, i_fine, i_coarse):
    # P_i and P_{J_i} are symmetric and share the sine eigenvectors, so their
    # 2-norms are the largest moduli of their symbols over the DST spectrum
    dT, J, eps = 0.03, 9, 0.07
    lam = ops.eigenvalues_paper(n)
    Lam = lam if dim == 1 else (lam[:, None] + lam[None, :]).ravel()
    gJ = _symbol(Lam, dT / J, eps, i_fine) ** J
    g = _symbol(Lam, dT, eps, i_coarse)
    alpha, beta = lm.alpha_beta(n, dim, dT, J, eps, i_fine, i_coarse)
    assert abs(alpha - np.max(np.abs(gJ - g))) <= 1e-12 * alpha
    assert abs(beta - np.max(np.abs(g))) <= 1e-12 * beta


@pytest.mark.parametrize("kind,m", [("approx2", 3), ("stab", 4), ("eyre", 2)])
def test_coarse_substeps_take_tau_dT_over_m(kind, m):
    # f == 0: the coarse step is diagonal on a sine mode, with factor
    # 1 / (1 + eps^2 tau Lam^2) for (2.4) and (1 - s tau Lam) / (1 + eps^2 tau
    # Lam^2 - s tau Lam) for the stabilised step; m substeps of tau = dT/m give
    # that factor to the power m
    n, eps, s = 24, 0.05, 2.0
    p = workloads.Problem(dim=2, n=n, eps=eps, T=0.02, n_slices=2, j_fine=5, m_coarse=m,
                          coarse_kind=kind, f_zero=True)
    x = np.arange(1, n + 1) / (n + 1)
    u = np.outer(np.sin(2 * np.pi * x), np.sin(3 * np.pi * x))
    lam = ops.eigenvalues_paper(n)
    Lam = lam[1] + lam[2]
    tau = p.dT / m
    sv = s if kind == "stab" else 0.0
    rho = (1 - sv * tau * Lam) / (1 + eps * eps * tau * Lam * Lam - sv * tau * Lam)
    v = propagators.coarse(p, u)
    assert np.max(np.abs(v - rho ** m * u)) <= 1e-13 * np.max(np.abs(u))
    # one coarse step of the whole slice differs (the substeps are taken)
    rho1 = (1 - sv * p.dT * Lam) / (1 + eps * eps * p.dT * Lam * Lam - sv * p.dT * Lam)
    assert abs(rho ** m - rho1) > 1e-3 * abs(rho1)


def test_parareal_closed_form_with_coarse_substeps():
    # the binomial closed form of the iterates on one sine mode, with the
    # propagators themselves (f == 0, m_c = 3 coarse substeps)
    n, N = 16, 6
    p = workloads.Problem(dim=1, n=n, eps=0.06, T=0.06, n_slices=N, j_fine=7, m_coarse=3,
                          f_zero=True)
    S = ops.sine_matrix(n)
    u0 = S[:, 3].copy()
    Lam = ops.eigenvalues_paper(n)[3]
    tf = p.dt
    phi = ((1 - p.s_fine * tf * Lam) / (1 + p.eps ** 2 * tf * Lam ** 2 - p.s_fine * tf * Lam)) ** p.j_fine
    tc = p.dT / p.m_coarse
    gam = (1.0 / (1 + p.eps ** 2 * tc * Lam ** 2)) ** p.m_coarse
    out = parareal.parareal(u0, N, lambda u: propagators.fine(p, u),
                            lambda u: propagators.coarse(p, u), _norm1, tol=0.0)
    for k, Uk in enumerate(out["U"]):
        for nn in range(N + 1):
            c = sum(math.comb(nn, j) * (phi - gam) ** j * gam ** (nn - j)
                    for j in range(0, min(k, nn) + 1))
            assert np.max(np.abs(Uk[nn] - c * u0)) < 1e-12, (k, nn)


@pytest.mark.parametrize("pairing", ["PA-I", "NPA-II"])
def test_finite_termination_of_the_other_pairings(pairing):
    # PA-I (F = G = (2.4)) and NPA-II (F = G = (2.3), coarse by Newton):
    # Parareal reproduces the serial fine solve bit for bit at k = N
    kw = dict(fine_kind="approx2") if pairing == "PA-I" else dict(fine_kind="nonlinear",
                                                                   coarse_kind="eyre")
    p = workloads.Problem(dim=1, n=32, eps=0.05, T=0.12, n_slices=5, j_fine=10, **kw)
    u0 = workloads.u0_uniform(32, 1, 0.3, 3)
    seq = propagators.fine_sequential(p, u0)
    out = parareal.parareal(u0, p.n_slices, lambda u: propagators.fine(p, u),
                            lambda u: propagators.coarse(p, u), _norm1, tol=0.0)
    for nn in range(p.n_slices + 1):
        assert np.array_equal(out["final"][nn], seq[nn])
    assert out["delta"][0] > 0


def test_eyre_coarse_with_one_substep_is_one_newton_step_of_the_slice():
    # the NPA-II coarse propagator with m_c = 1 is one step of (2.3) with
    # tau = dT, i.e. the fine propagator of a one-step slice
    p = workloads.Problem(dim=2, n=10, eps=0.05, T=0.02, n_slices=2, j_fine=7,
                          fine_kind="nonlinear", coarse_kind="eyre")
    q = workloads.Problem(dim=2, n=10, eps=0.05, T=0.02, n_slices=2, j_fine=1,
                          fine_kind="nonlinear")
    u = workloads.u0_uniform(10, 2, 0.5, 8)
    assert np.array_equal(propagators.coarse(p, u), propagators.fine(q, u))


def test_pa1_fine_propagator_closed_form():
    # PA-I's fine propagator is J steps of (2.4) with tau = dt; with f == 0 a
    # sine mode decays by 1 / (1 + eps^2 dt Lam^2) per step
    n = 20
    p = workloads.Problem(dim=2, n=n, eps=0.05, T=0.02, n_slices=2, j_fine=9,
                          fine_kind="approx2", f_zero=True)
    x = np.arange(1, n + 1) / (n + 1)
    u = np.outer(np.sin(4 * np.pi * x), np.sin(1 * np.pi * x))
    lam = ops.eigenvalues_paper(n)
    rho = 1.0 / (1 + p.eps ** 2 * p.dt * (lam[3] + lam[0]) ** 2)
    v = propagators.fine(p, u)
    assert np.max(np.abs(v - rho ** p.j_fine * u)) <= 1e-13 * np.max(np.abs(u))


def test_harness_bound_factor_equals_the_theorem_factor():
    # the study harness's bound factor against the oracle's, incl. the
    # binomial branch of the minimum
    from paper_2304_14074_amd import study
    for a, b, N, k in ((0.6, 0.98, 20, 3), (0.3, 0.5, 10, 7), (0.9, 0.999, 50, 1)):
        assert abs(study.bound_factor(a, b, N, k) - lm.bound_factor(a, b, N, k)) <= \
            1e-14 * lm.bound_factor(a, b, N, k)
