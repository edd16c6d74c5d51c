"""The paper's other pairings of Section 2.1 on the GPU through the C ABI:
PA-I (fine propagator = scheme (2.4) with tau = dt, a variable-coefficient
solve every fine step) and NPA-II (coarse propagator = scheme (2.3) solved
by Newton's method), each against the FP64 oracle: single propagations at
every grid size and Parareal iterates."""
import numpy as np
import pytest
import torch

import workloads
from oracle import operators, parareal, propagators
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _oracle_run(p, u0, K):
    return parareal.parareal(u0, p.n_slices, lambda u: propagators.fine(p, u),
                             lambda u: propagators.coarse(p, u),
                             lambda v: operators.norm_h(v, p.dim), tol=0.0, kmax=K)


@pytest.mark.parametrize("n,J", [(32, 8), (64, 6), (128, 4), (256, 2)])
def test_pa1_fine_step_matches_oracle(n, J):
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=2 * J * 1e-4, n_slices=2, j_fine=J,
                          fine_kind="approx2")
    ctx = chlib.Context([p])
    rng = np.random.default_rng(500 + n)
    X = np.stack([0.3 * rng.uniform(-1, 1, (n, n)), 0.9 * rng.uniform(-1, 1, (n, n))])
    print(f"PA-I fine n={n} J={J}", flush=True)
    out = gu.fine(ctx, [X])[0]
    assert ctx.ch_check_status() == [0]
    for s in range(2):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


@pytest.mark.parametrize("n,m", [(32, 1), (64, 2), (128, 1), (256, 1)])
def test_npa2_coarse_step_matches_oracle(n, m):
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=2 * 1e-3, n_slices=2, j_fine=10, m_coarse=m,
                          coarse_kind="eyre", fine_kind="nonlinear")
    ctx = chlib.Context([p])
    rng = np.random.default_rng(600 + n)
    X = np.stack([0.25 + 0.05 * rng.standard_normal((n, n)), 0.8 * rng.uniform(-1, 1, (n, n))])
    print(f"NPA-II coarse n={n} m={m}", flush=True)
    out = gu.coarse(ctx, [X])[0]
    assert ctx.ch_check_status() == [0]
    for s in range(2):
        ref = propagators.coarse(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


@pytest.mark.parametrize("pairing,n", [("PA-I", 64), ("NPA-II", 64), ("PA-I", 128)])
def test_pairing_parareal_iterates_match_oracle(pairing, n):
    from paper_2304_14074_amd import chlib
    N, J = 4, 5
    kw = (dict(fine_kind="approx2") if pairing == "PA-I"
          else dict(fine_kind="nonlinear", coarse_kind="eyre"))
    p = workloads.Problem(dim=2, n=n, eps=0.03, T=N * J * 4e-5, n_slices=N, j_fine=J, **kw)
    u0 = workloads.u0_uniform(n, 2, 0.4, 17)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    ref = _oracle_run(p, u0, N)
    print(f"{pairing} parareal n={n}", flush=True)
    ctx.ch_parareal_iterate(st, 0.0)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(N + 1):
            assert gu.rel(U[j], ref["U"][k][j]) < TOL, (k, j, gu.rel(U[j], ref["U"][k][j]))
        d = st["delta"][0].item()
        assert abs(d - ref["delta"][k - 1]) <= 1e-9 * max(ref["delta"][k - 1], 1e-300) + 1e-15
    assert ctx.ch_check_status(st) == [0]


# ---- 1D: any n <= 128 (the paper's grids: h = 1/64 is n = 63), every pairing
@pytest.mark.parametrize("fine_kind,n", [("linear", 63), ("approx2", 63), ("nonlinear", 63),
                                         ("nonlinear", 128), ("approx2", 100), ("linear", 17)])
def test_1d_fine_kinds_match_oracle(fine_kind, n):
    from paper_2304_14074_amd import chlib
    J = 20
    p = workloads.Problem(dim=1, n=n, eps=0.0725, T=2 * J * 1e-4, n_slices=2, j_fine=J,
                          fine_kind=fine_kind)
    ctx = chlib.Context([p])
    rng = np.random.default_rng(700 + n)
    X = np.stack([0.3 * rng.uniform(-1, 1, n), 0.9 * rng.uniform(-1, 1, n)])
    print(f"1D fine {fine_kind} n={n}", flush=True)
    out = gu.fine(ctx, [X])[0]
    assert ctx.ch_check_status() == [0]
    for s in range(2):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


@pytest.mark.parametrize("kind,n,m", [("eyre", 63, 1), ("eyre", 64, 3), ("approx2", 63, 2),
                                      ("stab", 63, 4)])
def test_1d_coarse_kinds_match_oracle(kind, n, m):
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=1, n=n, eps=0.0725, T=2 * 0.02, n_slices=2, j_fine=10, m_coarse=m,
                          coarse_kind=kind)
    ctx = chlib.Context([p])
    rng = np.random.default_rng(800 + n)
    X = np.stack([0.3 * rng.uniform(-1, 1, n), 0.9 * rng.uniform(-1, 1, n)])
    print(f"1D coarse {kind} n={n} m={m}", flush=True)
    out = gu.coarse(ctx, [X])[0]
    assert ctx.ch_check_status() == [0]
    for s in range(2):
        ref = propagators.coarse(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


@pytest.mark.parametrize("pairing", ["PA-I", "PA-II", "PA-III", "NPA-I", "NPA-II"])
def test_1d_paper_pairings_parareal_iterates(pairing):
    # the paper's 1D setting (eps = 0.0725, h = 1/64, J = 200 fine steps per
    # slice) on a short horizon: every iterate against the oracle
    from paper_2304_14074_amd import chlib
    fine, coarse = {"PA-I": ("approx2", "approx2"), "PA-II": ("linear", "stab"),
                    "PA-III": ("linear", "approx2"), "NPA-I": ("nonlinear", "approx2"),
                    "NPA-II": ("nonlinear", "eyre")}[pairing]
    N, J, n = 5, 200, 63
    p = workloads.Problem(dim=1, n=n, eps=0.0725, T=N * 0.01, n_slices=N, j_fine=J,
                          fine_kind=fine, coarse_kind=coarse)
    u0 = workloads.u0_uniform(n, 1, 0.5, 31)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    st["U"][:n] = torch.from_numpy(u0).cuda()
    ref = _oracle_run(p, u0, N)
    print(f"1D {pairing} parareal", flush=True)
    ctx.ch_parareal_iterate(st, 0.0)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(N + 1):
            assert gu.rel(U[j], ref["U"][k][j]) < TOL, (k, j, gu.rel(U[j], ref["U"][k][j]))
    assert ctx.ch_check_status(st) == [0]
