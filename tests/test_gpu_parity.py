"""GPU vs oracle parity of every hot-path call, through the C ABI.

FP64 path bound: relative L2 <= 1e-11 per state (the two sides use different
solvers -- sine-transform GEMMs vs sparse LU -- so agreement is to rounding).
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import energy as o_energy, operators, parareal, propagators
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _states(n, dim, count, seed, amps=(0.05, 0.5, 0.9)):
    rng = np.random.default_rng(seed)
    return np.stack([amps[i % len(amps)] * rng.uniform(-1, 1, (n,) * dim) for i in range(count)])


@pytest.mark.parametrize("n", [32, 64, 128])
def test_fine_2d_matches_oracle(n):
    from paper_2304_14074_amd import chlib
    J = 40
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=3 * J * 2e-5, n_slices=3, j_fine=J)
    ctx = chlib.Context([p])
    X = _states(n, 2, 3, seed=n)
    print(f"fine 2D n={n} J={J}", flush=True)
    out = gu.fine(ctx, [X])[0]
    for s in range(3):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


def test_fine_1d_full_small_config():
    from paper_2304_14074_amd import chlib
    p = workloads.small_1d()
    ctx = chlib.Context([p])
    X = _states(128, 1, p.n_slices, seed=1, amps=(0.1, 0.6, 0.95))
    print("fine 1D n=128 J=313 N=16", flush=True)
    out = gu.fine(ctx, [X])[0]
    for s in range(p.n_slices):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


@pytest.mark.parametrize("dim,n,kind,m", [(2, 32, "approx2", 1), (2, 64, "approx2", 1),
                                          (2, 128, "approx2", 1), (2, 64, "approx2", 2),
                                          (2, 64, "stab", 4), (1, 128, "approx2", 1),
                                          (1, 128, "stab", 2)])
def test_coarse_matches_oracle(dim, n, kind, m):
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=dim, n=n, eps=0.02, T=3 / 32, n_slices=3, j_fine=10, m_coarse=m,
                          coarse_kind=kind)
    ctx = chlib.Context([p])
    X = _states(n, dim, 3, seed=7 + n)
    print(f"coarse {kind} dim={dim} n={n} m={m}", flush=True)
    out = gu.coarse(ctx, [X])[0]
    for s in range(3):
        ref = propagators.coarse(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


def test_mask_leaves_unmasked_slices_untouched():
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=64, eps=0.03, T=4e-4, n_slices=4, j_fine=5)
    ctx = chlib.Context([p])
    X = _states(64, 2, 4, seed=3)
    U = gu.pack_slices(ctx, [X])
    F = torch.full_like(U, 7.0)
    mask = torch.tensor([1, 0, 1, 0], dtype=torch.uint8, device="cuda")
    ctx.ch_fine_propagate(U, F, mask)
    torch.cuda.synchronize()
    out = gu.unpack_slices(ctx, F)[0]
    assert np.all(out[1] == 7.0) and np.all(out[3] == 7.0)
    assert gu.rel(out[0], propagators.fine(p, X[0])) < TOL


def test_ragged_batch_of_instances():
    from paper_2304_14074_amd import chlib
    probs = [workloads.Problem(dim=2, n=64, eps=0.03, T=2 * 10 * 2e-5, n_slices=2, j_fine=10),
             workloads.Problem(dim=2, n=128, eps=0.015, T=1 * 10 * 2e-5, n_slices=1, j_fine=10),
             workloads.Problem(dim=1, n=128, eps=0.03, T=3 * 20 * 1e-4, n_slices=3, j_fine=20),
             workloads.Problem(dim=2, n=32, eps=0.04, T=2 * 7 * 3e-5, n_slices=2, j_fine=7)]
    ctx = chlib.Context(probs)
    states = [_states(p.n, p.dim, p.n_slices, seed=20 + i) for i, p in enumerate(probs)]
    outs = gu.fine(ctx, states)
    for p, X, out in zip(probs, states, outs):
        for s in range(p.n_slices):
            assert gu.rel(out[s], propagators.fine(p, X[s])) < TOL


def test_f_zero_closed_form_mode_decay():
    # f == 0: a sine mode decays by rho^J exactly (up to rounding)
    from paper_2304_14074_amd import chlib
    n, J, dt, eps, s = 64, 50, 2e-5, 0.02, 2.0
    p = workloads.Problem(dim=2, n=n, eps=eps, T=J * dt, n_slices=1, j_fine=J, f_zero=True)
    ctx = chlib.Context([p])
    x = np.arange(1, n + 1) / (n + 1)
    u = np.outer(np.sin(3 * np.pi * x), np.sin(5 * np.pi * x))
    lam = lambda k: 2 * (n + 1) ** 2 * (np.cos(k * np.pi / (n + 1)) - 1)
    L = lam(3) + lam(5)
    rho = (1 - s * dt * L) / (1 + dt * eps ** 2 * L ** 2 - s * dt * L)
    out = gu.fine(ctx, [u[None]])[0][0]
    assert gu.rel(out, rho ** J * u) < 1e-12


def test_energy_matches_oracle():
    from paper_2304_14074_amd import chlib
    # every 2D size (the row-walking kernel, including n = 32's partial wave) and 1D
    for dim, n in [(2, 32), (2, 64), (2, 128), (2, 256), (1, 128), (1, 50)]:
        p = workloads.Problem(dim=dim, n=n, eps=0.02, T=1.0, n_slices=3, j_fine=1)
        ctx = chlib.Context([p])
        X = _states(n, dim, 3, seed=5)
        u = torch.from_numpy(X.reshape(-1)).cuda()
        E = torch.zeros(3, dtype=torch.float64, device="cuda")
        ctx.ch_energy(0, u, 3, E)
        torch.cuda.synchronize()
        for s in range(3):
            ref = o_energy.energy(X[s], 0.02)
            assert abs(E[s].item() - ref) <= 1e-13 * abs(ref)


def _oracle_run(p, u0, K):
    return parareal.parareal(u0, p.n_slices, lambda u: propagators.fine(p, u),
                             lambda u: propagators.coarse(p, u),
                             lambda v: operators.norm_h(v, p.dim), tol=0.0, kmax=K)


@pytest.mark.parametrize("dim,n,kind", [(2, 64, "approx2"), (1, 128, "approx2"), (2, 32, "stab")])
def test_parareal_iterates_match_oracle(dim, n, kind):
    from paper_2304_14074_amd import chlib
    N, J = 5, 25
    p = workloads.Problem(dim=dim, n=n, eps=0.03, T=N * J * 4e-5, n_slices=N, j_fine=J,
                          coarse_kind=kind, m_coarse=2 if kind == "stab" else 1)
    u0 = workloads.u0_uniform(n, dim, 0.3, 11)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    st["U"][: n ** dim] = torch.from_numpy(u0.reshape(-1)).cuda()
    ref = _oracle_run(p, u0, N)
    print(f"parareal dim={dim} n={n} {kind}", flush=True)
    ctx.ch_parareal_iterate(st, 0.0)   # coarse prediction
    torch.cuda.synchronize()
    U = gu.unpack_iter(ctx, st["U"])[0]
    for j in range(N + 1):
        assert gu.rel(U[j], ref["U"][0][j]) < TOL, ("k=0", j)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(N + 1):
            assert gu.rel(U[j], ref["U"][k][j]) < TOL, (k, j, gu.rel(U[j], ref["U"][k][j]))
        d = st["delta"][0].item()
        assert abs(d - ref["delta"][k - 1]) <= 1e-9 * max(ref["delta"][k - 1], 1e-300) + 1e-15


def test_finite_termination_bitwise_on_gpu():
    # U_n^k equals the GPU's own sequential fine chain bit for bit for n <= k
    from paper_2304_14074_amd import chlib
    N, J, n = 4, 15, 64
    p = workloads.Problem(dim=2, n=n, eps=0.03, T=N * J * 4e-5, n_slices=N, j_fine=J)
    u0 = workloads.u0_uniform(n, 2, 0.3, 12)
    ctx = chlib.Context([p])
    one = chlib.Context([workloads.Problem(dim=2, n=n, eps=0.03, T=J * 4e-5, n_slices=1, j_fine=J)])
    seq = [u0]
    for _ in range(N):
        seq.append(gu.fine(one, [seq[-1][None]])[0][0])
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    ctx.ch_parareal_iterate(st, 0.0)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(0, k + 1):
            assert np.array_equal(U[j], seq[j]), (k, j)


def test_full_size_2d_sampled_slices():
    # the 128x128, eps=0.02, J=1563 fine sweep in the benchmark's launch shape
    # (all 64 slices in one launch); two sampled slices against the oracle
    from paper_2304_14074_amd import chlib
    p = workloads.linear_2d_128()
    ctx = chlib.Context([p])
    rng = np.random.default_rng(99)
    X = np.stack([(0.05 if s % 2 == 0 else 0.6) * rng.uniform(-1, 1, (128, 128))
                  for s in range(p.n_slices)])
    print("full-size fine sweep 64 x 1563 steps", flush=True)
    out = gu.fine(ctx, [X])[0]
    for s in (0, 37):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))
    assert np.all(np.isfinite(out))


def test_full_small_1d_parareal_to_tolerance():
    # 1D, n=128, eps=0.03, T=0.5, N=16, J=313, Parareal to 1e-10 (or k = N)
    from paper_2304_14074_amd import chlib
    p = workloads.small_1d()
    u0 = workloads.small_1d_u0(0)
    ref = parareal.parareal(u0, p.n_slices, lambda u: propagators.fine(p, u),
                            lambda u: propagators.coarse(p, u),
                            lambda v: operators.norm_h(v, 1), tol=1e-10)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    st["U"][:128] = torch.from_numpy(u0).cuda()
    ctx.ch_parareal_iterate(st, 1e-10)
    k = 0
    while k < p.n_slices:
        ctx.ch_parareal_iterate(st, 1e-10)
        k += 1
        if st["delta"][0].item() < 1e-10:
            break
    assert k == ref["k"]
    U = gu.unpack_iter(ctx, st["U"])[0]
    # bound: 1e-11 or the oracle's own two-route floor of this run
    from tests._floor import dense_route_sequence
    alt = dense_route_sequence(p, u0)
    for j in range(p.n_slices + 1):
        floor = gu.rel(alt[j], ref["final"][j])
        err = gu.rel(U[j], ref["final"][j])
        print(f"T_{j}: gpu-vs-oracle {err:.2e}  oracle two-route floor {floor:.2e}", flush=True)
        assert err <= max(TOL, floor), (j, err, floor)


@pytest.mark.parametrize("n,variant,groups", [(32, "eyre", 1), (64, "eyre", 1), (128, "eyre", 1),
                                              (128, "eyre", 8), (128, "be", 8), (64, "be", 1)])
def test_nonlinear_fine_matches_oracle(n, variant, groups):
    # implicit fine step (scheme (2.3) or backward Euler) by Newton + spectral CG,
    # on one workgroup per slice or on a group of eight
    from paper_2304_14074_amd import chlib
    J = 4 if n == 128 else 6
    p = workloads.Problem(dim=2, n=n, eps=0.015, T=2 * J * 1e-5, n_slices=2, j_fine=J,
                          fine_kind="nonlinear", nl_variant=variant)
    ctx = chlib.Context([p])
    if n == 128:
        assert ctx.ch_fine_groups(n, groups, fine_kind="nonlinear") == groups
    rng = np.random.default_rng(n)
    X = np.stack([0.25 + 0.05 * rng.standard_normal((n, n)), 0.9 * rng.uniform(-1, 1, (n, n))])
    print(f"nonlinear fine n={n} {variant} groups={groups}", flush=True)
    out = gu.fine(ctx, [X])[0]
    for s in range(2):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


def test_nonlinear_f_zero_is_linear_biharmonic_solve():
    from paper_2304_14074_amd import chlib
    n, J, tau, eps = 64, 3, 1e-4, 0.03
    p = workloads.Problem(dim=2, n=n, eps=eps, T=J * tau, n_slices=1, j_fine=J,
                          fine_kind="nonlinear", f_zero=True)
    ctx = chlib.Context([p])
    x = np.arange(1, n + 1) / (n + 1)
    u = np.outer(np.sin(2 * np.pi * x), np.sin(3 * np.pi * x))
    lam = lambda k: 2 * (n + 1) ** 2 * (np.cos(k * np.pi / (n + 1)) - 1)
    L = lam(2) + lam(3)
    out = gu.fine(ctx, [u[None]])[0][0]
    assert gu.rel(out, (1.0 / (1 + tau * eps ** 2 * L ** 2)) ** J * u) < 1e-12


def test_nonlinear_parareal_iterates_match_oracle():
    # NPA-I: implicit fine step, coarse scheme (2.4)
    from paper_2304_14074_amd import chlib
    N, J, n = 3, 4, 32
    p = workloads.Problem(dim=2, n=n, eps=0.03, T=N * J * 5e-5, n_slices=N, j_fine=J,
                          fine_kind="nonlinear")
    u0 = workloads.u0_gauss(n, 2, 0.25, 0.05, 3)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    ref = _oracle_run(p, u0, N)
    ctx.ch_parareal_iterate(st, 0.0)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(N + 1):
            assert gu.rel(U[j], ref["U"][k][j]) < TOL, (k, j)
    assert int(st["status"][0].item()) == 0


SPLIT_TOL = 1e-4   # reduced-precision bound on a whole fine propagation


@pytest.mark.parametrize("n", [64, 128])
def test_split_bf16_fine_within_reduced_precision_bound(n):
    # BF16x3 transforms inside FP64 defect correction vs the FP64 oracle
    from paper_2304_14074_amd import chlib
    J = 200
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=2 * J * 2e-5, n_slices=2, j_fine=J,
                          precision="split_bf16")
    ctx = chlib.Context([p])
    rng = np.random.default_rng(40 + n)
    X = np.stack([0.05 * rng.uniform(-1, 1, (n, n)), 0.8 * rng.uniform(-1, 1, (n, n))])
    out = gu.fine(ctx, [X])[0]
    for s in range(2):
        ref = propagators.fine(p, X[s])
        err = gu.rel(out[s], ref)
        print(f"split-bf16 n={n} slice {s}: rel L2 vs FP64 oracle {err:.2e}", flush=True)
        assert err < SPLIT_TOL, err


def test_split_bf16_full_slice_128():
    # one full slice of the 128x128, eps=0.02, J=1563 workload in split precision
    from paper_2304_14074_amd import chlib
    p = workloads.linear_2d_128()
    p.precision = "split_bf16"
    p.n_slices, p.T = 1, p.dT
    ctx = chlib.Context([p])
    u0 = workloads.linear_2d_128_u0(0)
    out = gu.fine(ctx, [u0[None]])[0][0]
    ref = propagators.fine(p, u0)
    err = gu.rel(out, ref)
    print(f"split-bf16 full slice: rel L2 vs FP64 oracle {err:.2e}", flush=True)
    assert err < SPLIT_TOL, err


@pytest.mark.parametrize("groups", [1, 8])
def test_streamed_256_fine_matches_oracle(groups):
    # n = 256: one workgroup per slice streams the state through global memory
    # (it does not fit on a CU); a group of eight keeps it in the members' LDS
    from paper_2304_14074_amd import chlib
    J = 8
    p = workloads.Problem(dim=2, n=256, eps=0.015, T=2 * J * 1e-5, n_slices=2, j_fine=J)
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(256, groups) == groups
    print(f"n=256 fine groups={groups}", flush=True)
    rng = np.random.default_rng(256)
    X = np.stack([0.25 + 0.05 * rng.standard_normal((256, 256)), 0.9 * rng.uniform(-1, 1, (256, 256))])
    out = gu.fine(ctx, [X])[0]
    for s in range(2):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


@pytest.mark.parametrize("kind,m", [("approx2", 1), ("stab", 2)])
def test_streamed_256_coarse_matches_oracle(kind, m):
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=256, eps=0.015, T=2 / 32, n_slices=2, j_fine=10,
                          coarse_kind=kind, m_coarse=m)
    ctx = chlib.Context([p])
    rng = np.random.default_rng(257)
    X = np.stack([0.25 + 0.05 * rng.standard_normal((256, 256)), 0.9 * rng.uniform(-1, 1, (256, 256))])
    out = gu.coarse(ctx, [X])[0]
    for s in range(2):
        ref = propagators.coarse(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


def test_streamed_256_parareal_iterates_match_oracle():
    from paper_2304_14074_amd import chlib
    N, J, n = 3, 6, 256
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J)
    u0 = workloads.u0_uniform(n, 2, 0.3, 9)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    ref = _oracle_run(p, u0, N)
    ctx.ch_parareal_iterate(st, 0.0)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(N + 1):
            assert gu.rel(U[j], ref["U"][k][j]) < TOL, (k, j)


def test_batched_256_instances_sampled_against_oracle():
    # the full 256-instance batch in one fine-sweep call (the benchmark's
    # launch shape); sampled slices of two instances against the oracle
    from paper_2304_14074_amd import chlib
    probs = workloads.batched_instances(256, 4)
    ctx = chlib.Context(probs)
    rng = np.random.default_rng(77)
    states = [0.05 * rng.uniform(-1, 1, (p.n_slices, p.n, p.n)) for p in probs]
    print("batched fine sweep of 256 instances", flush=True)
    outs = gu.fine(ctx, states)
    checked = 0
    for i, p in enumerate(probs):
        if p.n in (64, 128) and checked < 2 and p.n == (64 if checked == 0 else 128):
            ref = propagators.fine(p, states[i][1])
            assert gu.rel(outs[i][1], ref) < TOL, (i, gu.rel(outs[i][1], ref))
            checked += 1
    assert checked == 2
    # n = 256 (groups of eight, persistent over the class's items): the first
    # item of the class and its last one, which a group takes at the end of
    # its loop; the oracle's sine-basis route (equal to its LU route up to
    # rounding) keeps these two full slices to seconds
    big = [i for i, p in enumerate(probs) if p.n == 256]
    for i, s_ in ((big[0], 0), (big[-1], probs[big[-1]].n_slices - 1)):
        ref = propagators.fine(probs[i], states[i][s_], route="sine")
        err = gu.rel(outs[i][s_], ref)
        print(f"n=256 instance {i} slice {s_}: {err:.2e}", flush=True)
        assert err < TOL, (i, s_, err)
    assert all(np.all(np.isfinite(o)) for o in outs)


@pytest.mark.parametrize("groups", [1, 16])
def test_streamed_256_nonlinear_step_full_size_parameters(groups):
    # the 256x256, eps=0.015, dt=1e-5 implicit step: one step against the oracle,
    # streamed on one workgroup per slice or on a group of sixteen
    from paper_2304_14074_amd import chlib
    base = workloads.nonlinear_2d_256()
    p = workloads.Problem(dim=2, n=256, eps=base.eps, T=2 * base.dt, n_slices=2, j_fine=1,
                          fine_kind="nonlinear")
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(256, groups, fine_kind="nonlinear") == groups
    X = np.stack([workloads.nonlinear_2d_256_u0(0), workloads.u0_uniform(256, 2, 0.9, 5)])
    print(f"nonlinear 256 single step groups={groups}", flush=True)
    out = gu.fine(ctx, [X])[0]
    for s in range(2):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


def test_streamed_256_nonlinear_energy_decays():
    # scheme (2.3) is unconditionally gradient stable: the discrete energy of
    # the 256x256 run cannot increase (property at the full size)
    from paper_2304_14074_amd import chlib
    base = workloads.nonlinear_2d_256()
    J = 200
    p = workloads.Problem(dim=2, n=256, eps=base.eps, T=J * base.dt, n_slices=1, j_fine=J,
                          fine_kind="nonlinear")
    ctx = chlib.Context([p])
    u0 = workloads.u0_uniform(256, 2, 0.5, 6)
    out = gu.fine(ctx, [u0[None]])[0][0]
    e0, e1 = o_energy.energy(u0, p.eps), o_energy.energy(out, p.eps)
    assert np.all(np.isfinite(out)) and e1 < e0


@pytest.mark.parametrize("groups", [1, 4, 8])
def test_chain_variants_parareal_128_match_oracle(groups):
    # the coarse sweep of (2.2) on one workgroup per instance and split over a
    # group of four or eight workgroups: all against the oracle's iterates
    from paper_2304_14074_amd import chlib
    N, J, n = 4, 8, 128
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J)
    u0 = workloads.u0_uniform(n, 2, 0.3, 13)
    ctx = chlib.Context([p])
    assert ctx.ch_chain_variant(n, groups) == groups
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    ref = _oracle_run(p, u0, N)
    print(f"chain variant groups={groups}", flush=True)
    ctx.ch_parareal_iterate(st, 0.0)
    torch.cuda.synchronize()
    U = gu.unpack_iter(ctx, st["U"])[0]
    for j in range(N + 1):
        assert gu.rel(U[j], ref["U"][0][j]) < TOL, ("k=0", j)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(N + 1):
            assert gu.rel(U[j], ref["U"][k][j]) < TOL, (k, j, gu.rel(U[j], ref["U"][k][j]))
        d = st["delta"][0].item()
        assert abs(d - ref["delta"][k - 1]) <= 1e-9 * max(ref["delta"][k - 1], 1e-300) + 1e-15
    assert int(st["status"][0].item()) == 0


def test_chain_group_ragged_batch_matches_single_workgroup_chain():
    # nine instances (two groups of eight slots, seven idle) with different
    # eps, slice counts and amplitudes; a tenth with the stabilised coarse
    # step makes its class fall back to one workgroup per instance
    from paper_2304_14074_amd import chlib
    n = 128
    probs = [workloads.Problem(dim=2, n=n, eps=0.02 + 0.002 * i, T=(2 + i % 3) * 4 * 2e-5,
                               n_slices=2 + i % 3, j_fine=4) for i in range(9)]
    u0s = [workloads.u0_uniform(n, 2, (0.05, 0.5, 0.9)[i % 3], 40 + i) for i in range(9)]

    def run(groups, probs, u0s):
        ctx = chlib.Context(probs)
        assert ctx.ch_chain_variant(n, groups) == groups
        st = ctx.new_state()
        for i, u0 in enumerate(u0s):
            _, _, _, io = ctx.layout(i)
            st["U"][io: io + n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
        out = []
        for _ in range(4):
            ctx.ch_parareal_iterate(st, 0.0)
            torch.cuda.synchronize()
            out.append((gu.unpack_iter(ctx, st["U"]), st["delta"].cpu().numpy().copy(),
                        st["status"].cpu().numpy().copy()))
        return out

    a = run(4, probs, u0s)
    b = run(1, probs, u0s)
    for (Ua, da, sa), (Ub, db, sb) in zip(a, b):
        assert np.all(sa == 0) and np.all(sb == 0)
        for i in range(9):
            for j in range(len(Ua[i])):
                # two CG forms (one and three reductions per iteration) agree
                # to the solver tolerance, not bitwise
                assert gu.rel(Ua[i][j], Ub[i][j]) < TOL, (i, j)
            if np.isfinite(db[i]):
                assert abs(da[i] - db[i]) <= 1e-9 * max(db[i], 1e-300) + 1e-15
            else:   # no update norm yet after the prediction
                assert da[i] == db[i]
    ref = _oracle_run(probs[4], u0s[4], 3)
    for k in range(1, 4):
        for j in range(len(ref["U"][k])):
            assert gu.rel(a[k][0][4][j], ref["U"][k][j]) < TOL, (k, j)
    # a stabilised-coarse instance in the class: the whole class uses one
    # workgroup per instance and still matches
    mixed = probs[:2] + [workloads.Problem(dim=2, n=n, eps=0.02, T=2 * 4 * 2e-5, n_slices=2,
                                           j_fine=4, coarse_kind="stab", m_coarse=2)]
    c = run(4, mixed, u0s[:3])
    d = run(1, mixed, u0s[:3])
    for (Ua, _, sa), (Ub, _, _) in zip(c, d):
        assert np.all(sa == 0)
        for i in range(3):
            for j in range(len(Ua[i])):
                assert np.array_equal(Ua[i][j], Ub[i][j]), (i, j)


@pytest.mark.parametrize("groups", [1, 4, 8])
def test_fine_groups_128_mask_and_oracle(groups):
    # the n = 128 fine sweep on one workgroup per slice and on groups of four
    # or eight (spectral Laplacian): masked slices against the oracle, unmasked
    # slices untouched; five slices fill one group slot set with three idle
    from paper_2304_14074_amd import chlib
    n, N, J = 128, 5, 12
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J)
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(n, groups) == groups
    X = _states(n, 2, N, seed=5)
    U = gu.pack_slices(ctx, [X])
    F = torch.full_like(U, 7.0)
    mask = torch.tensor([1, 0, 1, 1, 0], dtype=torch.uint8, device="cuda")
    print(f"fine groups={groups}", flush=True)
    ctx.ch_fine_propagate(U, F, mask)
    torch.cuda.synchronize()
    out = gu.unpack_slices(ctx, F)[0]
    assert np.all(out[1] == 7.0) and np.all(out[4] == 7.0)
    for s in (0, 2, 3):
        ref = propagators.fine(p, X[s])
        assert gu.rel(out[s], ref) < TOL, (s, gu.rel(out[s], ref))


@pytest.mark.parametrize("groups", [4, 8])
def test_fine_groups_128_f_zero_mode_decay(groups):
    # f == 0 on the group path: a sine mode decays by rho^J
    from paper_2304_14074_amd import chlib
    n, J, dt, eps, s = 128, 40, 2e-5, 0.02, 2.0
    p = workloads.Problem(dim=2, n=n, eps=eps, T=J * dt, n_slices=1, j_fine=J, f_zero=True)
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(n) == 8
    assert ctx.ch_fine_groups(n, groups) == groups
    x = np.arange(1, n + 1) / (n + 1)
    u = np.outer(np.sin(7 * np.pi * x), np.sin(2 * np.pi * x))
    lam = lambda k: 2 * (n + 1) ** 2 * (np.cos(k * np.pi / (n + 1)) - 1)
    L = lam(7) + lam(2)
    rho = (1 - s * dt * L) / (1 + dt * eps ** 2 * L ** 2 - s * dt * L)
    out = gu.fine(ctx, [u[None]])[0][0]
    assert gu.rel(out, rho ** J * u) < 1e-12


def test_fine_groups_persistent_over_more_slices_than_groups():
    # 300 slices on groups of four: the resident groups (at most 64 on a
    # 256-CU device) each take several slices in turn; every slice agrees with
    # the one-workgroup kernel, two sampled ones with the oracle
    from paper_2304_14074_amd import chlib
    n, N, J = 128, 300, 3
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J)
    X = _states(n, 2, N, seed=17)
    outs = {}
    for groups in (4, 1):
        ctx = chlib.Context([p])
        assert ctx.ch_fine_groups(n, groups) == groups
        print(f"persistent fine groups={groups}", flush=True)
        outs[groups] = gu.fine(ctx, [X])[0]
    for s_ in range(N):
        assert gu.rel(outs[4][s_], outs[1][s_]) < TOL, s_
    for s_ in (0, 299):
        assert gu.rel(outs[4][s_], propagators.fine(p, X[s_])) < TOL, s_


def test_nonlinear_group_parareal_iterates_128_match_oracle():
    # NPA-I at n = 128 with the implicit fine step on groups of eight and the
    # coarse sweep on a group of eight: iterates against the oracle, with the
    # default CG targets
    from paper_2304_14074_amd import chlib
    N, J, n = 3, 3, 128
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J,
                          fine_kind="nonlinear")
    u0 = workloads.u0_gauss(n, 2, 0.25, 0.05, 4)
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(n, fine_kind="nonlinear") == 8
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    ref = _oracle_run(p, u0, N)
    print("nonlinear group parareal n=128", flush=True)
    ctx.ch_parareal_iterate(st, 0.0)
    for k in range(1, N + 1):
        ctx.ch_parareal_iterate(st, 0.0)
        torch.cuda.synchronize()
        U = gu.unpack_iter(ctx, st["U"])[0]
        for j in range(N + 1):
            assert gu.rel(U[j], ref["U"][k][j]) < TOL, (k, j, gu.rel(U[j], ref["U"][k][j]))
    assert int(st["status"][0].item()) == 0
