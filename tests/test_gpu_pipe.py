"""Pipelined Parareal iterations (ch_parareal_run) through the C ABI.

The pipelined launch computes the iterates of (2.2) with the same code as the
two-launch iteration (fine sweep, then the coarse sweep and correction), only
scheduled differently, so its states, G_old and update norms must equal those
of ch_parareal_iterate bit for bit, and match the oracle to the FP64 bound.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import operators, parareal, propagators
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
TOL = 1e-11
N128 = 128


def _setup(N, J, eps=0.02, dt=2e-5, seed=31, amp=0.3):
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=N128, eps=eps, T=N * J * dt, n_slices=N, j_fine=J)
    u0 = workloads.u0_uniform(N128, 2, amp, seed)
    ctx = chlib.Context([p])
    # the two-launch reference on the same group kernels as the pipelined one
    assert ctx.ch_fine_groups(N128, 8) == 8
    assert ctx.ch_chain_variant(N128) == 8
    st = ctx.new_state()
    st["U"][: N128 * N128] = torch.from_numpy(u0.reshape(-1)).cuda()
    return p, u0, ctx, st


def _snap(st):
    torch.cuda.synchronize()
    return (st["U"].cpu().numpy().copy(), st["G_old"].cpu().numpy().copy(),
            st["delta"].cpu().numpy().copy(), st["status"].cpu().numpy().copy())


def _same(a, b, what):
    for name, x, y in zip(("U", "G_old", "delta", "status"), a, b):
        assert np.array_equal(x, y), (what, name, np.max(np.abs(x - y)) if x.dtype != np.int32 else None)


def _reference(N, J, K, sweep_all, tol, **kw):
    """K calls of ch_parareal_iterate after the prediction; with sweep_all the
    counter is reset to 0 before each, so every slice is swept."""
    _, _, ctx, st = _setup(N, J, **kw)
    ctx.ch_parareal_iterate(st, tol)
    snaps = [_snap(st)]
    for _ in range(K):
        if sweep_all:
            ctx.ch_set_iteration(st, 0)
        ctx.ch_parareal_iterate(st, tol)
        snaps.append(_snap(st))
    return snaps


@pytest.mark.parametrize("N,J,K,sweep_all", [(8, 6, 3, False), (8, 6, 3, True), (2, 5, 2, False),
                                             (9, 4, 4, True), (5, 4, 5, False)])
def test_pipelined_run_equals_iterate_bitwise(N, J, K, sweep_all):
    print(f"pipelined run N={N} J={J} K={K} sweep_all={sweep_all}", flush=True)
    ref = _reference(N, J, K, sweep_all, -1.0)
    _, _, ctx, st = _setup(N, J)
    ctx.ch_parareal_run(st, -1.0, K, sweep_all=sweep_all)
    got = _snap(st)
    _same(got, ref[K], "after K iterations")
    assert ctx.ch_iteration_count(st) == K
    assert int(got[3][0]) == 0


def test_pipelined_run_in_two_calls_continues_the_iteration():
    # a second call picks up the device counter: 2 + 2 iterations == 4
    N, J = 8, 5
    ref = _reference(N, J, 4, False, -1.0)
    _, _, ctx, st = _setup(N, J)
    print("pipelined run 2 + 2", flush=True)
    ctx.ch_parareal_run(st, -1.0, 2)
    _same(_snap(st), ref[2], "first call")
    ctx.ch_parareal_run(st, -1.0, 2)
    _same(_snap(st), ref[4], "second call")
    assert ctx.ch_iteration_count(st) == 4


def test_pipelined_run_stops_at_n_slices():
    # finite termination: with max_iters > N the run ends at k = N, where the
    # iterate is the sequential fine solution
    N, J = 4, 6
    ref = _reference(N, J, N, False, -1.0)
    _, _, ctx, st = _setup(N, J)
    print("pipelined run to k = N", flush=True)
    ctx.ch_parareal_run(st, -1.0, 10)
    _same(_snap(st), ref[N], "k = N")
    assert ctx.ch_iteration_count(st) == N


def test_pipelined_run_stops_below_tolerance():
    # a contracting regime (eps = 0.03, short slices): the run ends after the
    # first iteration whose update norm is below tol, as the iterate loop does
    N, J, dt = 12, 8, 2.5e-5
    kw = dict(eps=0.03, dt=dt, amp=0.05)
    full = _reference(N, J, 6, False, -1.0, **kw)
    deltas = [s[2][0] for s in full[1:]]
    print("update norms", deltas, flush=True)
    k_stop = 3
    tol = float(deltas[k_stop - 1]) * 1.0000001
    stop = next(k for k, d in enumerate(deltas, start=1) if d < tol)
    _, _, ctx, st = _setup(N, J, **kw)
    ctx.ch_parareal_run(st, tol, 10)
    got = _snap(st)
    assert ctx.ch_iteration_count(st) == stop
    _same(got, full[stop], "stopped")
    # a later call does nothing: the instance has converged
    ctx.ch_parareal_run(st, tol, 3)
    _same(_snap(st), full[stop], "after convergence")
    assert ctx.ch_iteration_count(st) == stop


def test_pipelined_run_more_slices_than_fine_groups():
    # 70 slices: the 62 fine groups of a 256-CU device take several items per
    # iteration (persistent), in iteration-major order
    N, J, K = 70, 3, 2
    print(f"pipelined run N={N}", flush=True)
    ref = _reference(N, J, K, True, -1.0)
    _, _, ctx, st = _setup(N, J)
    ctx.ch_parareal_run(st, -1.0, K, sweep_all=True)
    _same(_snap(st), ref[K], "N = 70")


def test_pipelined_run_matches_oracle():
    N, J, K = 4, 8, 2
    p, u0, ctx, st = _setup(N, J)
    ref = parareal.parareal(u0, N, lambda u: propagators.fine(p, u),
                            lambda u: propagators.coarse(p, u),
                            lambda v: operators.norm_h(v, 2), tol=0.0, kmax=K)
    print("pipelined run vs oracle", flush=True)
    ctx.ch_parareal_run(st, -1.0, K)
    torch.cuda.synchronize()
    U = gu.unpack_iter(ctx, st["U"])[0]
    for j in range(N + 1):
        assert gu.rel(U[j], ref["U"][K][j]) < TOL, (j, gu.rel(U[j], ref["U"][K][j]))
    d = st["delta"][0].item()
    assert abs(d - ref["delta"][K - 1]) <= 1e-9 * ref["delta"][K - 1]
    assert int(st["status"][0].item()) == 0


def test_pipelined_run_with_coarse_substeps_and_after_iterate_calls():
    # m_c = 2 coarse substeps per slice, and a run that continues an iteration
    # begun with ch_parareal_iterate: 2 iterate calls + a 2-iteration run
    # equal 4 iterate calls
    from paper_2304_14074_amd import chlib
    N, J = 6, 5
    p = workloads.Problem(dim=2, n=N128, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J,
                          m_coarse=2)
    u0 = workloads.u0_uniform(N128, 2, 0.3, 41)

    def fresh():
        ctx = chlib.Context([p])
        assert ctx.ch_fine_groups(N128, 8) == 8
        st = ctx.new_state()
        st["U"][: N128 * N128] = torch.from_numpy(u0.reshape(-1)).cuda()
        return ctx, st

    ctx, st = fresh()
    print("pipelined run m_c = 2 after iterate calls", flush=True)
    for _ in range(5):              # prediction + 4 iterations
        ctx.ch_parareal_iterate(st, -1.0)
    ref = _snap(st)
    ctx, st = fresh()
    for _ in range(3):              # prediction + 2 iterations
        ctx.ch_parareal_iterate(st, -1.0)
    ctx.ch_parareal_run(st, -1.0, 2)
    _same(_snap(st), ref, "m_c = 2, 2 + 2")
    assert ctx.ch_iteration_count(st) == 4


def test_pipelined_run_zero_iterations_forms_only_the_prediction():
    N, J = 4, 5
    ref = _reference(N, J, 0, False, -1.0)
    _, _, ctx, st = _setup(N, J)
    ctx.ch_parareal_run(st, -1.0, 0)
    _same(_snap(st), ref[0], "prediction only")
    assert ctx.ch_iteration_count(st) == 0


def test_pipelined_full_size_matches_two_launch_and_oracle_samples():
    # the benchmark's workload and launch shape (128^2, N = 64, J = 1563, one
    # coarse group and 62 fine groups): two pipelined iterations (every slice
    # swept) equal two two-launch iterations bit for bit, and sampled values
    # of the first iteration match the oracle: U_1^1 = F(U_0) and
    # U_2^1 = F(U_1^0) + G(U_1^1) - G(U_1^0)
    from paper_2304_14074_amd import chlib
    p = workloads.linear_2d_128()
    u0 = workloads.linear_2d_128_u0(0)
    n, N = p.n, p.n_slices
    P = n * n

    def fresh():
        ctx = chlib.Context([p])
        st = ctx.new_state()
        st["U"][:P] = torch.from_numpy(u0.reshape(-1)).cuda()
        ctx.ch_parareal_iterate(st, 0.0)          # the coarse prediction U^0
        return ctx, st

    print("full-size pipelined vs two-launch, 2 iterations", flush=True)
    ctx, st = fresh()
    U0 = st["U"].cpu().numpy().reshape(N + 1, n, n)
    ctx.ch_parareal_run(st, -1.0, 1, sweep_all=True)
    U1 = st["U"].cpu().numpy().reshape(N + 1, n, n)
    ctx.ch_set_iteration(st, 0)
    ctx.ch_parareal_run(st, -1.0, 1, sweep_all=True)
    pipe2 = _snap(st)
    ctx, st = fresh()
    for _ in range(2):
        ctx.ch_set_iteration(st, 0)
        ctx.ch_parareal_iterate(st, -1.0)
    _same(pipe2, _snap(st), "two iterations at full size")
    # oracle samples of the first iteration
    ref1 = propagators.fine(p, U0[0])
    assert gu.rel(U1[1], ref1) < TOL, gu.rel(U1[1], ref1)
    ref2 = propagators.fine(p, U0[1]) + (propagators.coarse(p, U1[1]) - propagators.coarse(p, U0[1]))
    assert gu.rel(U1[2], ref2) < TOL, gu.rel(U1[2], ref2)
