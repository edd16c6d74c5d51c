"""Device-side failures reach the caller: ch_check_status maps the status
words to CH_ERR_TIMEOUT / CH_ERR_NOCONV, the flags of one call do not leak
into the next, and a Parareal run keeps its flags until the next prediction.
The group waits are made to give up from the host (ch_set_wait_limit with a
limit of 0), so every kernel still runs to its end.

Also the regression case of several grid-size classes in one context whose
n = 128 class runs its coarse sweep on groups of workgroups: that launch
must have the device to itself (no side-stream sweep beside it)."""
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


def test_forced_group_timeout_is_reported_then_cleared():
    from paper_2304_14074_amd import chlib
    n, N, J = 128, 4, 20
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J)
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(n) == 8
    X = np.stack([workloads.u0_uniform(n, 2, 0.3, 70 + i) for i in range(N)])
    assert ctx.ch_check_status() == [0]
    print("fine sweep on groups with a zero wait limit", flush=True)
    ctx.ch_set_wait_limit(0.0, 0.0)
    gu.fine(ctx, [X])
    with pytest.raises(chlib.CHError) as e:
        ctx.ch_check_status()
    assert e.value.status == chlib.CH_ERR_TIMEOUT
    print("same sweep with the default limits", flush=True)
    ctx.ch_set_wait_limit()
    out = gu.fine(ctx, [X])[0]
    assert ctx.ch_check_status() == [0]
    assert gu.rel(out[1], propagators.fine(p, X[1])) < TOL


def test_forced_pipeline_timeout_sticks_to_the_run():
    from paper_2304_14074_amd import chlib
    n, N, J = 128, 4, 8
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J)
    u0 = workloads.u0_uniform(n, 2, 0.3, 81)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    ctx.ch_parareal_iterate(st, 0.0)
    print("pipelined run with a zero hand-off limit", flush=True)
    ctx.ch_set_wait_limit(0.2, 0.0)
    ctx.ch_parareal_run(st, -1.0, 2)
    with pytest.raises(chlib.CHError) as e:
        ctx.ch_check_status(st)
    assert e.value.status == chlib.CH_ERR_TIMEOUT
    assert int(st["status"][0].item()) & 4
    # the run's flags stay: a later healthy iteration still reports them
    ctx.ch_set_wait_limit()
    ctx.ch_parareal_iterate(st, 0.0)
    with pytest.raises(chlib.CHError):
        ctx.ch_check_status(st)
    assert ctx.ch_check_status() == [0]          # that call's own flags are clear
    # a new run starts clean and matches the oracle
    s2 = ctx.new_state()
    s2["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    print("pipelined run with the default limits", flush=True)
    ctx.ch_parareal_run(s2, -1.0, 2)
    assert ctx.ch_check_status(s2) == [0]
    U = gu.unpack_iter(ctx, s2["U"])[0]
    ref = _oracle_run(p, u0, 2)
    for j in range(N + 1):
        assert gu.rel(U[j], ref["U"][2][j]) < TOL, j


def test_mixed_classes_beside_a_group_coarse_sweep():
    # 40 instances of n = 128 (coarse sweep on groups of four: 160 workgroups,
    # one per CU) with n = 256 and n = 64 instances whose one-workgroup sweeps
    # used to run on side streams at the same time
    from paper_2304_14074_amd import chlib
    probs, u0s = [], []
    for i in range(40):
        probs.append(workloads.Problem(dim=2, n=128, eps=0.02, T=2 * 3 * 2e-5, n_slices=2,
                                       j_fine=3))
    for i in range(3):
        probs.append(workloads.Problem(dim=2, n=256, eps=0.015, T=2 * 2 * 1e-5, n_slices=2,
                                       j_fine=2))
    for i in range(3):
        probs.append(workloads.Problem(dim=2, n=64, eps=0.03, T=3 * 3 * 4e-5, n_slices=3,
                                       j_fine=3))
    for i, p in enumerate(probs):
        u0s.append(workloads.u0_uniform(p.n, 2, 0.3, 300 + i))
    ctx = chlib.Context(probs)
    assert ctx.ch_chain_variant(128) == 4
    st = ctx.new_state()
    U0 = torch.zeros(ctx.iter_total, dtype=torch.float64)
    for i, p in enumerate(probs):
        io = ctx.layout(i)[3]
        U0[io:io + p.n * p.n] = torch.from_numpy(u0s[i].reshape(-1))
    st["U"].copy_(U0.cuda())
    print("mixed classes: prediction + 2 iterations", flush=True)
    ctx.ch_parareal_iterate(st, 0.0)
    for _ in range(2):
        ctx.ch_parareal_iterate(st, 0.0)
    torch.cuda.synchronize()
    assert ctx.ch_check_status(st) == [0] * len(probs)
    U = gu.unpack_iter(ctx, st["U"])
    for i in (0, 39, 41, 44):
        p = probs[i]
        ref = _oracle_run(p, u0s[i], 2)
        for j in range(p.n_slices + 1):
            assert gu.rel(U[i][j], ref["U"][2][j]) < TOL, (i, j, gu.rel(U[i][j], ref["U"][2][j]))
