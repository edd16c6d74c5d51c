"""Degenerate and edge cases of the hot path through the C ABI: one slice,
an all-zero mask, the zero state (a steady state of the equation: f(0) = 0),
and finished iterations."""
import numpy as np
import pytest
import torch

import workloads
from oracle import operators, propagators
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [64, 128])
def test_single_slice_parareal_is_the_fine_solve(n):
    # N = 1: the first correction gives U_1 = F(U_0) bit for bit (the fine
    # sweep's own value); the update norm is ||F(U_0) - G(U_0)||_h; a further
    # call (k = N) changes nothing and reports 0
    from paper_2304_14074_amd import chlib
    J = 12
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=J * 2e-5, n_slices=1, j_fine=J)
    u0 = workloads.u0_uniform(n, 2, 0.3, 51)
    ctx = chlib.Context([p])
    f = gu.fine(ctx, [u0[None]])[0][0]
    g = gu.coarse(ctx, [u0[None]])[0][0]
    st = ctx.new_state()
    st["U"][: n * n] = torch.from_numpy(u0.reshape(-1)).cuda()
    print(f"single slice n={n}", flush=True)
    ctx.ch_parareal_iterate(st, 0.0)
    ctx.ch_parareal_iterate(st, 0.0)
    torch.cuda.synchronize()
    U = gu.unpack_iter(ctx, st["U"])[0]
    assert np.array_equal(U[1], f)
    d = st["delta"][0].item()
    want = operators.norm_h(f - g, 2)
    assert abs(d - want) <= 1e-12 * want
    ctx.ch_parareal_iterate(st, 0.0)
    torch.cuda.synchronize()
    assert np.array_equal(gu.unpack_iter(ctx, st["U"])[0], U)
    assert st["delta"][0].item() == 0.0
    assert int(st["status"][0].item()) == 0


@pytest.mark.parametrize("n", [64, 128])
def test_all_zero_mask_computes_nothing(n):
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=4 * 5 * 2e-5, n_slices=4, j_fine=5)
    ctx = chlib.Context([p])
    X = np.stack([workloads.u0_uniform(n, 2, 0.3, 60 + i) for i in range(4)])
    U = gu.pack_slices(ctx, [X])
    F = torch.full_like(U, 3.0)
    G = torch.full_like(U, 3.0)
    mask = torch.zeros(4, dtype=torch.uint8, device="cuda")
    ctx.ch_fine_propagate(U, F, mask)
    ctx.ch_coarse_propagate(U, G, mask)
    torch.cuda.synchronize()
    assert bool((F == 3.0).all()) and bool((G == 3.0).all())


@pytest.mark.parametrize("n,pipelined", [(64, False), (128, False), (128, True)])
def test_zero_state_stays_zero(n, pipelined):
    # u = 0 is a steady state (f(0) = 0, Lap 0 = 0): every propagator and every
    # Parareal iterate keeps it exactly, and the update norms are 0
    from paper_2304_14074_amd import chlib
    N, J = 4, 6
    p = workloads.Problem(dim=2, n=n, eps=0.02, T=N * J * 2e-5, n_slices=N, j_fine=J)
    ctx = chlib.Context([p])
    st = ctx.new_state()
    print(f"zero state n={n} pipelined={pipelined}", flush=True)
    if pipelined:
        ctx.ch_parareal_run(st, -1.0, 3)
    else:
        for _ in range(4):
            ctx.ch_parareal_iterate(st, -1.0)
    torch.cuda.synchronize()
    assert bool((st["U"] == 0).all())
    assert st["delta"][0].item() == 0.0
    assert int(st["status"][0].item()) == 0
