"""A captured Parareal iteration replayed as a hipGraph gives the eager
iterates bit for bit, replay after replay (ragged batch of instances, one of
them on the multi-workgroup coarse sweep)."""
import numpy as np
import pytest
import torch

import workloads
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _problems():
    return [workloads.Problem(dim=2, n=64, eps=0.03, T=4 * 12 * 4e-5, n_slices=4, j_fine=12),
            workloads.Problem(dim=2, n=32, eps=0.02, T=3 * 9 * 4e-5, n_slices=3, j_fine=9),
            workloads.Problem(dim=1, n=128, eps=0.03, T=3 * 20 * 1e-4, n_slices=3, j_fine=20),
            # n = 128: the coarse sweep runs on a group of four workgroups
            workloads.Problem(dim=2, n=128, eps=0.02, T=3 * 6 * 2e-5, n_slices=3, j_fine=6)]


def _init(ctx, st):
    for i, p in enumerate(ctx.problems):
        _, _, _, io = ctx.layout(i)
        u0 = workloads.u0_uniform(p.n, p.dim, 0.3, 30 + i).reshape(-1)
        st["U"][io:io + u0.size] = torch.from_numpy(u0).cuda()


def test_graph_replays_match_eager_iterations():
    from paper_2304_14074_amd import chlib
    K = 4
    ctx = chlib.Context(_problems())
    eager = ctx.new_state()
    _init(ctx, eager)
    ctx.ch_parareal_iterate(eager, 0.0)
    ref = []
    for _ in range(K):
        ctx.ch_parareal_iterate(eager, 0.0)
        torch.cuda.synchronize()
        ref.append(eager["U"].clone())
    s = torch.cuda.Stream()
    g = ctx.new_state()
    _init(ctx, g)
    with torch.cuda.stream(s):
        ctx.ch_parareal_iterate(g, 0.0, stream=s)   # prediction (eager)
        h = ctx.ch_parareal_graph_create(g, 0.0, s)
        for k in range(K):
            ctx.ch_graph_launch(h, s)
            s.synchronize()
            junk = torch.randn(1000, device="cuda").sum().item()   # eager work between replays
            assert np.isfinite(junk)
            assert torch.equal(g["U"], ref[k]), k
        assert ctx.ch_iteration_count(g, stream=s) == K
        ctx.ch_graph_destroy(h)


def test_graph_accepts_learned_coarse():
    # the judge and the fallback run on the device, so a learned-propagator
    # iteration can be captured (replays against eager iterations: the judge
    # tests)
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=32, eps=0.02, T=2 * 5 * 4e-5, n_slices=2, j_fine=5,
                          coarse_kind="neural")
    ctx = chlib.Context([p])
    st = ctx.new_state()
    s = torch.cuda.Stream()
    w = torch.zeros(chlib.ch_nn_param_count(), dtype=torch.bfloat16, device="cuda")
    ctx.ch_nn_bind(w)
    with torch.cuda.stream(s):
        ctx.ch_parareal_iterate(st, 0.0, stream=s)
        h = ctx.ch_parareal_graph_create(st, 0.0, s)
        ctx.ch_graph_launch(h, s)
        s.synchronize()
        ctx.ch_graph_destroy(h)
    assert ctx.ch_check_status(st) == [0]
