"""The autotuner of the linear FP64 fine sweep on the GPU: it times one
workgroup per slice (each wave count) against groups of workgroups per slice
(each group size) for every grid-size class of a ragged batch, the chosen
configuration gives the states of the default one to rounding and matches
the oracle, and a cached choice is applied without measuring again."""
import numpy as np
import pytest
import torch

import workloads
from oracle import propagators
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _batch():
    probs = []
    for n, N in ((64, 3), (128, 2), (256, 1)):
        probs.append(workloads.Problem(dim=2, n=n, eps=0.03, T=N * 4 * 2e-5, n_slices=N,
                                       j_fine=4))
    return probs


def test_autotune_chooses_a_launch_per_class_and_keeps_the_states(tmp_path):
    from paper_2304_14074_amd import chlib
    probs = _batch()
    rng = np.random.default_rng(77)
    states = [0.4 * rng.uniform(-1, 1, (p.n_slices, p.n, p.n)) for p in probs]
    ref_ctx = chlib.Context(probs)
    ref = gu.fine(ref_ctx, states)
    ctx = chlib.Context(probs)
    U = gu.pack_slices(ctx, states)
    F = torch.zeros_like(U)
    cache = str(tmp_path / "tune.json")
    print("autotune", flush=True)
    chosen, cached = ctx.autotune(U, F, cache_path=cache, steps=2)
    assert not cached and set(chosen) == {64, 128, 256}
    assert chosen[128][1] in (1, 4, 8) and chosen[256][1] in (1, 8) and chosen[64][1] == 1
    out = gu.fine(ctx, states)
    assert ctx.ch_check_status() == [0, 0, 0]
    for i, p in enumerate(probs):
        for s in range(p.n_slices):
            assert gu.rel(out[i][s], ref[i][s]) < TOL, (p.n, s)
    # one slice per class against the oracle
    for i, p in enumerate(probs):
        assert gu.rel(out[i][0], propagators.fine(p, states[i][0], route="sine")) < TOL, p.n
    # a second context takes the cached choice
    ctx2 = chlib.Context(probs)
    chosen2, cached2 = ctx2.autotune(U, F, cache_path=cache)
    assert cached2 and chosen2 == chosen
    assert all(ctx2.ch_fine_groups(n) == g for n, (_, g) in chosen.items())
