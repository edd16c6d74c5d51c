"""The judge and fallback of the learned coarse propagator run on the
device, inside ch_parareal_iterate: against the oracle's loop (same BF16
weights) for a network that is a constant shift of its input, and a
graph-captured run against the eager one, bit for bit."""
import copy

import numpy as np
import pytest
import torch

import workloads
from oracle import nn as onn, operators, parareal, propagators
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _shift_weights(c):
    th = np.zeros(onn.n_params())
    o = 0
    for name, ci, co, k, _, _, _ in onn.LAYERS:
        o += co * ci * k * k
        if name == "head":
            th[o:o + co] = c
        o += co
    wb = torch.tensor(th, dtype=torch.float32).to(torch.bfloat16)
    return wb.cuda(), wb.to(torch.float64).numpy()


def _problem(N=6, J=20, n=32, nn_base=0):
    return workloads.Problem(dim=2, n=n, eps=0.03, T=N * J * 4e-5, n_slices=N, j_fine=J,
                             coarse_kind="neural", nn_base=nn_base)


@pytest.mark.parametrize("shift,base", [(0.002, 0), (0.05, 0), (0.002, 1), (0.05, 1)])
def test_device_judge_and_fallback_match_the_oracle(shift, base):
    # base 1: the learned propagator on top of the plain one, G_plain(u) + net(u)
    from paper_2304_14074_amd import chlib, surrogate
    p = _problem(nn_base=base)
    wb, th = _shift_weights(shift)
    u0 = workloads.u0_uniform(p.n, 2, 0.3, 41)
    ctx = chlib.Context([p])
    ctx.ch_nn_bind(wb)
    print(f"device judge, shift {shift}", flush=True)
    r = surrogate.run_parareal(ctx, u0, 1e-12)
    plain = copy.copy(p)
    plain.coarse_kind = "approx2"
    ref = parareal.parareal(u0, p.n_slices, lambda u: propagators.fine(p, u),
                            lambda u: propagators.coarse(p, u, nn_params=th),
                            lambda v: operators.norm_h(v, 2), tol=1e-12,
                            fallback_G=lambda u: propagators.coarse(plain, u))
    print("gpu", r["judge"], r["fallback_at"], "oracle", ref["judge"], ref["fallback_at"],
          flush=True)
    assert r["fallback_at"] == ref["fallback_at"]
    assert len(r["judge"]) == len(ref["judge"]) > 0
    for a, b in zip(r["judge"], ref["judge"]):
        assert abs(a - b) <= 1e-3 * abs(b), (r["judge"], ref["judge"])
    assert r["iterations"] == ref["k"]
    U = r["U"].view(p.n_slices + 1, p.n, p.n).cpu().numpy()
    for j in range(p.n_slices + 1):
        assert gu.rel(U[j], ref["final"][j]) < 1e-9, j


@pytest.mark.parametrize("base", [0, 1])
def test_captured_learned_iteration_equals_eager(base):
    from paper_2304_14074_amd import chlib, surrogate
    p = _problem(N=5, nn_base=base)
    wb, _ = _shift_weights(0.05)
    u0 = workloads.u0_uniform(p.n, 2, 0.3, 42)
    outs = []
    for graph in (False, True):
        ctx = chlib.Context([p])
        ctx.ch_nn_bind(wb)
        print(f"learned G run, graph={graph}", flush=True)
        r = surrogate.run_parareal(ctx, u0, 0.0, graph=graph)
        outs.append(r)
    a, b = outs
    assert a["deltas"] == b["deltas"] and a["fallback_at"] == b["fallback_at"]
    assert np.array_equal(np.array(a["judge"]), np.array(b["judge"]), equal_nan=True)
    assert torch.equal(a["U"], b["U"])


def test_plain_base_prediction_and_parallel_propagation_match_the_oracle():
    # G(u) = clip(G_plain(u) + net(u)): the prediction chain and the parallel
    # propagation of every slice against the oracle with the same weights
    from paper_2304_14074_amd import chlib
    p = _problem(N=4, nn_base=1, n=64)
    wb, th = _shift_weights(0.01)
    u0 = workloads.u0_uniform(p.n, 2, 0.3, 43)
    ctx = chlib.Context([p])
    ctx.ch_nn_bind(wb)
    st = ctx.new_state()
    st["U"][: p.n ** 2] = torch.from_numpy(u0.reshape(-1)).cuda()
    ctx.ch_parareal_iterate(st, 0.0)
    torch.cuda.synchronize()
    U = gu.unpack_iter(ctx, st["U"])[0]
    G = lambda u: propagators.coarse(p, u, nn_params=th)
    ref = [u0]
    for _ in range(p.n_slices):
        ref.append(G(ref[-1]))
    for j in range(p.n_slices + 1):
        assert gu.rel(U[j], ref[j]) < 1e-10, j
    out = gu.coarse(ctx, [U[:-1]])[0]
    for j in range(p.n_slices):
        assert gu.rel(out[j], G(U[j])) < 1e-10, j
