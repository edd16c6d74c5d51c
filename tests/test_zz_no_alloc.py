"""The allocation-free forward pass of the learned coarse propagator
(ch_nn_forward_static, static device scratch) against the workspace form
(ch_nn_forward): same kernels, so the same values bit for bit, on two calls
in a row with the second smaller; sizes past the static scratch are refused
on the host."""
import pytest
import torch

from paper_2304_14074_amd import chlib, surrogate

pytestmark = pytest.mark.gpu


def _weights():
    wm = surrogate.init_weights(seed=3)
    # a non-zero head, so the network's output is not the identity
    wm += 0.01 * torch.randn(wm.shape, generator=torch.Generator().manual_seed(4)).cuda()
    wb = torch.empty(wm.numel(), dtype=torch.bfloat16, device="cuda")
    chlib.ch_nn_to_bf16(wm, wb)
    return wb


def _workspace_forward(wb, u):
    ws = chlib.NNWorkspace(u.shape[0], u.shape[-1])
    out = torch.empty_like(u)
    chlib.ch_nn_forward(wb, u, out, ws)
    torch.cuda.synchronize()
    return out


def test_static_forward_equals_workspace_forward_twice():
    wb = _weights()
    g = torch.Generator().manual_seed(5)
    u1 = (0.6 * (2 * torch.rand((5, 128, 128), generator=g, dtype=torch.float64) - 1)).cuda()
    u2 = (0.6 * (2 * torch.rand((2, 64, 64), generator=g, dtype=torch.float64) - 1)).cuda()
    want1 = _workspace_forward(wb, u1)
    want2 = _workspace_forward(wb, u2)
    print("static forward: batch 5 at n = 128, then batch 2 at n = 64", flush=True)
    o1 = torch.full_like(u1, float("nan"))
    chlib.ch_nn_forward_static(wb, u1, o1)
    torch.cuda.synchronize()
    o2 = torch.full_like(u2, float("nan"))
    chlib.ch_nn_forward_static(wb, u2, o2)
    torch.cuda.synchronize()
    assert torch.equal(o1, want1)
    assert torch.equal(o2, want2)
    assert float((o1 - u1).abs().max()) > 0.0          # the network did something


def test_static_forward_refuses_batches_past_the_scratch():
    wb = _weights()
    u = torch.zeros((6, 128, 128), dtype=torch.float64, device="cuda")
    out = torch.empty_like(u)
    with pytest.raises(chlib.CHError) as e:
        chlib.ch_nn_forward_static(wb, u, out)
    assert e.value.status == chlib.CH_ERR_ARG
