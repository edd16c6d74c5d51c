"""FP64 reference of the convolutional coarse surrogate (test infrastructure).

The learned coarse propagator maps u(T_n) to u(T_{n+1}) on an n x n grid as
u + net(u).  net is a 4-level encoder-decoder of 3x3 convolutions with zero
padding (the field and its features vanish on the Dirichlet boundary),
stride-2 convolutions going down, nearest x2 upsampling and channel
concatenation with the skip features going up, LeakyReLU(0.1) activations
and a 1x1 head.  Parameter vector layout: for each layer in LAYERS order,
W[c_out][c_in][k][k] followed by b[c_out].

Written with plain PyTorch CPU float64 ops (conv2d, nearest interpolation,
autograd); nothing here is shared with the HIP implementation.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fnn

SLOPE = 0.1
# (name, c_in, c_out, k, stride, act, concat_with) -- concat_with names the
# skip tensor joined (first) with the upsampled input of a decoder layer.
LAYERS = [
    ("c1a", 1, 16, 3, 1, True, None),
    ("c1b", 16, 16, 3, 1, True, None),
    ("d2", 16, 32, 3, 2, True, None),
    ("c2", 32, 32, 3, 1, True, None),
    ("d3", 32, 64, 3, 2, True, None),
    ("c3", 64, 64, 3, 1, True, None),
    ("d4", 64, 64, 3, 2, True, None),
    ("c4", 64, 64, 3, 1, True, None),
    ("u3", 128, 64, 3, 1, True, "c3"),
    ("u2", 96, 32, 3, 1, True, "c2"),
    ("u1", 48, 16, 3, 1, True, "c1b"),
    ("head", 16, 1, 1, 1, False, None),
]


def n_params(layers=LAYERS) -> int:
    return sum(co * ci * k * k + co for _, ci, co, k, _, _, _ in layers)


def unpack(theta: torch.Tensor, layers=LAYERS):
    out, o = {}, 0
    for name, ci, co, k, _, _, _ in layers:
        w = theta[o:o + co * ci * k * k].reshape(co, ci, k, k)
        o += co * ci * k * k
        b = theta[o:o + co]
        o += co
        out[name] = (w, b)
    return out


def forward(theta: torch.Tensor, u: torch.Tensor, layers=LAYERS) -> torch.Tensor:
    """u: (batch, n, n) float64 -> u + net(u)."""
    p = unpack(theta, layers)
    x = u[:, None]
    feats = {}
    for name, ci, co, k, stride, act, cat in layers:
        w, b = p[name]
        if cat is not None:
            x = torch.cat([feats[cat], Fnn.interpolate(x, scale_factor=2, mode="nearest")], dim=1)
        x = Fnn.conv2d(x, w, b, stride=stride, padding=k // 2)
        if act:
            x = Fnn.leaky_relu(x, SLOPE)
        feats[name] = x
    return u + x[:, 0]


def loss_and_grad(theta: np.ndarray, u: np.ndarray, target: np.ndarray, layers=LAYERS):
    """MSE over all points of (forward(u) - target) and its gradient (FP64)."""
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    pred = forward(th, torch.tensor(u, dtype=torch.float64), layers)
    loss = torch.mean((pred - torch.tensor(target, dtype=torch.float64)) ** 2)
    loss.backward()
    return float(loss.detach()), th.grad.numpy().copy()


OUT_BOUND = 1.5


def surrogate_step(theta, u: np.ndarray, base: np.ndarray | None = None) -> np.ndarray:
    """G_nn(u) for one state (n x n), FP64: u + net(u), or base + net(u) when a
    base state is given (the learned propagator on top of the plain one, base
    = G_plain(u)), clipped to [-1.5, 1.5] (the propagator is applied
    repeatedly in the coarse sweep, possibly far from its training states;
    training uses the unclipped output)."""
    with torch.no_grad():
        th = torch.as_tensor(np.asarray(theta, dtype=np.float64))
        ut = torch.tensor(u[None], dtype=torch.float64)
        out = forward(th, ut)[0].numpy()
        if base is not None:
            out = base + (out - u)
        return np.clip(out, -OUT_BOUND, OUT_BOUND)
