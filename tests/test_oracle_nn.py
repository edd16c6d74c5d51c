"""Pins of the FP64 surrogate reference: central differences on a tiny net,
and its convolutions against explicit loops (padding, stride, orientation)."""
import numpy as np
import torch

from oracle import nn

TINY = [("a", 1, 4, 3, 1, True, None), ("d", 4, 4, 3, 2, True, None),
        ("u", 8, 4, 3, 1, True, "a"), ("h", 4, 1, 1, 1, False, None)]


def test_param_count_of_the_surrogate():
    assert nn.n_params() == 254065


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    th = 0.3 * rng.standard_normal(nn.n_params(TINY))
    u = rng.uniform(-1, 1, (2, 8, 8))
    tgt = rng.uniform(-1, 1, (2, 8, 8))
    _, g = nn.loss_and_grad(th, u, tgt, TINY)
    for i in rng.choice(len(th), 25, replace=False):
        e = np.zeros_like(th)
        e[i] = 1e-6
        lp, _ = nn.loss_and_grad(th + e, u, tgt, TINY)
        lm, _ = nn.loss_and_grad(th - e, u, tgt, TINY)
        fd = (lp - lm) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def _conv_loops(x, w, b, stride, pad):
    C, H, W = x.shape
    co, ci, k, _ = w.shape
    Ho, Wo = (H + 2 * pad - k) // stride + 1, (W + 2 * pad - k) // stride + 1
    out = np.zeros((co, Ho, Wo))
    for o in range(co):
        for y in range(Ho):
            for xx in range(Wo):
                s = b[o]
                for c in range(ci):
                    for dy in range(k):
                        for dx in range(k):
                            iy, ix = y * stride + dy - pad, xx * stride + dx - pad
                            if 0 <= iy < H and 0 <= ix < W:
                                s += w[o, c, dy, dx] * x[c, iy, ix]
                out[o, y, xx] = s
    return out


def test_network_layers_match_loop_convolutions():
    rng = np.random.default_rng(1)
    th = 0.5 * rng.standard_normal(nn.n_params(TINY))
    u = rng.uniform(-1, 1, (1, 6, 6))
    p = {k: (w.numpy(), b.numpy()) for k, (w, b) in nn.unpack(torch.tensor(th), TINY).items()}
    lr = lambda z: np.where(z > 0, z, nn.SLOPE * z)
    a = lr(_conv_loops(u, *p["a"], 1, 1))
    d = lr(_conv_loops(a, *p["d"], 2, 1))
    up = np.repeat(np.repeat(d, 2, axis=1), 2, axis=2)
    uu = lr(_conv_loops(np.concatenate([a, up]), *p["u"], 1, 1))
    h = _conv_loops(uu, *p["h"], 1, 0)
    ref = u[0] + h[0]
    got = nn.forward(torch.tensor(th), torch.tensor(u), TINY)[0].numpy()
    assert np.max(np.abs(got - ref)) < 1e-12


def _constant_shift_theta(c):
    # every weight and bias zero except the 1x1 head's bias: all hidden
    # features vanish and the network adds the constant c to its input
    th = np.zeros(nn.n_params())
    o = 0
    for name, ci, co, k, _, _, _ in nn.LAYERS:
        o += co * ci * k * k
        if name == "head":
            th[o:o + co] = c
        o += co
    return th


def test_surrogate_step_clips_only_outside_the_bound():
    # with a zero network plus head bias c, forward(u) = u + c exactly; the
    # coarse propagator clips that to [-1.5, 1.5] and leaves the rest as is
    u = np.random.default_rng(5).uniform(-1, 1, (16, 16))
    for c in (0.7, -0.7):
        th = _constant_shift_theta(c)
        raw = nn.forward(torch.tensor(th), torch.tensor(u[None]))[0].numpy()
        assert np.max(np.abs(raw - (u + c))) == 0.0
        got = nn.surrogate_step(th, u)
        out = np.abs(u + c) > nn.OUT_BOUND
        assert out.any() and (~out).any()
        assert np.array_equal(got[~out], raw[~out])
        assert np.all(got[out] == np.sign(c) * nn.OUT_BOUND)


def test_surrogate_step_equals_forward_inside_the_bound():
    rng = np.random.default_rng(6)
    th = 0.05 * rng.standard_normal(nn.n_params())
    u = rng.uniform(-0.5, 0.5, (16, 16))
    raw = nn.forward(torch.tensor(th), torch.tensor(u[None]))[0].numpy()
    assert np.max(np.abs(raw)) < nn.OUT_BOUND
    assert np.array_equal(nn.surrogate_step(th, u), raw)
