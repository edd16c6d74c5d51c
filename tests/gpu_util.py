"""Helpers of the GPU tests: pack/unpack states and run library calls."""
import numpy as np
import torch

from paper_2304_14074_amd import chlib


def npts(p):
    return p.n ** p.dim


def pack_slices(ctx, per_inst_states):
    """per_inst_states[i]: array (N_i, n^d...) -> slice-layout device tensor."""
    out = torch.zeros(ctx.slice_total, dtype=torch.float64)
    for i, arr in enumerate(per_inst_states):
        _, _, so, _ = ctx.layout(i)
        flat = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        out[so:so + flat.size] = torch.from_numpy(flat)
    return out.cuda()


def unpack_slices(ctx, t):
    h = t.cpu().numpy()
    res = []
    for i, p in enumerate(ctx.problems):
        _, _, so, _ = ctx.layout(i)
        P = npts(p)
        res.append(h[so:so + p.n_slices * P].reshape((p.n_slices,) + (p.n,) * p.dim))
    return res


def unpack_iter(ctx, t):
    h = t.cpu().numpy()
    res = []
    for i, p in enumerate(ctx.problems):
        _, _, _, io = ctx.layout(i)
        P = npts(p)
        res.append(h[io:io + (p.n_slices + 1) * P].reshape((p.n_slices + 1,) + (p.n,) * p.dim))
    return res


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def fine(ctx, states, mask=None):
    U = pack_slices(ctx, states)
    F = torch.zeros_like(U)
    ctx.ch_fine_propagate(U, F, mask)
    torch.cuda.synchronize()
    return unpack_slices(ctx, F)


def coarse(ctx, states, mask=None):
    U = pack_slices(ctx, states)
    G = torch.zeros_like(U)
    ctx.ch_coarse_propagate(U, G, mask)
    torch.cuda.synchronize()
    return unpack_slices(ctx, G)
