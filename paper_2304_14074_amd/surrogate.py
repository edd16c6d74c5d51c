"""Training and use of the learned coarse propagator.

Training data are fine trajectories produced by the library's own fine
propagator: for S seeded initial states, u(T_0), u(T_1), ..., u(T_N) with
u(T_{n+1}) = F(u(T_n)).  All S trajectories advance together: one context
whose "slices" are the S current states, so one ch_fine_propagate moves every
trajectory by dT.  The network (ch_nn_*) is trained on the pairs
(u(T_n), u(T_{n+1})) with Adam; weights are BF16 with an FP32 master copy.

The Parareal loop implements the fallback: the learned propagator is used
until the update norm stops contracting (delta^{k+1} >= delta^k, or a
non-finite delta) or the plain propagator, its judge, finds it further from F
than itself in two consecutive iterations; the instance then switches to the
plain propagator and G_old is recomputed with it at the current iterate.
"""
from __future__ import annotations

import copy
import math
import time

import numpy as np
import torch

from . import chlib


def generate_trajectories(prob, u0s: np.ndarray, device="cuda") -> torch.Tensor:
    """u0s: (S, n, n) float64 -> (S, N+1, n, n) float64 on the device."""
    S, n = u0s.shape[0], prob.n
    N = prob.n_slices
    batch = copy.copy(prob)
    batch.n_slices = S
    batch.T = prob.dT * S          # keeps dT and hence dt
    batch.coarse_kind = "approx2"
    ctx = chlib.Context([batch], device=device)
    traj = torch.empty((S, N + 1, n, n), dtype=torch.float64, device=device)
    cur = torch.from_numpy(np.ascontiguousarray(u0s)).to(device).reshape(-1)
    traj[:, 0] = cur.view(S, n, n)
    nxt = torch.empty_like(cur)
    for k in range(N):
        ctx.ch_fine_propagate(cur, nxt)
        traj[:, k + 1] = nxt.view(S, n, n)
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    return traj


def init_weights(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-normal weights, small biases, zero head (G_nn starts as identity)."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    layers = chlib.ch_nn_layers()
    for li, (ci, co, k, _, _, _) in enumerate(layers):
        std = math.sqrt(2.0 / (ci * k * k))
        w = torch.randn(co * ci * k * k, generator=g, dtype=torch.float32) * std
        if li == len(layers) - 1:
            w.zero_()
        parts += [w, torch.zeros(co, dtype=torch.float32)]
    return torch.cat(parts).to(device)


def train(traj: torch.Tensor, steps: int = 3000, batch: int = 16, lr: float = 1e-3,
          seed: int = 0, time_budget_s: float | None = None, w_master=None, log=None,
          k_min: int = 1):
    """Adam with a cosine learning-rate decay over `steps` mini-batches of
    (u(T_n) -> u(T_{n+1})) pairs of the trajectories, n >= k_min.
    The first slice maps seeded noise through the spinodal amplification
    (growth up to exp(dT / (4 eps^2))); Parareal makes that slice exact after
    one iteration, so by default it is left out of the training pairs."""
    dev = traj.device
    S, N1, n, _ = traj.shape
    pairs = [(s, k) for s in range(S) for k in range(k_min, N1 - 1)]
    rng = np.random.default_rng(seed)
    P = chlib.ch_nn_param_count()
    wm = init_weights(seed, dev) if w_master is None else w_master
    wb = torch.empty(P, dtype=torch.bfloat16, device=dev)
    chlib.ch_nn_to_bf16(wm, wb)
    m = torch.zeros(P, dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    grad = torch.empty_like(m)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    ws = chlib.NNWorkspace(batch, n, device=dev)
    idx_s = torch.empty(batch, dtype=torch.long, device=dev)
    step, t0, hist = 0, time.perf_counter(), []
    total = steps
    while step < total:
        order = rng.permutation(len(pairs))
        for b0 in range(0, len(order) - batch + 1, batch):
            sel = [pairs[i] for i in order[b0:b0 + batch]]
            s_i = torch.tensor([a for a, _ in sel], device=dev)
            k_i = torch.tensor([b for _, b in sel], device=dev)
            u = traj[s_i, k_i].contiguous()
            tgt = traj[s_i, k_i + 1].contiguous()
            chlib.ch_nn_train_step(wb, u, tgt, grad, loss, ws)
            step += 1
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * min((step - 1) / max(total, 1), 1.0)))
            chlib.ch_nn_adam(wm, wb, m, v, grad, lr_t, step)
            if step % 50 == 0:
                hist.append((step, loss.item()))
                if log:
                    log(f"step {step} loss {hist[-1][1]:.3e} ({time.perf_counter() - t0:.1f}s)")
            if step >= total or (time_budget_s and time.perf_counter() - t0 > time_budget_s):
                torch.cuda.synchronize()
                return wm, wb, {"steps": step, "loss": hist, "seconds": time.perf_counter() - t0}
    torch.cuda.synchronize()
    return wm, wb, {"steps": step, "loss": hist, "seconds": time.perf_counter() - t0}


def run_parareal(ctx: "chlib.Context", u0: np.ndarray, tol: float, fallback: bool = True,
                 max_iter: int | None = None):
    """Single-instance Parareal to an update norm below tol (or k = N).

    With the learned propagator and the fallback on, the plain propagator
    also judges the learned one before every correction: the mean over the
    swept slices n >= k of ||G(U_n^k) - F_n||_h / ||G_plain(U_n^k) - F_n||_h
    (G(U_n^k) is G_old_n; slices where G_plain equals F are left out).  The
    instance falls back to the plain propagator when the update norm stops
    contracting or when that ratio exceeds 1 in two consecutive iterations.
    Returns iterations, update norms, the judge's ratios, wall time and the
    fallback iteration."""
    p = ctx.problems[0]
    P = p.n ** p.dim
    N = p.n_slices
    kind = p.coarse_kind
    judging = fallback and kind == "neural"
    st = ctx.new_state()
    st["U"][:P] = torch.from_numpy(np.ascontiguousarray(u0).reshape(-1)).to(ctx.device)
    U_in = st["U"][: N * P]                       # slice inputs U_0..U_{N-1}
    if judging:
        # the plain propagator on a context of its own (no kind switching on
        # the timed path); per-slice distances land in one small buffer
        q = copy.copy(p)
        q.coarse_kind = "approx2"
        plain = chlib.Context([q], device=ctx.device)
        Gp = torch.empty(N * P, dtype=torch.float64, device=ctx.device)
        dist = torch.empty((2, N), dtype=torch.float64, device=ctx.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.ch_parareal_iterate(st, tol)
    deltas, judge, fell_back = [], [], None
    while st["c"].k < (max_iter or N):
        k = st["c"].k
        if judging and fell_back is None:
            # one iteration as its two halves, with the judge in between
            ctx.ch_fine_propagate(U_in, st["F"])
            plain.ch_coarse_propagate(U_in, Gp)
            ctx.ch_slice_distance(st["G_old"], st["F"], dist[0])
            ctx.ch_slice_distance(Gp, st["F"], dist[1])
            ctx.ch_parareal_correct(st, tol)
            dn, dp = dist.cpu().numpy()
            sel = dp[k:] > 0
            judge.append(float(np.mean(dn[k:][sel] / dp[k:][sel])) if sel.any() else math.nan)
        else:
            ctx.ch_parareal_iterate(st, tol)
        d = st["delta"][0].item()
        deltas.append(d)
        if d < tol:
            break
        worse = len(judge) >= 2 and min(judge[-2:]) > 1.0
        if (judging and fell_back is None
                and (not math.isfinite(d) or (len(deltas) >= 2 and d >= deltas[-2]) or worse)):
            # plain propagator from now on, G_old recomputed with it at the
            # current iterate U^{k}
            ctx.ch_set_coarse_kind(0, "approx2")
            ctx.ch_coarse_propagate(U_in, st["G_old"])
            fell_back = st["c"].k
    torch.cuda.synchronize()
    ctx.ch_check_status(st)          # raises on a solver cap, non-finite state or time-out
    if judging:
        plain.ch_check_status()
    return {"iterations": len(deltas), "deltas": deltas, "judge": judge,
            "seconds": time.perf_counter() - t0, "fallback_at": fell_back, "U": st["U"],
            "status": int(st["status"][0].item())}


def pair_mse(traj: torch.Tensor, predict, k_min: int = 1, max_pairs: int = 512) -> float:
    """Mean squared error of predict(u(T_n)) against u(T_{n+1}) over pairs."""
    S, N1 = traj.shape[:2]
    tot, cnt = 0.0, 0
    for s in range(S):
        for k in range(k_min, N1 - 1):
            if cnt >= max_pairs:
                return tot / cnt
            d = predict(traj[s, k:k + 1]) - traj[s, k + 1:k + 2]
            tot += float(torch.mean(d * d))
            cnt += 1
    return tot / max(cnt, 1)
