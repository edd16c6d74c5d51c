"""Training and use of the learned coarse propagator.

Training data are fine trajectories produced by the library's own fine
propagator: for S seeded initial states, u(T_0), u(T_1), ..., u(T_N) with
u(T_{n+1}) = F(u(T_n)).  All S trajectories advance together: one context
whose "slices" are the S current states, so one ch_fine_propagate moves every
trajectory by dT.  The network (ch_nn_*) is trained on the pairs
(u(T_n), u(T_{n+1})) with Adam; weights are BF16 with an FP32 master copy.

The library implements the fallback on the device (ch_judge_read): the
learned propagator is used until the update norm stops contracting
(delta^{k+1} >= delta^k, or a non-finite delta) or the plain propagator, its
judge, finds it further from F than itself in two consecutive iterations;
the instance then switches to the plain propagator and G_old is recomputed
with it at the current iterate.
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


def plain_coarse_of(prob, traj: torch.Tensor) -> torch.Tensor:
    """G_plain(u(T_n)) for every state of the trajectories (S, N+1, n, n):
    the plain coarse propagator (2.4) of the problem, all states at once."""
    S, N1, n, _ = traj.shape
    batch = copy.copy(prob)
    batch.n_slices = S * N1
    batch.T = prob.dT * S * N1
    batch.coarse_kind = "approx2"
    ctx = chlib.Context([batch], device=traj.device)
    out = torch.empty_like(traj)
    ctx.ch_coarse_propagate(traj.reshape(-1), out.view(-1))
    torch.cuda.synchronize()
    ctx.ch_check_status()
    return out


def train(traj: torch.Tensor, steps: int = 3000, batch: int = 16, lr: float = 1e-3,
          seed: int = 0, time_budget_s: float | None = None, w_master=None, log=None,
          k_min: int = 1, base: torch.Tensor | None = None):
    """Adam with a cosine learning-rate decay over `steps` mini-batches of
    (u(T_n) -> u(T_{n+1})) pairs of the trajectories, n >= k_min.
    The first slice maps seeded noise through the spinodal amplification
    (growth up to exp(dT / (4 eps^2))); Parareal makes that slice exact after
    one iteration, so by default it is left out of the training pairs.
    With base = G_plain of every trajectory state (plain_coarse_of), the
    network learns the plain propagator's defect: the loss of u + net(u)
    against u(T_{n+1}) - G_plain(u) + u is that of G_plain(u) + net(u)
    against u(T_{n+1})."""
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
            if base is not None:
                tgt = tgt - base[s_i, k_i] + u
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


def run_parareal(ctx: "chlib.Context", u0: np.ndarray, tol: float, max_iter: int | None = None,
                 graph: bool = False):
    """Single-instance Parareal to an update norm below tol (or k = N), one
    ch_parareal_iterate per iteration (graph=True: one captured iteration,
    replayed), reading the update norm after each.

    With the learned propagator, the library judges it against the plain
    propagator and falls back to the plain one on the device (ch_judge_read).
    Returns iterations, update norms, the judge's ratios of the judged
    iterations, wall time (from the upload of U_0 to the last norm read) and
    the fallback iteration."""
    p = ctx.problems[0]
    P = p.n ** p.dim
    N = p.n_slices
    st = ctx.new_state()
    s = torch.cuda.Stream() if graph else torch.cuda.current_stream()
    h = None
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st["U"][:P] = torch.from_numpy(np.ascontiguousarray(u0).reshape(-1)).to(ctx.device)
        ctx.ch_parareal_iterate(st, tol, stream=s)
        if graph:
            h = ctx.ch_parareal_graph_create(st, tol, s)
        deltas = []
        while len(deltas) < (max_iter or N):
            if graph:
                ctx.ch_graph_launch(h, s)
            else:
                ctx.ch_parareal_iterate(st, tol, stream=s)
            d = st["delta"][0].item()
            deltas.append(d)
            if d < tol:
                break
        s.synchronize()
        secs = time.perf_counter() - t0
        if h is not None:
            ctx.ch_graph_destroy(h)
        ctx.ch_iteration_count(st, stream=s)
        ctx.ch_check_status(st, stream=s)  # raises on a cap, a non-finite state or a time-out
        judge, fell_back = [], None
        if p.coarse_kind == "neural":
            ratios, fell_back, _ = ctx.ch_judge_read(0, stream=s)
            judge = ratios[:fell_back if fell_back is not None else len(deltas)]
    return {"iterations": len(deltas), "deltas": deltas, "judge": judge,
            "seconds": secs, "fallback_at": fell_back, "U": st["U"],
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
