"""ctypes binding of libch.so (C ABI declared in include/ch.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch provides the device memory (workspace, states) and the
stream.  Names mirror the C entry points.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libch.so")

CH_OK, CH_ERR_ARG, CH_ERR_HIP, CH_ERR_UNSUPPORTED, CH_ERR_NOCONV, CH_ERR_STATE, CH_ERR_TIMEOUT = range(7)
FINE = {"linear": 0, "nonlinear": 1, "approx2": 2, "approx2_dd": 3}
NL = {"eyre": 0, "be": 1}
COARSE = {"approx2": 0, "stab": 1, "neural": 2, "eyre": 3}
PREC = {"fp64": 0, "split_bf16": 1}

# every symbol include/ch.h declares
EXPORTS = ("ch_create", "ch_destroy", "ch_workspace_size", "ch_bind_workspace", "ch_layout",
           "ch_fine_propagate", "ch_coarse_propagate", "ch_parareal_iterate",
           "ch_parareal_correct", "ch_energy", "ch_status_str", "ch_last_error",
           "ch_nn_param_count", "ch_nn_layer", "ch_nn_workspace_bytes", "ch_nn_forward",
           "ch_nn_train_step", "ch_nn_adam", "ch_nn_to_bf16", "ch_nn_bind", "ch_set_coarse_kind",
           "ch_parareal_graph_create", "ch_graph_launch", "ch_graph_destroy", "ch_iteration_count",
           "ch_autotune", "ch_fine_variant", "ch_set_iteration", "ch_chain_variant", "ch_fine_groups",
           "ch_parareal_run", "ch_slice_distance", "ch_check_status", "ch_set_wait_limit",
           "ch_nn_forward_static", "ch_linear_bound", "ch_judge_read", "ch_dd_iterations",
           "ch_solver_counts")


class ChProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("eps", ctypes.c_double),
                ("T", ctypes.c_double), ("n_slices", ctypes.c_int32), ("j_fine", ctypes.c_int32),
                ("m_coarse", ctypes.c_int32), ("s_fine", ctypes.c_double),
                ("fine_kind", ctypes.c_int32), ("nl_variant", ctypes.c_int32),
                ("coarse_kind", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("newton_tol", ctypes.c_double), ("newton_max", ctypes.c_int32),
                ("krylov_rtol", ctypes.c_double), ("krylov_max", ctypes.c_int32),
                ("f_zero", ctypes.c_int32), ("nl_krylov_rtol", ctypes.c_double),
                ("nn_base", ctypes.c_int32), ("dd_subdomains", ctypes.c_int32),
                ("dd_theta", ctypes.c_double), ("dd_tol", ctypes.c_double),
                ("dd_max", ctypes.c_int32)]


class ChPrState(ctypes.Structure):
    _fields_ = [("U", ctypes.c_void_p), ("F", ctypes.c_void_p), ("G_old", ctypes.c_void_p),
                ("delta", ctypes.c_void_p), ("status", ctypes.c_void_p), ("k", ctypes.c_int32),
                ("predicted", ctypes.c_int32)]


class CHError(RuntimeError):
    """A failed call; ``status`` holds the ch_status code."""

    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libch.so; raise if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CHError(f"{LIB_PATH} is missing: build it with paper_2304_14074_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    lib.ch_create.argtypes = [ctypes.POINTER(ChProblem), i32, ctypes.POINTER(vp)]
    lib.ch_destroy.argtypes = [vp]
    lib.ch_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.ch_bind_workspace.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.ch_layout.argtypes = [vp, i32, i64p, i64p, i64p, i64p]
    lib.ch_fine_propagate.argtypes = [vp, vp, vp, vp, vp]
    lib.ch_coarse_propagate.argtypes = [vp, vp, vp, vp, vp]
    lib.ch_parareal_iterate.argtypes = [vp, ctypes.POINTER(ChPrState), ctypes.c_double, vp]
    lib.ch_parareal_correct.argtypes = [vp, ctypes.POINTER(ChPrState), ctypes.c_double, vp]
    lib.ch_parareal_run.argtypes = [vp, ctypes.POINTER(ChPrState), ctypes.c_double, i32, i32, vp]
    lib.ch_slice_distance.argtypes = [vp, vp, vp, vp, vp]
    lib.ch_energy.argtypes = [vp, i32, vp, i32, vp, vp]
    lib.ch_status_str.argtypes = [i32]
    lib.ch_status_str.restype = ctypes.c_char_p
    lib.ch_last_error.argtypes = [vp]
    lib.ch_last_error.restype = ctypes.c_char_p
    f32, i64 = ctypes.c_float, ctypes.c_int64
    lib.ch_nn_param_count.argtypes = []
    lib.ch_nn_param_count.restype = i64
    lib.ch_nn_layer.argtypes = [i32] + [ctypes.POINTER(i32)] * 6
    lib.ch_nn_workspace_bytes.argtypes = [i32, i32]
    lib.ch_nn_workspace_bytes.restype = ctypes.c_size_t
    lib.ch_nn_forward.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    lib.ch_nn_forward_static.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.ch_nn_train_step.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
    lib.ch_nn_adam.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
    lib.ch_nn_to_bf16.argtypes = [vp, vp, i64, vp]
    lib.ch_nn_bind.argtypes = [vp, vp]
    lib.ch_set_coarse_kind.argtypes = [vp, i32, i32, vp]
    lib.ch_parareal_graph_create.argtypes = [vp, ctypes.POINTER(ChPrState), ctypes.c_double, vp,
                                             ctypes.POINTER(vp)]
    lib.ch_graph_launch.argtypes = [vp, vp]
    lib.ch_autotune.argtypes = [vp, vp, vp, i32, vp]
    lib.ch_set_iteration.argtypes = [vp, ctypes.POINTER(ChPrState), i32, vp]
    lib.ch_fine_variant.argtypes = [vp, i32, ctypes.POINTER(i32), i32]
    lib.ch_chain_variant.argtypes = [vp, i32, ctypes.POINTER(i32), i32]
    lib.ch_fine_groups.argtypes = [vp, i32, i32, ctypes.POINTER(i32), i32]
    lib.ch_graph_destroy.argtypes = [vp]
    lib.ch_iteration_count.argtypes = [vp, ctypes.POINTER(ChPrState), vp]
    lib.ch_check_status.argtypes = [vp, ctypes.POINTER(ChPrState), ctypes.POINTER(i32), vp]
    lib.ch_set_wait_limit.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.ch_judge_read.argtypes = [vp, i32, dp, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
    lib.ch_dd_iterations.argtypes = [vp, i32, ctypes.POINTER(i32), vp]
    lib.ch_solver_counts.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
    lib.ch_linear_bound.argtypes = [i32, i32, ctypes.c_double, ctypes.c_double, i32, i32,
                                    ctypes.c_double, ctypes.c_double, dp, dp]
    for name in ("ch_nn_layer", "ch_nn_forward", "ch_nn_forward_static", "ch_nn_train_step", "ch_nn_adam", "ch_nn_to_bf16",
                 "ch_nn_bind", "ch_set_coarse_kind", "ch_parareal_graph_create", "ch_graph_launch",
                 "ch_graph_destroy", "ch_iteration_count", "ch_autotune", "ch_fine_variant",
                 "ch_set_iteration", "ch_chain_variant", "ch_fine_groups", "ch_parareal_run",
                 "ch_slice_distance", "ch_check_status", "ch_set_wait_limit",
                 "ch_linear_bound", "ch_judge_read", "ch_dd_iterations", "ch_solver_counts"):
        getattr(lib, name).restype = i32
    for name in ("ch_create", "ch_destroy", "ch_workspace_size", "ch_bind_workspace", "ch_layout",
                 "ch_fine_propagate", "ch_coarse_propagate", "ch_parareal_iterate",
                 "ch_parareal_correct", "ch_energy"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def to_problem(p) -> ChProblem:
    """Marshal any object with the problem attributes (dim, n, eps, ...)."""
    g = lambda name, default: getattr(p, name, default)
    return ChProblem(dim=int(g("dim", 2)), n=int(g("n", 128)), eps=float(g("eps", 0.02)),
                     T=float(g("T", 1.0)), n_slices=int(g("n_slices", 1)),
                     j_fine=int(g("j_fine", 1)), m_coarse=int(g("m_coarse", 1)),
                     s_fine=float(g("s_fine", 2.0)), fine_kind=FINE[g("fine_kind", "linear")],
                     nl_variant=NL[g("nl_variant", "eyre")],
                     coarse_kind=COARSE[g("coarse_kind", "approx2")],
                     precision=PREC[g("precision", "fp64")],
                     newton_tol=float(g("newton_tol", 1e-10)), newton_max=int(g("newton_max", 20)),
                     krylov_rtol=float(g("krylov_rtol", 0.0)),
                     krylov_max=int(g("krylov_max", 200)), f_zero=int(bool(g("f_zero", False))),
                     nl_krylov_rtol=float(g("nl_krylov_rtol", 1e-9)),
                     nn_base=int(g("nn_base", 0)),
                     dd_subdomains=int(g("dd_subdomains", 0)), dd_theta=float(g("dd_theta", 0.0)),
                     dd_tol=float(g("dd_tol", 0.0)), dd_max=int(g("dd_max", 0)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """One ch_ctx with its workspace (a torch uint8 tensor on the device)."""

    def __init__(self, problems, device="cuda"):
        self.lib = load()
        self.problems = list(problems)
        arr = (ChProblem * len(self.problems))(*[to_problem(p) for p in self.problems])
        handle = ctypes.c_void_p()
        st = self.lib.ch_create(arr, len(self.problems), ctypes.byref(handle))
        if st != CH_OK:
            raise CHError(f"ch_create: {self.lib.ch_status_str(st).decode()}")
        self.h = handle
        nbytes = ctypes.c_size_t()
        self._check(self.lib.ch_workspace_size(self.h, ctypes.byref(nbytes)))
        self.device = torch.device(device)
        # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        self._check(self.lib.ch_bind_workspace(self.h, _ptr(self.workspace), nbytes.value, _stream()))
        self.slice_total, self.iter_total = self.layout(0)[:2]

    def _check(self, st):
        if st != CH_OK:
            msg = self.lib.ch_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise CHError(f"{self.lib.ch_status_str(st).decode()}: {msg}", st)

    def layout(self, inst):
        a, b, c, d = (ctypes.c_int64() for _ in range(4))
        self._check(self.lib.ch_layout(self.h, inst, ctypes.byref(a), ctypes.byref(b),
                                       ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def ch_fine_propagate(self, U_in, F_out, mask=None, stream=None):
        self._check(self.lib.ch_fine_propagate(self.h, _ptr(U_in), _ptr(F_out), _ptr(mask), _stream(stream)))

    def ch_coarse_propagate(self, U_in, G_out, mask=None, stream=None):
        self._check(self.lib.ch_coarse_propagate(self.h, _ptr(U_in), _ptr(G_out), _ptr(mask), _stream(stream)))

    def new_state(self):
        """Device buffers of one Parareal run (U_0 of each instance still to be set)."""
        dev = self.device
        n = len(self.problems)
        return {"U": torch.zeros(self.iter_total, dtype=torch.float64, device=dev),
                "F": torch.zeros(self.slice_total, dtype=torch.float64, device=dev),
                "G_old": torch.zeros(self.slice_total, dtype=torch.float64, device=dev),
                "delta": torch.full((n,), float("inf"), dtype=torch.float64, device=dev),
                "status": torch.zeros(n, dtype=torch.int32, device=dev),
                "c": ChPrState(0, 0, 0, 0, 0, 0, 0)}

    @staticmethod
    def _state_struct(state):
        c = state["c"]
        c.U, c.F, c.G_old = state["U"].data_ptr(), state["F"].data_ptr(), state["G_old"].data_ptr()
        c.delta, c.status = state["delta"].data_ptr(), state["status"].data_ptr()
        return c

    def ch_parareal_iterate(self, state, tol, stream=None):
        c = self._state_struct(state)
        self._check(self.lib.ch_parareal_iterate(self.h, ctypes.byref(c), float(tol), _stream(stream)))

    def ch_parareal_correct(self, state, tol, stream=None):
        c = self._state_struct(state)
        self._check(self.lib.ch_parareal_correct(self.h, ctypes.byref(c), float(tol), _stream(stream)))

    def ch_parareal_run(self, state, tol, max_iters, sweep_all=False, stream=None):
        c = self._state_struct(state)
        self._check(self.lib.ch_parareal_run(self.h, ctypes.byref(c), float(tol), int(max_iters),
                                             1 if sweep_all else 0, _stream(stream)))

    def ch_slice_distance(self, A, B, out, stream=None):
        self._check(self.lib.ch_slice_distance(self.h, _ptr(A), _ptr(B), _ptr(out), _stream(stream)))

    def ch_energy(self, inst, u, count, E_out, stream=None):
        self._check(self.lib.ch_energy(self.h, inst, _ptr(u), count, _ptr(E_out), _stream(stream)))

    def ch_parareal_graph_create(self, state, tol, stream):
        """Capture one iteration on a non-default torch stream; returns a handle."""
        c = self._state_struct(state)
        h = ctypes.c_void_p()
        self._check(self.lib.ch_parareal_graph_create(self.h, ctypes.byref(c), float(tol),
                                                      _stream(stream), ctypes.byref(h)))
        return h

    def ch_graph_launch(self, handle, stream):
        self._check(self.lib.ch_graph_launch(handle, _stream(stream)))

    def ch_graph_destroy(self, handle):
        self._check(self.lib.ch_graph_destroy(handle))

    def ch_iteration_count(self, state, stream=None):
        c = self._state_struct(state)
        self._check(self.lib.ch_iteration_count(self.h, ctypes.byref(c), _stream(stream)))
        return c.k

    def ch_check_status(self, state=None, stream=None):
        """Per-instance device flags (list of ints); raises CHError with
        CH_ERR_TIMEOUT or CH_ERR_NOCONV when any is set."""
        bits = (ctypes.c_int32 * len(self.problems))()
        c = ctypes.byref(self._state_struct(state)) if state is not None else None
        self._check(self.lib.ch_check_status(self.h, c, bits, _stream(stream)))
        return list(bits)

    def ch_judge_read(self, inst=0, stream=None):
        """(ratios per iteration (NaN: not judged), fallback_at or None,
        learned propagator still in use) of an instance with the learned G."""
        N = self.problems[inst].n_slices
        r = (ctypes.c_double * N)()
        fb, now = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.ch_judge_read(self.h, inst, r, ctypes.byref(fb), ctypes.byref(now),
                                           _stream(stream)))
        return list(r), (fb.value if fb.value >= 0 else None), bool(now.value)

    def ch_dd_iterations(self, inst=0, stream=None):
        """Neumann-Neumann iterations of each slice's J fine steps in the
        latest fine sweep (list of N ints)."""
        N = self.problems[inst].n_slices
        r = (ctypes.c_int32 * N)()
        self._check(self.lib.ch_dd_iterations(self.h, inst, r, _stream(stream)))
        return list(r)

    def ch_solver_counts(self, inst=0, stream=None):
        """(Newton iterations, CG operator applications) of each slice's J
        implicit fine steps in the latest fine sweep (two lists of N ints)."""
        N = self.problems[inst].n_slices
        a, b = (ctypes.c_int32 * N)(), (ctypes.c_int32 * N)()
        self._check(self.lib.ch_solver_counts(self.h, inst, a, b, _stream(stream)))
        return list(a), list(b)

    def ch_set_wait_limit(self, group_seconds=0.2, pipe_seconds=10.0, stream=None):
        self._check(self.lib.ch_set_wait_limit(self.h, float(group_seconds), float(pipe_seconds),
                                               _stream(stream)))

    def ch_set_iteration(self, state, k, stream=None):
        c = self._state_struct(state)
        self._check(self.lib.ch_set_iteration(self.h, ctypes.byref(c), k, _stream(stream)))

    def ch_autotune(self, U_in, F_out, steps=20, stream=None):
        self._check(self.lib.ch_autotune(self.h, _ptr(U_in), _ptr(F_out), steps, _stream(stream)))

    def ch_fine_variant(self, n, waves=None):
        w = ctypes.c_int32(0 if waves is None else waves)
        self._check(self.lib.ch_fine_variant(self.h, n, ctypes.byref(w), 0 if waves is None else 1))
        return w.value

    def ch_chain_variant(self, n, groups=None):
        g = ctypes.c_int32(0 if groups is None else groups)
        self._check(self.lib.ch_chain_variant(self.h, n, ctypes.byref(g), 0 if groups is None else 1))
        return g.value

    def ch_fine_groups(self, n, groups=None, fine_kind="linear"):
        g = ctypes.c_int32(0 if groups is None else groups)
        self._check(self.lib.ch_fine_groups(self.h, n, FINE[fine_kind], ctypes.byref(g),
                                            0 if groups is None else 1))
        return g.value

    def autotune(self, U_in, F_out, cache_path=None, steps=20):
        """Tuned launch configurations of the linear FP64 fine sweep per grid
        size, {n: (waves, groups)}, from a JSON cache keyed by GPU
        architecture and grid size when present, else measured and cached."""
        import json
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        sizes = sorted({p.n for p in self.problems if p.dim == 2
                        and getattr(p, "fine_kind", "linear") == "linear"
                        and getattr(p, "precision", "fp64") == "fp64"})
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        entry = cache.get(arch, {})
        key = lambda n: f"linear-fp64-n{n}-launch"
        if all(key(n) in entry for n in sizes):
            for n in sizes:
                self.ch_fine_variant(n, entry[key(n)]["waves"])
                self.ch_fine_groups(n, entry[key(n)]["groups"])
            return {n: (entry[key(n)]["waves"], entry[key(n)]["groups"]) for n in sizes}, True
        self.ch_autotune(U_in, F_out, steps)
        chosen = {n: (self.ch_fine_variant(n), self.ch_fine_groups(n)) for n in sizes}
        if cache_path:
            entry.update({key(n): {"waves": w, "groups": g} for n, (w, g) in chosen.items()})
            cache[arch] = entry
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        return chosen, False

    def ch_nn_bind(self, w_bf16):
        self._nn_w = w_bf16          # keep the weights alive while bound
        self._check(self.lib.ch_nn_bind(self.h, _ptr(w_bf16)))

    def ch_set_coarse_kind(self, inst, kind, stream=None):
        self._check(self.lib.ch_set_coarse_kind(self.h, inst, COARSE[kind], _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.ch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ch_linear_bound(dim, n, eps, dT, J, i_fine, i_coarse, m_coarse=1):
    """(alpha, beta) of the convergence theorems for linear pairings."""
    a, b = ctypes.c_double(), ctypes.c_double()
    st = load().ch_linear_bound(dim, n, eps, dT, J, m_coarse, i_fine, i_coarse, ctypes.byref(a),
                                ctypes.byref(b))
    if st != CH_OK:
        raise CHError(f"ch_linear_bound: {load().ch_status_str(st).decode()}", st)
    return a.value, b.value


# ------------------------------------------------ learned coarse propagator
def _nn_check(st, what):
    if st != CH_OK:
        raise CHError(f"{what}: {load().ch_status_str(st).decode()}")


def ch_nn_param_count() -> int:
    return int(load().ch_nn_param_count())


def ch_nn_layers():
    lib = load()
    out, l = [], 0
    while True:
        v = [ctypes.c_int32() for _ in range(6)]
        if lib.ch_nn_layer(l, *[ctypes.byref(x) for x in v]) != CH_OK:
            return out
        out.append(tuple(x.value for x in v))
        l += 1


class NNWorkspace:
    """Activation workspace of the surrogate for a given batch and grid."""

    def __init__(self, batch, n, device="cuda"):
        nbytes = int(load().ch_nn_workspace_bytes(batch, n))
        if nbytes == 0:
            raise CHError("bad surrogate workspace shape")
        self.batch, self.n = batch, n
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.grad = None


def ch_nn_forward(w_bf16, u, out, ws: NNWorkspace, stream=None):
    b, n = u.shape[0], u.shape[-1]
    _nn_check(load().ch_nn_forward(_ptr(w_bf16), _ptr(u), b, n, _ptr(ws.buf), _ptr(out),
                                   _stream(stream)), "ch_nn_forward")


def ch_nn_forward_static(w_bf16, u, out, stream=None):
    """The forward pass without a workspace (the library's static device
    scratch); raises CHError (CH_ERR_ARG) when the batch exceeds it."""
    b, n = u.shape[0], u.shape[-1]
    st = load().ch_nn_forward_static(_ptr(w_bf16), _ptr(u), b, n, _ptr(out), _stream(stream))
    if st != CH_OK:
        raise CHError(f"ch_nn_forward_static: {load().ch_status_str(st).decode()}", st)


def ch_nn_train_step(w_bf16, u, target, grad, loss, ws: NNWorkspace, stream=None):
    b, n = u.shape[0], u.shape[-1]
    _nn_check(load().ch_nn_train_step(_ptr(w_bf16), _ptr(u), _ptr(target), b, n, _ptr(ws.buf),
                                      _ptr(grad), _ptr(loss), _stream(stream)), "ch_nn_train_step")


def ch_nn_adam(w_master, w_bf16, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _nn_check(load().ch_nn_adam(_ptr(w_master), _ptr(w_bf16), _ptr(m), _ptr(v), _ptr(grad),
                                w_master.numel(), lr, beta1, beta2, eps, step, _stream(stream)),
              "ch_nn_adam")


def ch_nn_to_bf16(w_master, w_bf16, stream=None):
    _nn_check(load().ch_nn_to_bf16(_ptr(w_master), _ptr(w_bf16), w_master.numel(), _stream(stream)),
              "ch_nn_to_bf16")
