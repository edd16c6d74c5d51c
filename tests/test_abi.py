"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates problems on the host (no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ch.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ch_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ch_create", "ch_fine_propagate", "ch_coarse_propagate", "ch_parareal_iterate", "ch_energy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2304_14074_amd import chlib
    lib = chlib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(chlib.EXPORTS) == set(_declared())


def _create(probs):
    from paper_2304_14074_amd import chlib
    lib = chlib.load()
    arr = (chlib.ChProblem * len(probs))(*[chlib.to_problem(p) for p in probs])
    h = ctypes.c_void_p()
    st = lib.ch_create(arr, len(probs), ctypes.byref(h))
    return lib, st, h


def test_create_and_layout_host_only():
    import workloads
    from paper_2304_14074_amd import chlib
    probs = [workloads.Problem(dim=2, n=64, n_slices=3, j_fine=5),
             workloads.Problem(dim=2, n=128, n_slices=2, j_fine=5),
             workloads.Problem(dim=1, n=128, n_slices=4, j_fine=5)]
    lib, st, h = _create(probs)
    assert st == chlib.CH_OK
    sz = ctypes.c_size_t()
    assert lib.ch_workspace_size(h, ctypes.byref(sz)) == chlib.CH_OK and sz.value > 0
    vals = [ctypes.c_int64() for _ in range(4)]
    assert lib.ch_layout(h, 1, *[ctypes.byref(v) for v in vals]) == chlib.CH_OK
    st_tot, it_tot, so, io = [v.value for v in vals]
    assert st_tot == 3 * 64 * 64 + 2 * 128 * 128 + 4 * 128
    assert it_tot == 4 * 64 * 64 + 3 * 128 * 128 + 5 * 128
    assert so == 3 * 64 * 64 and io == 4 * 64 * 64
    assert lib.ch_layout(h, 3, *[ctypes.byref(v) for v in vals]) == chlib.CH_ERR_ARG
    # compute calls before binding a workspace are refused
    assert lib.ch_fine_propagate(h, ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), None, None) == chlib.CH_ERR_STATE
    lib.ch_destroy(h)


@pytest.mark.parametrize("kw,code", [
    (dict(dim=3), 3), (dict(n=96), 3), (dict(eps=0.0), 1), (dict(n_slices=0), 1),
    (dict(j_fine=0), 1), (dict(dim=1, n=129), 3), (dict(m_coarse=0), 1),
    # Neumann-Neumann fine step: 1D only, no f == 0 form, n + 1 split into
    # N0 pieces of >= 2 intervals, 0 <= theta < 1
    (dict(fine_kind="approx2_dd"), 3), (dict(dim=1, n=63, fine_kind="approx2_dd", f_zero=True), 3),
    (dict(dim=1, n=63, fine_kind="approx2_dd", dd_subdomains=3), 1),
    (dict(dim=1, n=63, fine_kind="approx2_dd", dd_subdomains=64), 1),
    (dict(dim=1, n=63, fine_kind="approx2_dd", dd_theta=1.0), 1),
    (dict(dim=1, n=63, fine_kind="approx2_dd", dd_tol=-1.0), 1),
    (dict(dim=1, n=63, fine_kind="approx2_dd", dd_max=-1), 1)])
def test_create_rejects_bad_problems(kw, code):
    import workloads
    p = workloads.Problem(dim=2, n=64, n_slices=2, j_fine=2)
    for k, v in kw.items():
        setattr(p, k, v)
    lib, st, h = _create([p])
    assert st == code
    assert not h.value


def test_dd_problems_accepted_host_only():
    import workloads
    from paper_2304_14074_amd import chlib
    for n, k in ((127, 8), (127, 64), (63, 1), (15, 2), (31, 16)):
        lib, st, h = _create([workloads.Problem(dim=1, n=n, n_slices=3, j_fine=2,
                                                fine_kind="approx2_dd", dd_subdomains=k)])
        assert st == chlib.CH_OK, (n, k)
        it = (ctypes.c_int32 * 3)()
        assert lib.ch_dd_iterations(h, 0, it, None) == chlib.CH_ERR_STATE
        lib.ch_destroy(h)


def test_status_strings():
    from paper_2304_14074_amd import chlib
    lib = chlib.load()
    assert lib.ch_status_str(0) == b"CH_OK"
    assert lib.ch_status_str(4) == b"CH_ERR_NOCONV"
    assert lib.ch_status_str(6) == b"CH_ERR_TIMEOUT"


def test_status_calls_need_a_workspace():
    import workloads
    from paper_2304_14074_amd import chlib
    lib, st, h = _create([workloads.Problem(dim=2, n=128, n_slices=2, j_fine=5)])
    assert st == chlib.CH_OK
    bits = (ctypes.c_int32 * 1)()
    assert lib.ch_check_status(h, None, bits, None) == chlib.CH_ERR_STATE
    assert lib.ch_set_wait_limit(h, 0.2, 10.0, None) == chlib.CH_ERR_STATE
    lib.ch_destroy(h)


def test_static_forward_refuses_bad_shapes_on_the_host():
    # shapes are checked before any device work: n not divisible by 8, an
    # empty batch, and a batch past the 32 MiB static scratch
    from paper_2304_14074_amd import chlib
    lib = chlib.load()
    p = ctypes.c_void_p(1 << 20)
    assert lib.ch_nn_forward_static(p, p, 1, 100, p, None) == chlib.CH_ERR_ARG
    assert lib.ch_nn_forward_static(p, p, 0, 128, p, None) == chlib.CH_ERR_ARG
    assert lib.ch_nn_forward_static(p, p, 6, 128, p, None) == chlib.CH_ERR_ARG
    assert lib.ch_nn_forward_static(p, p, 2, 256, p, None) == chlib.CH_ERR_ARG


def test_chain_variant_selection_host_only():
    import workloads
    from paper_2304_14074_amd import chlib
    probs = [workloads.Problem(dim=2, n=128, n_slices=2, j_fine=5),
             workloads.Problem(dim=2, n=64, n_slices=2, j_fine=5)]
    lib, st, h = _create(probs)
    assert st == chlib.CH_OK
    g = ctypes.c_int32(0)
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 8
    assert lib.ch_chain_variant(h, 64, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 1
    g.value = 4
    assert lib.ch_chain_variant(h, 64, ctypes.byref(g), 1) == chlib.CH_ERR_UNSUPPORTED
    g.value = 3
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 1) == chlib.CH_ERR_ARG
    g.value = 8
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 1) == chlib.CH_OK
    g.value = 1
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 1) == chlib.CH_OK
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 1
    assert lib.ch_chain_variant(h, 32, ctypes.byref(g), 0) == chlib.CH_ERR_ARG
    lib.ch_destroy(h)
    # 33..64 instances: groups of four (eight would exceed 256 workgroups);
    # more: one workgroup each
    lib, st, h = _create([workloads.Problem(dim=2, n=128, n_slices=1, j_fine=1)] * 40)
    assert st == chlib.CH_OK
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 4
    g.value = 8
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 1) == chlib.CH_ERR_UNSUPPORTED
    lib.ch_destroy(h)
    lib, st, h = _create([workloads.Problem(dim=2, n=128, n_slices=1, j_fine=1)] * 65)
    assert st == chlib.CH_OK
    assert lib.ch_chain_variant(h, 128, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 1
    lib.ch_destroy(h)


def test_fine_groups_selection_host_only():
    import workloads
    from paper_2304_14074_amd import chlib
    lib, st, h = _create([workloads.Problem(dim=2, n=128, n_slices=64, j_fine=5),
                          workloads.Problem(dim=2, n=64, n_slices=2, j_fine=5)])
    assert st == chlib.CH_OK
    g = ctypes.c_int32(0)
    assert lib.ch_fine_groups(h, 128, 0, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 8
    assert lib.ch_fine_groups(h, 64, 0, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 1
    g.value = 4
    assert lib.ch_fine_groups(h, 64, 0, ctypes.byref(g), 1) == chlib.CH_ERR_UNSUPPORTED
    g.value = 1
    assert lib.ch_fine_groups(h, 64, 0, ctypes.byref(g), 1) == chlib.CH_OK
    g.value = 2
    assert lib.ch_fine_groups(h, 128, 0, ctypes.byref(g), 1) == chlib.CH_ERR_ARG
    g.value = 8
    assert lib.ch_fine_groups(h, 128, 0, ctypes.byref(g), 1) == chlib.CH_OK
    g.value = 1
    assert lib.ch_fine_groups(h, 128, 0, ctypes.byref(g), 1) == chlib.CH_OK
    assert lib.ch_fine_groups(h, 128, 0, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 1
    lib.ch_destroy(h)
    # 65 slices, a nonlinear class, a split-precision class: one workgroup per
    # item at n = 128; n = 256 takes groups of eight at any slice count
    probs = [workloads.Problem(dim=2, n=128, n_slices=65, j_fine=5),
             workloads.Problem(dim=2, n=128, n_slices=2, j_fine=5, fine_kind="nonlinear"),
             workloads.Problem(dim=2, n=128, n_slices=2, j_fine=5, precision="split_bf16"),
             workloads.Problem(dim=2, n=256, n_slices=300, j_fine=5)]
    lib, st, h = _create(probs)
    assert st == chlib.CH_OK
    assert lib.ch_fine_groups(h, 128, 0, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 1
    assert lib.ch_fine_groups(h, 256, 0, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 8
    g.value = 4
    assert lib.ch_fine_groups(h, 256, 0, ctypes.byref(g), 1) == chlib.CH_ERR_UNSUPPORTED
    # the implicit class of n = 128 (two slices) takes groups of eight
    assert lib.ch_fine_groups(h, 128, 1, ctypes.byref(g), 0) == chlib.CH_OK and g.value == 8
    g.value = 4
    assert lib.ch_fine_groups(h, 128, 1, ctypes.byref(g), 1) == chlib.CH_ERR_UNSUPPORTED
    g.value = 1
    assert lib.ch_fine_groups(h, 128, 1, ctypes.byref(g), 1) == chlib.CH_OK
    assert lib.ch_fine_groups(h, 128, 2, ctypes.byref(g), 0) == chlib.CH_ERR_ARG
    lib.ch_destroy(h)


def test_pipelined_run_coverage_host_only():
    # ch_parareal_run covers one 2D n = 128 instance with the linear FP64 fine
    # step and coarse scheme (2.4), N >= 2; other contexts are refused on the
    # host, before any workspace exists; a covered context without a bound
    # workspace gets the usual state error
    import workloads
    from paper_2304_14074_amd import chlib
    st_struct = chlib.ChPrState()
    cases = [
        ([workloads.Problem(dim=2, n=64, n_slices=4, j_fine=5)], chlib.CH_ERR_UNSUPPORTED),
        ([workloads.Problem(dim=2, n=128, n_slices=4, j_fine=5)] * 2, chlib.CH_ERR_UNSUPPORTED),
        ([workloads.Problem(dim=2, n=128, n_slices=1, j_fine=5)], chlib.CH_ERR_UNSUPPORTED),
        ([workloads.Problem(dim=2, n=128, n_slices=4, j_fine=5, coarse_kind="stab")],
         chlib.CH_ERR_UNSUPPORTED),
        ([workloads.Problem(dim=2, n=128, n_slices=4, j_fine=5, precision="split_bf16")],
         chlib.CH_ERR_UNSUPPORTED),
        ([workloads.Problem(dim=2, n=128, n_slices=4, j_fine=5)], chlib.CH_ERR_STATE),
    ]
    for probs, code in cases:
        lib, st, h = _create(probs)
        assert st == chlib.CH_OK
        r = lib.ch_parareal_run(h, ctypes.byref(st_struct), 0.0, 3, 0, None)
        assert r == code, (probs[0], len(probs), r)
        lib.ch_destroy(h)
    lib, st, h = _create([workloads.Problem(dim=2, n=128, n_slices=4, j_fine=5)])
    assert lib.ch_parareal_run(h, ctypes.byref(st_struct), 0.0, -1, 0, None) == chlib.CH_ERR_ARG
    assert lib.ch_parareal_run(h, ctypes.byref(st_struct), 0.0, 3, 2, None) == chlib.CH_ERR_ARG
    lib.ch_destroy(h)


@pytest.mark.parametrize("dim,n,i_f,i_c,m", [(1, 15, 1.0, 1.0, 1), (1, 63, 2.0, 1.0, 1),
                                            (2, 6, 2.0, 2.0, 1), (1, 20, 2.0, 1.0, 3)])
def test_linear_bound_constants_match_the_oracle(dim, n, i_f, i_c, m):
    # host-only: alpha and beta of the convergence theorems against the
    # oracle's dense matrix norms of the linearised propagators
    import numpy as np
    from oracle import linear_model as lm
    from paper_2304_14074_amd import chlib
    dT, J, eps = 0.05, 11, 0.0725
    a, b = chlib.ch_linear_bound(dim, n, eps, dT, J, i_f, i_c, m)
    PJ = lm.propagator_matrix(n, dim, dT / J, eps, i_f, J)
    P = lm.propagator_matrix(n, dim, dT / m, eps, i_c, m)
    # the oracle's dense solves carry the condition number of
    # I - i dT D + eps^2 dT D^2 (up to ~1e5 here) times the unit roundoff
    assert abs(a - np.linalg.norm(PJ - P, 2)) <= 1e-10 * a
    assert abs(b - np.linalg.norm(P, 2)) <= 1e-10 * b
