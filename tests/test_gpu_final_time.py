"""Whole runs to the final time against stored oracle results
(tests/golden/, written by tests/golden/make_goldens.py from the oracle
alone): the serial fine solve of the 2D 128x128 workload to T = 2 in FP64
and with split-BF16 transforms, and all J = 3125 implicit steps of the first
slice of the 2D 256x256 workload.  Each FP64 comparison is judged against
max(1e-11, the floor), the floor being the distance between two equally
correct oracle routes of the same run; the reduced-precision one against
1e-4 at the final time."""
import dataclasses
import os

import numpy as np
import pytest
import torch

import workloads
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _serial_fine(prob, u0):
    from paper_2304_14074_amd import chlib
    one = chlib.Context([dataclasses.replace(prob, n_slices=1, T=prob.dT)])
    n = prob.n
    cur = torch.from_numpy(u0.reshape(-1)).cuda()
    nxt = torch.empty_like(cur)
    out = {}
    for k in range(1, prob.n_slices + 1):
        one.ch_fine_propagate(cur, nxt)
        cur, nxt = nxt, cur
        if k in (32, 64):
            torch.cuda.synchronize()
            out[k // 32] = cur.cpu().numpy().reshape(n, n)
    assert one.ch_check_status() == [0]
    return out


@pytest.mark.parametrize("precision", ["fp64", "split_bf16"])
def test_serial_fine_solve_to_final_time(precision):
    g = np.load(os.path.join(GOLD, "c2_serial_fine.npz"))
    prob = dataclasses.replace(workloads.linear_2d_128(), precision=precision)
    print(f"serial fine solve to T = 2, {precision}", flush=True)
    got = _serial_fine(prob, workloads.linear_2d_128_u0(0))
    for t in (1, 2):
        err = gu.rel(got[t], g[f"T{t}"])
        floor = float(g[f"floor_T{t}"])
        print(f"T = {t}: {precision} vs oracle {err:.2e} (oracle two-route floor {floor:.2e})",
              flush=True)
        bound = max(1e-11, floor) if precision == "fp64" else 1e-4
        assert err <= bound, (t, err, bound)


def test_implicit_fine_slice_full_length():
    path = os.path.join(GOLD, "c3_slice0_fine.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle result missing: python tests/golden/make_goldens.py c3")
    g = np.load(path)
    from paper_2304_14074_amd import chlib
    p = workloads.nonlinear_2d_256()
    one = chlib.Context([dataclasses.replace(p, n_slices=1, T=p.dT)])
    assert one.ch_fine_groups(256, fine_kind="nonlinear") == 16
    u0 = workloads.nonlinear_2d_256_u0(0)
    print("implicit fine slice, 256^2, J = 3125", flush=True)
    out = gu.fine(one, [u0[None]])[0][0]
    assert one.ch_check_status() == [0]
    err, floor = gu.rel(out, g["F"]), float(g["floor"])
    print(f"F(u0) vs oracle {err:.2e} (oracle two-route floor {floor:.2e})", flush=True)
    assert err <= max(1e-11, floor), (err, floor)
