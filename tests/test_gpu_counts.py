"""Solver counts the group kernels record on the device (the implicit fine
step (2.3) by Newton with spectral CG, Section 3): per slice, the Newton
iterations of its J steps match the oracle's (the same stop on the Newton
step; floating point may move a decision near the tolerance by one
iteration per step), every Newton iteration takes at least one CG operator
application, and a class run on one workgroup per slice refuses to report
(it does not count)."""
import numpy as np
import pytest

import workloads
from oracle import schemes
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_newton_group_counts_match_the_oracle():
    from paper_2304_14074_amd import chlib
    n, J = 128, 3
    p = workloads.Problem(dim=2, n=n, eps=0.03, T=2 * J * 1e-4, n_slices=2, j_fine=J,
                          fine_kind="nonlinear")
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(n, fine_kind="nonlinear") == 8
    rng = np.random.default_rng(91)
    X = np.stack([0.3 * rng.uniform(-1, 1, (n, n)), 0.25 + 0.05 * rng.standard_normal((n, n))])
    print("newton group counts", flush=True)
    gu.fine(ctx, [X])
    assert ctx.ch_check_status() == [0]
    newton, applies = ctx.ch_solver_counts(0)
    for s in range(2):
        v, total = X[s], 0
        for _ in range(J):
            hist = []
            v = schemes.step_newton_pcg(v, p.dt, p.eps, "eyre", p.newton_tol, p.newton_max,
                                        history=hist)
            total += len(hist)
        assert J <= newton[s] <= J * p.newton_max
        assert abs(newton[s] - total) <= J, (s, newton[s], total)
        assert applies[s] >= newton[s]


def test_one_workgroup_classes_do_not_count():
    from paper_2304_14074_amd import chlib
    p = workloads.Problem(dim=2, n=64, eps=0.03, T=2e-4, n_slices=2, j_fine=1,
                          fine_kind="nonlinear")
    ctx = chlib.Context([p])
    assert ctx.ch_fine_groups(64, fine_kind="nonlinear") == 1
    gu.fine(ctx, [np.zeros((2, 64, 64))])
    with pytest.raises(chlib.CHError) as e:
        ctx.ch_solver_counts(0)
    assert e.value.status == chlib.CH_ERR_UNSUPPORTED
