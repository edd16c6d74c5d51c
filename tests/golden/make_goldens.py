"""Write the stored expected values of the long GPU runs (tests/golden/*.npz).

Calls the FP64 oracle only.  Each file holds the oracle's states and, as the
noise floor of the comparison, the relative L2 distance between two equally
correct oracle routes of the same run (different rounding).

  c2_serial_fine.npz -- the 2D 128x128 workload (eps = 0.02, u0 = 0.05 U(-1,1)
      seed 0, N = 64, J = 1563): the serial fine solve F^n(u0) at T = 1
      (n = 32) and T = 2 (n = 64) by the sparse-LU route; floors: the largest
      distance between it and two sine-basis routes (dense and FFT transforms).
  c3_slice0_fine.npz -- the 2D 256x256 implicit workload (eps = 0.015,
      u0 = 0.25 + 0.05 N(0,1) seed 0, dt = 1e-5): F(u0) = all J = 3125 steps of
      slice 0, scheme (2.3) by Newton (stop 1e-10) with PCG solves, sine
      transforms as dense products; floor: the largest distance between it and
      two more routes (FFT transforms; another preconditioner shift).

Run:  python tests/golden/make_goldens.py [c2|c3]   (minutes to an hour)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import propagators, schemes  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_c2():
    """Three routes of the serial fine solve: sparse LU, the sine basis with
    dense transforms, the sine basis with FFT transforms; the floor is the
    largest of their pairwise distances."""
    p = workloads.linear_2d_128()
    u0 = workloads.linear_2d_128_u0(0)
    step = {"lu": lambda u: schemes.step_stab(u, p.dt, p.eps, p.s_fine),
            "dense": lambda u: schemes.step_stab_dst(u, p.dt, p.eps, p.s_fine),
            "fft": lambda u: schemes.step_stab_dst(u, p.dt, p.eps, p.s_fine, transform="fft")}
    out = {}
    for route, f in step.items():
        u = u0.copy()
        t0 = time.time()
        for n in range(1, p.n_slices + 1):
            for _ in range(p.j_fine):
                u = f(u)
            if n in (32, 64):
                out[(route, n // 32)] = u.copy()
        print(f"c2 {route}: {time.time() - t0:.0f} s", flush=True)
    res = {}
    for t in (1, 2):
        res[f"T{t}"] = out[("lu", t)]
        d = [rel(out[(a, t)], out[(b, t)]) for a, b in (("dense", "lu"), ("fft", "lu"),
                                                          ("fft", "dense"))]
        print(f"c2 T={t}: route distances dense-lu {d[0]:.2e} fft-lu {d[1]:.2e} "
              f"fft-dense {d[2]:.2e}", flush=True)
        res[f"floor_T{t}"] = max(d)
        res[f"routes_T{t}"] = np.array(d)
    np.savez(os.path.join(HERE, "c2_serial_fine.npz"), **res)


def make_c3():
    """Three routes of the slice: PCG with dense transforms, with FFT
    transforms, and with dense transforms and another preconditioner shift
    (other CG iterates); the floor is the largest pairwise distance."""
    p = workloads.nonlinear_2d_256()
    u0 = workloads.nonlinear_2d_256_u0(0)
    routes = {"dense": dict(transform="dense"), "fft": dict(transform="fft"),
              "dense_shift1": dict(transform="dense", s_pc=1.0)}
    res = {}
    for name, kw in routes.items():
        u = u0.copy()
        t0 = time.time()
        for j in range(p.j_fine):
            u = schemes.step_newton_pcg(u, p.dt, p.eps, p.nl_variant, p.newton_tol, p.newton_max,
                                        **kw)
            if j % 500 == 0:
                print(f"c3 {name}: step {j} ({time.time() - t0:.0f} s)", flush=True)
        res[name] = u
    pairs = (("fft", "dense"), ("dense_shift1", "dense"), ("dense_shift1", "fft"))
    d = [rel(res[a], res[b]) for a, b in pairs]
    print("c3 route distances " + " ".join(f"{a}-{b} {x:.2e}" for (a, b), x in zip(pairs, d)))
    np.savez(os.path.join(HERE, "c3_slice0_fine.npz"), F=res["dense"], floor=max(d),
             routes=np.array(d))


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3"]
    if "c2" in which:
        make_c2()
    if "c3" in which:
        make_c3()
