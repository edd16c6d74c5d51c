"""Neumann-Neumann domain decomposition solve of the PA-I fine step (2.4) in 1D
(Section 4, the experiments with the Neumann-Neumann method as fine solver
of PA-I).

TEST INFRASTRUCTURE ONLY (see the package docstring): the plain definition the
HIP path is checked against.  Dense local solves, one subdomain at a time.

The step (2.4), (I - tau L diag(u_n^2) + eps^2 tau L^2) u = (I - tau L) u_n, is
written in mixed form with v = -eps^2 L u + c u - u_n, c = u_n^2:

    [ I                -tau L ] [u]   [  u_n ]
    [ eps^2 L - diag(c)    I  ] [v] = [ -u_n ]

(the Neumann-Neumann system of Section 4 with f_u = u_n, f_v = -u_n; the text
prints the reaction coefficient as the square of c = u_n^2, which would make it
u_n^4 and not reproduce (2.4); it is read as c = u_n^2 taken once).

Discretisation of the subdomain problems (the paper states them for the
continuous operator):
  * Omega is cut into N0 equal pieces; with n + 1 mesh intervals divisible by
    N0 the interfaces Gamma_q, q = 1..N0-1, are the nodes p_q = q (n+1)/N0.
  * the global matrix is the sum of edge and node contributions; the local
    matrix A_i of Omega_i holds the contributions of its own edges and of its
    nodes, those of an interface node with weight 1/2 (the node is shared by
    two subdomains).  Summing the A_i gives the global matrix back.
  * Dirichlet step: the global equations at the interior nodes of Omega_i,
    with (u, v) = (g, h) on its interfaces and 0 on the physical boundary.
  * the jump of the Neumann traces at Gamma_q is the residual of the global
    equations at p_q of the assembled state; the Neumann step solves
    A_i [phi; psi] = that residual at the interface nodes of Omega_i (zero
    elsewhere; a physical end keeps its homogeneous Dirichlet value).
  * trace update: (g, h)_q += theta (phi, psi) of both neighbours at p_q.  The
    paper writes this with a minus sign and the difference of the two
    neighbours because its Neumann data are x-derivatives; with both
    subdomains' data taken along the outward normal (which the residual
    form is) the two neighbours' corrections add, and minus the residual is
    the outward-flux jump, so the sign turns into a plus.
  * stop when max_q |g_q^{v+1} - g_q^v| <= tol and max_q |h_q^{v+1} - h_q^v|
    <= tol (the paper's per-interface L2 criterion: an interface of a 1D
    domain is one point); the step's result is the Dirichlet solve with the
    last traces.
  * initial traces: the mixed variables of u_n itself at the interfaces,
    g^0 = u_n(p_q), h^0 = (-eps^2 L u_n + u_n^3 - u_n)(p_q).
"""
from __future__ import annotations

import numpy as np

from .operators import laplacian_1d, mesh_h


class NoConvergence(RuntimeError):
    pass


def interface_nodes(n: int, n_sub: int) -> list[int]:
    """Interface node numbers p_q = q (n+1)/N0 (nodes 0 and n+1 are the
    physical boundary, 1..n the unknowns)."""
    if n_sub < 1 or (n + 1) % n_sub or (n + 1) // n_sub < 2:
        raise ValueError("n + 1 must split into n_sub pieces of at least 2 intervals")
    m = (n + 1) // n_sub
    return [q * m for q in range(1, n_sub)]


def mixed_matrix(c: np.ndarray, tau: float, eps: float) -> np.ndarray:
    """Dense global mixed matrix [I, -tau L; eps^2 L - diag(c), I], unknowns
    ordered (u_1..u_n, v_1..v_n), from the sparse D_h."""
    n = c.shape[0]
    L = laplacian_1d(n).toarray()
    eye = np.eye(n)
    return np.block([[eye, -tau * L], [eps * eps * L - np.diag(c), eye]])


def assemble(c: np.ndarray, tau: float, eps: float, lo: int, hi: int,
             shared: set[int]) -> tuple[list[int], np.ndarray]:
    """Edge/node assembly over the nodes lo..hi (0..n+1 numbering): edges
    (j, j+1) with lo <= j < hi, nodes lo..hi, weight 1/2 for nodes in
    `shared`.  Unknowns are the nodes among 1..n, ordered (u block, v block).
    Returns (unknown nodes, matrix)."""
    n = c.shape[0]
    h = mesh_h(n)
    a, b = tau / (h * h), eps * eps / (h * h)
    nodes = [j for j in range(lo, hi + 1) if 1 <= j <= n]
    pos = {j: k for k, j in enumerate(nodes)}
    K = len(nodes)
    A = np.zeros((2 * K, 2 * K))
    for j in nodes:
        w = 0.5 if j in shared else 1.0
        k = pos[j]
        A[k, k] += w                      # u row: u
        A[K + k, K + k] += w              # v row: v
        A[K + k, k] -= w * c[j - 1]       # v row: -c u
    for j in range(lo, hi):
        for r, o in ((j, j + 1), (j + 1, j)):
            if r not in pos:
                continue
            kr = pos[r]
            # u row: -tau (v_o - v_r)/h^2 ; v row: eps^2 (u_o - u_r)/h^2
            A[kr, K + kr] += a
            A[K + kr, kr] -= b
            if o in pos:
                ko = pos[o]
                A[kr, K + ko] -= a
                A[K + kr, ko] += b
    return nodes, A


def global_matrix(c: np.ndarray, tau: float, eps: float) -> np.ndarray:
    n = c.shape[0]
    return assemble(c, tau, eps, 0, n + 1, set())[1]


def local_neumann_matrix(c: np.ndarray, tau: float, eps: float, i: int,
                         n_sub: int) -> tuple[list[int], np.ndarray]:
    """A_i of subdomain i (0-based) with interface nodes weighted 1/2."""
    n = c.shape[0]
    m = (n + 1) // n_sub
    lo, hi = i * m, (i + 1) * m
    shared = set(interface_nodes(n, n_sub)) & {lo, hi}
    return assemble(c, tau, eps, lo, hi, shared)


def step_approx2_dd(u_n: np.ndarray, tau: float, eps: float, n_sub: int = 8,
                    theta: float = 0.25, tol: float = 1e-10, maxit: int = 100,
                    history: list | None = None, g0=None) -> tuple[np.ndarray, int]:
    """One step of (2.4) by the Neumann-Neumann iteration (Section 4).
    Returns (u_{n+1}, iterations); ``history`` receives (max|dg|, max|dh|)
    per iteration.  g0 = (g, h) overrides the initial traces."""
    u_n = np.asarray(u_n, dtype=np.float64)
    n = u_n.shape[0]
    m = (n + 1) // n_sub
    P = interface_nodes(n, n_sub)
    c = u_n * u_n
    rhs = np.concatenate([u_n, -u_n])
    A = global_matrix(c, tau, eps)
    L = laplacian_1d(n)
    if g0 is None:
        mu = -eps * eps * (L @ u_n) + u_n ** 3 - u_n
        g = np.array([u_n[p - 1] for p in P])
        hh = np.array([mu[p - 1] for p in P])
    else:
        g, hh = (np.array(x, dtype=np.float64, copy=True) for x in g0)

    def dirichlet(g, hh):
        """Assembled state: Dirichlet solves in every subdomain, traces on the
        interfaces."""
        x = np.zeros(2 * n)
        for q, p in enumerate(P):
            x[p - 1], x[n + p - 1] = g[q], hh[q]
        for i in range(n_sub):
            inner = [j for j in range(i * m + 1, (i + 1) * m) if 1 <= j <= n]
            rows = np.array([j - 1 for j in inner] + [n + j - 1 for j in inner])
            known = np.array([p - 1 for p in P] + [n + p - 1 for p in P], dtype=int)
            b = rhs[rows] - (A[np.ix_(rows, known)] @ x[known] if len(P) else 0.0)
            x[rows] = np.linalg.solve(A[np.ix_(rows, rows)], b)
        return x

    it = 0
    while P:
        x = dirichlet(g, hh)
        res = rhs - A @ x
        dg = np.zeros(len(P))
        dh = np.zeros(len(P))
        for i in range(n_sub):
            nodes, Ai = local_neumann_matrix(c, tau, eps, i, n_sub)
            K = len(nodes)
            b = np.zeros(2 * K)
            for k, j in enumerate(nodes):
                if j in P:
                    b[k], b[K + k] = res[j - 1], res[n + j - 1]
            y = np.linalg.solve(Ai, b)
            for k, j in enumerate(nodes):
                if j in P:
                    q = P.index(j)
                    dg[q] += theta * y[k]
                    dh[q] += theta * y[K + k]
        g = g + dg
        hh = hh + dh
        it += 1
        sg, sh = float(np.max(np.abs(dg))), float(np.max(np.abs(dh)))
        if history is not None:
            history.append((sg, sh))
        if sg <= tol and sh <= tol:
            break
        if it >= maxit or not (np.isfinite(sg) and np.isfinite(sh)):
            raise NoConvergence(f"Neumann-Neumann did not reach {tol} in {maxit} iterations")
    x = dirichlet(g, hh)
    return x[:n].copy(), it
