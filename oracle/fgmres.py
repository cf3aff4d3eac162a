"""Flexible GMRES and the full iterative Radau IIA step (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

Sec. 2 / Sec. 5: GMRES on the premultiplied stage operator of eq. (irk:A),
A_Q^-1 (x) M + tau I (x) K, preconditioned by eq. (irk:P) and run until the
l2 norm of the residual has dropped by the requested factor.  Because the
preconditioner (a multigrid V-cycle) is applied on the right we use the
flexible variant, Saad, "Iterative Methods for Sparse Linear Systems",
Algorithm 9.6 (FGMRES), with the modified Gram-Schmidt Arnoldi loop written
there, Givens rotations for the least-squares problem, a zero initial guess
and restarts of length m.  Convergence: ||b - A x||_2 <= rtol ||b||_2.
"""
from __future__ import annotations

import numpy as np

from .multigrid import BlockMG, BlockPreconditioner, Hierarchy
from .step import premultiplied_operator, premultiplied_rhs


def fgmres(apply_A, apply_P, b, rtol=1e-10, restart=50, max_iter=500):
    """Returns (x, iterations, true relative residual)."""
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    its = 0
    r = b.copy()
    while True:
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm or its >= max_iter:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = apply_P(V[j])
            w = apply_A(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            # apply the previous rotations to the new column
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            if abs(g[j + 1]) <= rtol * bnorm or its >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
        r = b - apply_A(x)
    return x, its, np.linalg.norm(r) / bnorm


class IterativeStepper:
    """Radau IIA steps by FGMRES on eq. (irk:A) with the preconditioner of
    eq. (irk:P); all operators assembled (interior unknowns)."""

    def __init__(self, n, k, tab, tau, degree=3, coarse_degree=None, cheb_range=15.0,
                 eig_max=None, method="auto"):
        self.tab, self.tau = tab, tau
        self.hier = Hierarchy(n, k, method)
        fine = self.hier.levels[0]
        self.M, self.K = fine.M, fine.K
        self.op = premultiplied_operator(self.M, self.K, tab.Ainv, tau)
        self.mg = BlockMG(self.hier, tab.lam, tau, degree, coarse_degree, cheb_range, eig_max)
        self.prec = BlockPreconditioner(tab, self.mg)

    def step(self, y, gbar=None, rtol=1e-12, restart=50, max_iter=500):
        Q = self.tab.Q
        if gbar is None:
            gbar = np.zeros((Q, y.size))
        rhs = premultiplied_rhs(self.K, self.tab.Ainv, y, gbar).reshape(-1)
        k, its, rres = fgmres(lambda v: self.op @ v, self.prec.apply, rhs, rtol, restart, max_iter)
        k = k.reshape(Q, -1)
        return y + self.tau * (self.tab.b @ k), its, rres
