"""Chebyshev-Jacobi smoothing, geometric multigrid and the stage-block
preconditioner (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

Sec. 2, eq. (irk:P): A_Q^-1 = L U (U unit upper triangular), L = S Lam S^-1,
and

    P^-1 = (S (x) I)(Lam (x) M + tau I (x) K)^-1 (S^-1 (x) I),

so P^-1 costs two Q x Q basis changes and Q independent real blocks
lam_i M + tau K.  Sec. 5: each block is approximated by one V-cycle of
geometric multigrid whose smoother is a Chebyshev iteration around point
Jacobi; the batched runs (Sec. 5, batched execution) use the same Chebyshev
iteration as coarse solver and one eigenvalue bound (the largest over all
blocks) for every block.

Readings where the paper is silent (all stated in the design notes):
* levels: n, n/2, ... while n is even; the coarsest mesh has an odd number of
  cells per direction (1 for n = 2^L); the same degree k on every level;
  level matrices are re-assembled on each mesh; restriction is P^T.
* V(nu, nu): pre-smoothing is a degree-nu Chebyshev polynomial started from
  zero, post-smoothing the same started from the prolongated iterate; the
  coarsest level runs the same Chebyshev iteration from zero.
* Chebyshev interval [upper / range, upper] for D^-1 A with D = diag(A).
* The Chebyshev iteration is Saad, "Iterative Methods for Sparse Linear
  Systems", Algorithm 12.1 (Chebyshev acceleration), with the residual
  preconditioned by D^-1.  "Degree nu" means nu updates of the iterate, i.e.
  an error propagator that is a polynomial of degree nu in D^-1 A.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import Problem, Mesh, prolongation_3d


def level_sizes(n: int):
    """Cells per direction from fine to coarse."""
    out = [n]
    while out[-1] % 2 == 0:
        out.append(out[-1] // 2)
    return out


class Hierarchy:
    """Assembled level operators (interior) and interior prolongations."""

    def __init__(self, n: int, k: int, method: str = "auto"):
        self.k = k
        self.sizes = level_sizes(n)
        self.levels = [Problem(m, k, method) for m in self.sizes]   # fine -> coarse
        self.P = []   # P[l]: from level l+1 (coarser) to level l, interior
        for l in range(len(self.sizes) - 1):
            fine, coarse = self.levels[l], self.levels[l + 1]
            Pf = prolongation_3d(coarse.mesh)
            self.P.append(Pf[fine.idx][:, coarse.idx].tocsr())

    @property
    def nlevels(self):
        return len(self.levels)


def chebyshev(A, Dinv, b, x0, degree, upper, lower):
    """Saad Alg. 12.1 with Jacobi preconditioning: returns x after `degree`
    updates.  If x0 is None the start is zero and r_0 = b costs no product."""
    theta = 0.5 * (upper + lower)
    delta = 0.5 * (upper - lower)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - A @ x
    d = (Dinv * r) / theta
    for it in range(degree):
        x = x + d
        if it == degree - 1:
            break
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (Dinv * r)
        rho = rho_new
    return x


class BlockMG:
    """V-cycles for the blocks lam_i M + tau K on every level."""

    def __init__(self, hier: Hierarchy, lam, tau, degree=3, coarse_degree=None,
                 cheb_range=15.0, eig_max=None):
        self.h = hier
        self.lam = np.asarray(lam, dtype=float)
        self.tau = tau
        self.degree = degree
        self.coarse_degree = degree if coarse_degree is None else coarse_degree
        self.range = cheb_range
        self.A = []      # A[l][i]
        self.Dinv = []
        for lev in hier.levels:
            Al, Dl = [], []
            for li in self.lam:
                Ai = (li * lev.M + tau * lev.K).tocsr()
                Al.append(Ai)
                Dl.append(1.0 / Ai.diagonal())
            self.A.append(Al)
            self.Dinv.append(Dl)
        if eig_max is None:
            eig_max = [1.2 * self.max_eig_exact(l) for l in range(hier.nlevels)]
        self.eig_max = np.asarray(eig_max, dtype=float)

    def max_eig_exact(self, l):
        """Largest eigenvalue of D_i^-1 A_i over all blocks i (scipy eigsh on
        the symmetric pencil (A_i, D_i))."""
        best = 0.0
        for Ai, Di in zip(self.A[l], self.Dinv[l]):
            n = Ai.shape[0]
            if n == 0:          # no interior unknowns on this level
                return 1.0
            if n <= 400:
                ev = np.linalg.eigvalsh((Ai.toarray() * np.sqrt(Di)[:, None]) * np.sqrt(Di)[None, :])
                best = max(best, ev[-1])
            else:
                Ds = sp.diags(np.sqrt(Di))
                ev = spla.eigsh(Ds @ Ai @ Ds, k=1, which="LA", return_eigenvectors=False, tol=1e-10)
                best = max(best, ev[0])
        return best

    def vcycle_block(self, i, b, l=0):
        """One V-cycle for block i starting on level l (interior vectors)."""
        A, Dinv = self.A[l][i], self.Dinv[l][i]
        up = self.eig_max[l]
        lo = up / self.range
        if l == self.h.nlevels - 1:
            if b.size == 0:
                return b.copy()
            return chebyshev(A, Dinv, b, None, self.coarse_degree, up, lo)
        x = chebyshev(A, Dinv, b, None, self.degree, up, lo)
        r = b - A @ x
        P = self.h.P[l]
        xc = self.vcycle_block(i, P.T @ r, l + 1)
        x = x + P @ xc
        return chebyshev(A, Dinv, b, x, self.degree, up, lo)

    def vcycle(self, b):
        """All blocks: b has shape (Q, nint)."""
        return np.stack([self.vcycle_block(i, b[i]) for i in range(b.shape[0])])


class BlockPreconditioner:
    """P^-1 r = (S (x) I) blockdiag(V-cycle_i) (S^-1 (x) I) r, eq. (irk:P)."""

    def __init__(self, tab, mg: BlockMG):
        self.tab = tab
        self.mg = mg

    def apply(self, r):
        Q = self.tab.Q
        w = self.tab.Sinv @ r.reshape(Q, -1)
        x = self.mg.vcycle(w)
        return (self.tab.S @ x).reshape(r.shape)
