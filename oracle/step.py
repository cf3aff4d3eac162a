"""The Radau IIA step for M y' + K y = g(t) (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

Sec. 2: with y_n the current solution, the stage derivatives k_1..k_Q solve

    (I_Q (x) M + tau A_Q (x) K) k = gbar - (I_Q (x) K)(e_Q (x) y_n),
    gbar_i = g(t_n + c_i tau),

and y_{n+1} = y_n + tau sum_i b_i k_i (Sec. 1).  The paper prints "+K u_0"
on the right-hand side; substituting y_n + tau sum_j a_ij k_j into
M k_i = g_i - K y shows that the term enters with a minus sign for the
equation M y' + K y = g stated in the same section, and that is the reading
used here (it makes Q = 1 reduce to backward Euler, which the tests pin).

Three solvers of the same definition:
* ``radau_step_direct``: sparse LU of the coupled Q N x Q N system.
* ``backward_euler``: (M + tau K) y_{n+1} = M y_n + tau g(t_{n+1}).
* ``ModalSolver``: the exact step through the generalised eigen-decomposition
  K v = lambda M v, which on the uniform mesh separates into 1D problems
  because M and K are Kronecker sums; per eigenmode the stage system is a
  Q x Q system (I + tau lambda A) khat = ghat - lambda yhat e.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import Mesh, global_1d


def stage_matrix(M, K, A, tau):
    """I_Q (x) M + tau A_Q (x) K."""
    Q = A.shape[0]
    return (sp.kron(sp.identity(Q), M) + tau * sp.kron(sp.csr_matrix(A), K)).tocsc()


def stage_rhs(K, y, gbar):
    """gbar - (I (x) K)(e (x) y); gbar has shape (Q, n)."""
    Ky = K @ y
    return np.asarray(gbar) - Ky[None, :]


def premultiplied_operator(M, K, Ainv, tau):
    """The operator of eq. (irk:A): A_Q^-1 (x) M + tau I_Q (x) K."""
    Q = Ainv.shape[0]
    return (sp.kron(sp.csr_matrix(Ainv), M) + tau * sp.kron(sp.identity(Q), K)).tocsr()


def premultiplied_rhs(K, Ainv, y, gbar):
    """Right-hand side of eq. (irk:A): (A^-1 (x) I)(gbar - e (x) K y)."""
    return Ainv @ stage_rhs(K, y, gbar)


class DirectStepper:
    """Radau IIA steps by a direct sparse solve of the coupled Q N x Q N
    stage system (factorised once for fixed tau)."""

    def __init__(self, M, K, tab, tau):
        self.M, self.K, self.tab, self.tau = M, K, tab, tau
        self.lu = spla.splu(stage_matrix(M, K, tab.A, tau))

    def step(self, y, gbar=None):
        """Returns (y_next, k)."""
        Q, n = self.tab.Q, y.shape[0]
        if gbar is None:
            gbar = np.zeros((Q, n))
        rhs = stage_rhs(self.K, y, gbar).reshape(-1)
        k = self.lu.solve(rhs).reshape(Q, n)
        return y + self.tau * (self.tab.b @ k), k


def radau_step_direct(M, K, tab, tau, y, gbar=None):
    """One Radau IIA step by a direct sparse solve.  Returns (y_next, k)."""
    return DirectStepper(M, K, tab, tau).step(y, gbar)


def backward_euler(M, K, tau, y, g_next=None):
    rhs = M @ y
    if g_next is not None:
        rhs = rhs + tau * g_next
    return spla.splu((M + tau * K).tocsc()).solve(rhs)


class ModalSolver:
    """Exact Radau IIA steps on the uniform mesh by fast diagonalisation.

    1D: interior m, a (N-2 square); eigh(a, m) gives V with V^T m V = I and
    V^T a V = diag(mu).  3D: W = V (x) V (x) V diagonalises the pencil,
    W^T M W = I, W^T K W = diag(mu_z + mu_y + mu_x).  Coordinates of a vector y
    are yhat = W^T M y, and y = W yhat.
    """

    def __init__(self, n: int, k: int):
        self.mesh = Mesh(n, k)
        m, a = global_1d(self.mesh)
        m = m.toarray()[1:-1, 1:-1]
        a = a.toarray()[1:-1, 1:-1]
        self.m1, self.a1 = m, a
        mu, V = sla.eigh(a, m)
        self.mu, self.V = mu, V
        ni = m.shape[0]
        self.ni = ni
        self.lam = (mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).reshape(-1)

    # --- tensor helpers on (z, y, x) arrays of the interior grid -----------
    def _apply_each_axis(self, T, x):
        x = x.reshape(self.ni, self.ni, self.ni)
        x = np.einsum("ia,zya->zyi", T, x, optimize=True)
        x = np.einsum("ia,zax->zix", T, x, optimize=True)
        x = np.einsum("ia,ayx->iyx", T, x, optimize=True)
        return x.reshape(-1)

    def to_modal(self, y_int):
        """yhat = W^T M y."""
        My = self._apply_each_axis(self.m1, y_int)
        return self._apply_each_axis(self.V.T, My)

    def from_modal(self, yhat):
        return self._apply_each_axis(self.V, yhat)

    def load_to_modal(self, g_int):
        """ghat = W^T g (g is a load vector, already integrated)."""
        return self._apply_each_axis(self.V.T, g_int)

    def step(self, tab, tau, y_int, gbar_int=None, chunk=1 << 20):
        """One exact step; gbar_int has shape (Q, nint) or None."""
        Q = tab.Q
        yhat = self.to_modal(y_int)
        if gbar_int is not None:
            ghat = np.stack([self.load_to_modal(g) for g in gbar_int])
        ynew = yhat.copy()
        I = np.eye(Q)
        e = np.ones(Q)
        for s in range(0, yhat.size, chunk):
            lam = self.lam[s:s + chunk]
            mats = I[None] + tau * lam[:, None, None] * tab.A[None]
            rhs = -(lam * yhat[s:s + chunk])[:, None] * e[None, :]
            if gbar_int is not None:
                rhs = rhs + ghat[:, s:s + chunk].T
            khat = np.linalg.solve(mats, rhs[..., None])[..., 0]
            ynew[s:s + chunk] += tau * khat @ tab.b
        return self.from_modal(ynew)
