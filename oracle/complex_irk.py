"""Direct (complex) diagonalisation of A_Q^-1 and the PRESB preconditioner
(oracle).

Test infrastructure only: see ``oracle/__init__.py``.

Sec. 2, eq. (irk:Ainv): A_Q^-1 = S Lam S^-1 with complex S, Lam; for Radau
IIA Lam holds floor(Q/2) complex-conjugate pairs and, for odd Q, one real
eigenvalue.  The stage system of eq. (irk:A) then splits into the blocks
lam_i M + tau K, solved independently; a conjugate pair needs only one of its
two members, because the stage vectors are real.

Real form used here (the paper leaves the bookkeeping open, Sec. 6 names the
two-by-two real blocks).  For a pair with lam = a + i b (b > 0), eigenvector
s (A^-1 s = lam s) and the matching row t of S^-1:
  * the block unknown u = t . k is complex; its real and imaginary parts are
    two real "slots", Re(t) . k and Im(t) . k;
  * k receives 2 Re(s u) = (2 Re s) Re u + (-2 Im s) Im u from the pair.
Collecting the slots gives real Q x Q matrices T (slots = T k) and U = T^-1
(k = U slots), and T A^-1 U = Lam_r, block diagonal with [[a, -b], [b, a]]
per pair (complex multiplication by lam) and the real eigenvalue as a 1 x 1
block.  So

    A^-1 (x) M + tau I (x) K = (U (x) I)(Lam_r (x) M + tau I (x) K)(T (x) I),

and a pair block is the two-by-two real system of Sec. 6,
[[K', -M'], [M', K']] with K' = a M + tau K and M' = b M.  (The paper prints
K instead of K' in the lower right corner; with K' the system is the real
form of (K' + i M') u = v written one line above, which is the reading taken.)

Slot order: n_b = ceil(Q/2) blocks; pairs sorted by ascending Re(lam), then
the real block (odd Q).  Slots 0 .. n_b-1 hold the real parts (and the real
block), slots n_b .. Q-1 the imaginary parts of the pairs, so pair j owns
slots j and n_b + j.

PRESB (Sec. 6, eq. presb:p): P = [[K', -M'], [M', K' + 2M']] factors as
[[I, -I], [0, I]] [[H, 0], [M', H]] [[I, I], [0, I]] with H = K' + M' =
(a + b) M + tau K, hence P^-1 (r1, r2) is
    g1 = H^-1 (r1 + r2),  g2 = H^-1 (r2 - M' g1),  u = (g1 - g2, g2),
two solves with H in sequence.  Each H^-1 is one V-cycle of the block
multigrid (Sec. 6: a single V-cycle); the real block takes one V-cycle on
lam M + tau K.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np
import scipy.sparse as sp

from .fgmres import fgmres
from .multigrid import BlockMG, Hierarchy
from .step import premultiplied_rhs
from .tableau import DPS, RadauIIA


class ComplexBlocks:
    """Eigen-decomposition of A_Q^-1 in the real slot form described above."""

    def __init__(self, tab: RadauIIA):
        Q = tab.Q
        self.Q = Q
        with mp.workdps(DPS):
            E, ER = mp.eig(tab._mp["Ainv"])
            tol = mp.mpf(10) ** (-DPS // 2)
            pairs, reals = [], []
            for i, e in enumerate(E):
                if abs(mp.im(e)) <= tol:
                    reals.append(i)
                elif mp.im(e) > 0:
                    pairs.append(i)
            if len(reals) != Q % 2 or 2 * len(pairs) + len(reals) != Q:
                raise ValueError("unexpected spectrum of A^-1")
            pairs.sort(key=lambda i: mp.re(E[i]))
            npair = len(pairs)
            nb = npair + len(reals)
            U = mp.matrix(Q, Q)
            for j, i in enumerate(pairs):
                for r in range(Q):
                    U[r, j] = 2 * mp.re(ER[r, i])
                    U[r, nb + j] = -2 * mp.im(ER[r, i])
            for i in reals:
                for r in range(Q):
                    U[r, npair] = mp.re(ER[r, i])
            T = U ** -1
            self.npair, self.nb = npair, nb
            self.lam = np.array([complex(E[i]) for i in pairs] + [complex(mp.re(E[i])) for i in reals])
            self.U = np.array([[float(U[i, j]) for j in range(Q)] for i in range(Q)])
            self.T = np.array([[float(T[i, j]) for j in range(Q)] for i in range(Q)])
            self._mp = dict(U=U, T=T, E=[E[i] for i in pairs + reals])
        LR = np.zeros((Q, Q))
        for j in range(npair):
            a, b = self.lam[j].real, self.lam[j].imag
            LR[j, j] = a
            LR[j, nb + j] = -b
            LR[nb + j, j] = b
            LR[nb + j, nb + j] = a
        if len(reals):
            LR[npair, npair] = self.lam[npair].real
        self.LamR = LR

    def block_slots(self, j):
        """Slots of block j: (re, im) for a pair, (re,) for the real block."""
        return (j, self.nb + j) if j < self.npair else (j,)

    def h_shift(self):
        """Per slot, the mass coefficient of the PRESB inner matrix H:
        a + b for both slots of a pair, lam for the real block."""
        out = np.zeros(self.Q)
        for j in range(self.nb):
            lam = self.lam[j]
            for s in self.block_slots(j):
                out[s] = lam.real + lam.imag if j < self.npair else lam.real
        return out


def block_operator(dec: ComplexBlocks, M, K, tau, u):
    """(Lam_r (x) M + tau I (x) K) u for slot vectors u of shape (Q, n)."""
    u = np.asarray(u)
    return np.stack([M @ (dec.LamR[s] @ u) + tau * (K @ u[s]) for s in range(dec.Q)])


class Presb:
    """P^-1 for every block (eq. presb:p), inner solves by `inner(slot, b)`."""

    def __init__(self, dec: ComplexBlocks, M, inner):
        self.dec, self.M, self.inner = dec, M, inner

    def apply_block(self, j, r):
        """r: (len(slots), n) for block j; returns the same shape."""
        dec = self.dec
        if j >= dec.npair:
            return self.inner(j, r[0])[None]
        s_re, s_im = dec.block_slots(j)
        b = dec.lam[j].imag
        g1 = self.inner(s_re, r[0] + r[1])
        g2 = self.inner(s_im, r[1] - b * (self.M @ g1))
        return np.stack([g1 - g2, g2])

    def apply(self, r):
        """All blocks on a (Q, n) slot vector."""
        out = np.zeros_like(r)
        for j in range(self.dec.nb):
            sl = list(self.dec.block_slots(j))
            out[sl] = self.apply_block(j, r[sl])
        return out


def presb_matrix(dec: ComplexBlocks, M, K, tau, j):
    """The PRESB matrix of pair j assembled, [[K', -M'], [M', K' + 2M']]."""
    lam = dec.lam[j]
    Kp = lam.real * M + tau * K
    Mp = lam.imag * M
    return sp.bmat([[Kp, -Mp], [Mp, Kp + 2 * Mp]]).tocsr()


def pair_matrix(dec: ComplexBlocks, M, K, tau, j):
    """The two-by-two real block of pair j, [[K', -M'], [M', K']]."""
    lam = dec.lam[j]
    Kp = lam.real * M + tau * K
    Mp = lam.imag * M
    return sp.bmat([[Kp, -Mp], [Mp, Kp]]).tocsr()


class ComplexStepper:
    """Radau IIA steps by direct diagonalisation (eq. irk:Ainv): slot basis
    change T, one right-preconditioned GMRES per block with PRESB, and
    k = U u.  Operators assembled on interior unknowns."""

    def __init__(self, n, k, tab, tau, degree=3, coarse_degree=None, cheb_range=15.0,
                 eig_max=None, method="auto"):
        self.tab, self.tau = tab, tau
        self.dec = ComplexBlocks(tab)
        self.hier = Hierarchy(n, k, method)
        fine = self.hier.levels[0]
        self.M, self.K = fine.M, fine.K
        self.mg = BlockMG(self.hier, self.dec.h_shift(), tau, degree, coarse_degree, cheb_range, eig_max)
        self.presb = Presb(self.dec, self.M, lambda s, b: self.mg.vcycle_block(s, b))

    def step(self, y, gbar=None, rtol=1e-12, restart=50, max_iter=500):
        """Returns (y_next, iterations per block)."""
        Q, dec = self.tab.Q, self.dec
        if gbar is None:
            gbar = np.zeros((Q, y.size))
        rhs = premultiplied_rhs(self.K, self.tab.Ainv, y, gbar)
        w = dec.T @ rhs
        u = np.zeros_like(w)
        its = []
        for j in range(dec.nb):
            sl = list(dec.block_slots(j))
            ns, n = len(sl), y.size

            def apply_A(v, sl=sl, ns=ns):
                full = np.zeros_like(w)
                full[sl] = v.reshape(ns, n)
                return block_operator(dec, self.M, self.K, self.tau, full)[sl].reshape(-1)

            def apply_P(v, j=j, ns=ns):
                return self.presb.apply_block(j, v.reshape(ns, n)).reshape(-1)

            x, it, _ = fgmres(apply_A, apply_P, w[sl].reshape(-1), rtol, restart, max_iter)
            u[sl] = x.reshape(ns, n)
            its.append(it)
        k = dec.U @ u
        return y + self.tau * (self.tab.b @ k), its
