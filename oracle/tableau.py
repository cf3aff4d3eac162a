"""Radau IIA Butcher tableau and the block-preconditioner factors (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

Everything here is computed in 50-digit mpmath arithmetic and rounded to
float64 at the end.

* Radau IIA with Q stages is the collocation method whose nodes are the right
  Radau points on [0, 1] (c_Q = 1); it has order 2Q-1 (Sec. 2).  The nodes are
  the roots of P_Q(2x-1) - P_{Q-1}(2x-1) with P_m the Legendre polynomials,
  a_ij is the integral of the j-th Lagrange polynomial on the nodes over
  [0, c_i] and b_j its integral over [0, 1] (textbook collocation definition).
* The preconditioner of eq. (irk:P) uses the LU factorisation of A_Q^-1 with a
  unit-diagonal U (Crout form, no pivoting), and the eigen-decomposition of the
  lower-triangular factor, L = S Lambda S^-1, which is real (Sec. 2).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np

DPS = 50


def _legendre_coeffs(m: int):
    """Monomial coefficients (ascending) of the Legendre polynomial P_m(s),
    from the three-term recurrence (m+1) P_{m+1} = (2m+1) s P_m - m P_{m-1}."""
    p_prev = [mp.mpf(1)]
    if m == 0:
        return p_prev
    p = [mp.mpf(0), mp.mpf(1)]
    for j in range(1, m):
        nxt = [mp.mpf(0)] * (j + 2)
        for i, c in enumerate(p):
            nxt[i + 1] += mp.mpf(2 * j + 1) * c
        for i, c in enumerate(p_prev):
            nxt[i] -= mp.mpf(j) * c
        nxt = [c / (j + 1) for c in nxt]
        p_prev, p = p, nxt
    return p


def _compose_2x_minus_1(coeffs):
    """Coefficients in x of p(2x - 1) given ascending coefficients of p(s)."""
    out = [mp.mpf(0)] * len(coeffs)
    for i, c in enumerate(coeffs):
        # (2x - 1)^i = sum_r binom(i, r) (2x)^r (-1)^(i-r)
        for r in range(i + 1):
            out[r] += c * mp.binomial(i, r) * mp.mpf(2) ** r * (-1) ** (i - r)
    return out


def radau_nodes_mp(Q: int):
    """Right Radau points on [0,1]: roots of P_Q(2x-1) - P_{Q-1}(2x-1)."""
    with mp.workdps(DPS):
        pq = _compose_2x_minus_1(_legendre_coeffs(Q))
        pq1 = _compose_2x_minus_1(_legendre_coeffs(Q - 1))
        poly = [a - (pq1[i] if i < len(pq1) else 0) for i, a in enumerate(pq)]
        # mpmath.polyroots wants descending coefficients
        roots = mp.polyroots(poly[::-1], maxsteps=400, extraprec=400)
        roots = sorted(mp.re(r) for r in roots)
        return roots


def _lagrange_integral(c, j, upper):
    """Integral over [0, upper] of the j-th Lagrange polynomial on nodes c."""
    # build the polynomial prod_{m != j} (x - c_m)/(c_j - c_m) in monomials
    poly = [mp.mpf(1)]
    denom = mp.mpf(1)
    for m, cm in enumerate(c):
        if m == j:
            continue
        new = [mp.mpf(0)] * (len(poly) + 1)
        for i, a in enumerate(poly):
            new[i + 1] += a
            new[i] -= a * cm
        poly = new
        denom *= c[j] - cm
    return sum(a * upper ** (i + 1) / (i + 1) for i, a in enumerate(poly)) / denom


def radau_tableau_mp(Q: int):
    """(A, b, c) of Radau IIA with Q stages as mpmath matrices/lists."""
    if Q < 1:
        raise ValueError("Q >= 1")
    with mp.workdps(DPS):
        c = radau_nodes_mp(Q)
        A = mp.matrix(Q, Q)
        for i in range(Q):
            for j in range(Q):
                A[i, j] = _lagrange_integral(c, j, c[i])
        b = [_lagrange_integral(c, j, mp.mpf(1)) for j in range(Q)]
        return A, b, c


def crout_mp(Ainv):
    """Crout factorisation Ainv = L U with U unit upper triangular, no pivoting.

    Column j of L and row j of U follow from matching entries (i >= j) and
    (i < j) of L U against Ainv in the usual Crout order.
    """
    Q = Ainv.rows
    L = mp.matrix(Q, Q)
    U = mp.eye(Q)
    for j in range(Q):
        for i in range(j, Q):
            L[i, j] = Ainv[i, j] - sum(L[i, m] * U[m, j] for m in range(j))
        if L[j, j] == 0:
            raise ZeroDivisionError("Crout factorisation breaks down (zero pivot)")
        for i in range(j + 1, Q):
            U[j, i] = (Ainv[j, i] - sum(L[j, m] * U[m, i] for m in range(j))) / L[j, j]
    return L, U


def lower_eig_mp(L):
    """Eigen-decomposition of a lower-triangular L with distinct diagonal.

    The eigenvalues are diag(L).  Eigenvector i has s_i(m) = 0 for m < i,
    s_i(i) = 1, and the remaining entries follow from forward substitution in
    (L - lambda_i I) s_i = 0.  Returns (S, lam) with L = S diag(lam) S^-1.
    """
    Q = L.rows
    lam = [L[i, i] for i in range(Q)]
    S = mp.matrix(Q, Q)
    for i in range(Q):
        S[i, i] = mp.mpf(1)
        for m in range(i + 1, Q):
            acc = sum(L[m, r] * S[r, i] for r in range(i, m))
            denom = lam[i] - L[m, m]
            if denom == 0:
                raise ZeroDivisionError("repeated eigenvalue in L")
            S[m, i] = acc / denom
    return S, lam


def _to_np(M):
    return np.array([[float(M[i, j]) for j in range(M.cols)] for i in range(M.rows)])


class RadauIIA:
    """All Q x Q data the method needs, rounded to float64."""

    def __init__(self, Q: int):
        with mp.workdps(DPS):
            A, b, c = radau_tableau_mp(Q)
            Ainv = A ** -1
            L, U = crout_mp(Ainv)
            S, lam = lower_eig_mp(L)
            Sinv = S ** -1
            self.Q = Q
            self.A = _to_np(A)
            self.b = np.array([float(x) for x in b])
            self.c = np.array([float(x) for x in c])
            self.Ainv = _to_np(Ainv)
            self.L = _to_np(L)
            self.U = _to_np(U)
            self.S = _to_np(S)
            self.Sinv = _to_np(Sinv)
            self.lam = np.array([float(x) for x in lam])
            # keep the high-precision objects for pins
            self._mp = dict(A=A, b=b, c=c, Ainv=Ainv, L=L, U=U, S=S, Sinv=Sinv, lam=lam)

    def stability(self, z):
        """R(z) = 1 + z b^T (I - z A)^-1 e, evaluated in float64/complex."""
        z = np.asarray(z, dtype=complex)
        out = np.empty(z.shape, dtype=complex)
        e = np.ones(self.Q)
        I = np.eye(self.Q)
        for idx, zz in np.ndenumerate(z):
            out[idx] = 1.0 + zz * self.b @ np.linalg.solve(I - zz * self.A, e)
        return out


def pade_exp(num_deg: int, den_deg: int, z):
    """The (num_deg, den_deg) Pade approximant of exp(z), closed form.

    P(z) = sum_n (k+j-n)! k! / ((k+j)! n! (k-n)!) z^n,
    D(z) = sum_n (k+j-n)! j! / ((k+j)! n! (j-n)!) (-z)^n, k = num_deg, j = den_deg.
    """
    k, j = num_deg, den_deg
    f = math.factorial
    P = sum(f(k + j - n) * f(k) / (f(k + j) * f(n) * f(k - n)) * z ** n for n in range(k + 1))
    D = sum(f(k + j - n) * f(j) / (f(k + j) * f(n) * f(j - n)) * (-z) ** n for n in range(j + 1))
    return P / D
