"""1D and 3D reference-element data for continuous Q_k Lagrange elements (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

Sec. 5 of the paper: continuous Lagrange elements that are tensor products of
1D elements of degree k, integrated with the (k+1)^3-point Gauss-Legendre
rule.  The paper does not say where the nodes sit; we take the Gauss-Lobatto-
Legendre points (the end points plus the roots of P_k'), which coincide with
equispaced nodes for k <= 2.  The finite-element space does not depend on this
choice; only nodal values (interpolation, the Jacobi diagonal) do.

Reference cell: [0, 1] per direction.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k: int) -> np.ndarray:
    """k+1 Gauss-Lobatto-Legendre points on [0, 1], ascending."""
    if k < 1:
        raise ValueError("degree k >= 1")
    if k == 1:
        return np.array([0.0, 1.0])
    # interior points: roots of P_k' on [-1, 1]
    dcoef = npleg.legder([0] * k + [1])
    inner = np.sort(np.real(npleg.legroots(dcoef)))
    # one Newton polish step per root on P_k' using P_k'' (library evaluation)
    d2 = npleg.legder(dcoef)
    for _ in range(3):
        inner = inner - npleg.legval(inner, dcoef) / npleg.legval(inner, d2)
    s = np.concatenate([[-1.0], inner, [1.0]])
    x = 0.5 * (s + 1.0)
    # exact symmetry about 1/2
    x = 0.5 * (x + (1.0 - x[::-1]))
    return x


def gauss_rule(nq: int):
    """nq-point Gauss-Legendre rule on [0, 1] (points ascending, weights)."""
    s, w = npleg.leggauss(nq)
    return 0.5 * (s + 1.0), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """V[q, a] = l_a(x_q), the Lagrange polynomial of node a evaluated at x_q."""
    x = np.asarray(x, dtype=float)
    V = np.ones((x.size, nodes.size))
    for a in range(nodes.size):
        for m in range(nodes.size):
            if m != a:
                V[:, a] *= (x - nodes[m]) / (nodes[a] - nodes[m])
    return V


def lagrange_derivs(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[q, a] = l_a'(x_q), by the product rule on the product form."""
    x = np.asarray(x, dtype=float)
    n = nodes.size
    D = np.zeros((x.size, n))
    for a in range(n):
        for skip in range(n):
            if skip == a:
                continue
            term = np.full(x.size, 1.0 / (nodes[a] - nodes[skip]))
            for m in range(n):
                if m != a and m != skip:
                    term = term * (x - nodes[m]) / (nodes[a] - nodes[m])
            D[:, a] += term
    return D


class Element1D:
    """Degree-k Lagrange element on [0,1] with Gauss-Lobatto nodes.

    mass[a, b]  = int_0^1 l_a l_b dx        (Gauss, k+1 points: exact)
    stiff[a, b] = int_0^1 l_a' l_b' dx
    On a cell of length h the 1D matrices are h*mass and stiff/h.
    """

    def __init__(self, k: int):
        self.k = k
        self.nodes = gll_nodes(k)
        self.qx, self.qw = gauss_rule(k + 1)
        self.B = lagrange_values(self.nodes, self.qx)   # (nq, k+1)
        self.D = lagrange_derivs(self.nodes, self.qx)   # (nq, k+1)
        W = np.diag(self.qw)
        self.mass = self.B.T @ W @ self.B
        self.stiff = self.D.T @ W @ self.D

    def prolongation(self) -> np.ndarray:
        """P[f, c] = l_c(x_f): a coarse cell [0,1] split into two fine cells
        [0,1/2] and [1/2,1]; the 2k+1 fine nodes are the fine cells' nodes.
        Interpolation of the coarse basis is exact (nested spaces)."""
        xf = np.concatenate([0.5 * self.nodes, 0.5 + 0.5 * self.nodes[1:]])
        return lagrange_values(self.nodes, xf)


def element_matrices_3d(k: int, h: float):
    """3D element mass and stiffness matrices on a cube of side h, computed
    directly from the definition: sum over the (k+1)^3 Gauss points of
    w_q |J| phi_i phi_j and w_q |J| grad phi_i . grad phi_j, where the 3D
    basis function with local index i = a + (k+1)(b + (k+1)c) is
    l_a(x) l_b(y) l_c(z) (x fastest).  No tensor-product factorisation is used.
    """
    el = Element1D(k)
    n1 = k + 1
    nq = n1
    qx, qw = el.qx, el.qw
    B, D = el.B, el.D
    # 3D quadrature points, index q = qa + nq (qb + nq qc)
    w3 = np.einsum("a,b,c->cba", qw, qw, qw).reshape(-1) * h ** 3
    # basis values / reference gradients at points: shape (nq^3, n1^3)
    val = np.einsum("xa,yb,zc->zyxcba", B, B, B).reshape(nq ** 3, n1 ** 3)
    gx = np.einsum("xa,yb,zc->zyxcba", D, B, B).reshape(nq ** 3, n1 ** 3) / h
    gy = np.einsum("xa,yb,zc->zyxcba", B, D, B).reshape(nq ** 3, n1 ** 3) / h
    gz = np.einsum("xa,yb,zc->zyxcba", B, B, D).reshape(nq ** 3, n1 ** 3) / h
    Me = val.T @ (w3[:, None] * val)
    Ke = gx.T @ (w3[:, None] * gx) + gy.T @ (w3[:, None] * gy) + gz.T @ (w3[:, None] * gz)
    return Me, Ke
