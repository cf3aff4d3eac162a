"""Global finite-element matrices on the uniform hexahedral mesh (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

Mesh (Sec. 5): the unit cube split into n^3 equal hexahedra (n = 2^L in the
paper; any n >= 1 here), continuous Q_k elements, N = n k + 1 nodes per
direction.  Global node (ix, iy, iz) has index ix + N (iy + N iz) (x fastest).
Homogeneous Dirichlet conditions: the unknowns are the interior nodes; the
boundary nodes are fixed at zero.

``assemble_cell_loop`` is the definition (a loop over cells adding element
matrices into a sparse matrix).  ``assemble_kron`` builds the same matrices as
Kronecker products of 1D global matrices; the two are pinned against each
other on small meshes and the Kronecker form is then used where the cell loop
would need too much memory.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fe import Element1D, element_matrices_3d, gauss_rule, lagrange_values


class Mesh:
    def __init__(self, n: int, k: int):
        if n < 1 or k < 1:
            raise ValueError("n >= 1, k >= 1")
        self.n, self.k = n, k
        self.N = n * k + 1
        self.h = 1.0 / n
        self.el = Element1D(k)
        # 1D node coordinates on [0, 1]
        x = np.empty(self.N)
        for e in range(n):
            x[e * k:(e + 1) * k + 1] = (e + self.el.nodes) * self.h
        self.x1d = x

    @property
    def ndofs(self) -> int:
        return self.N ** 3

    def interior_mask(self) -> np.ndarray:
        m1 = np.zeros(self.N, dtype=bool)
        m1[1:-1] = True
        return (m1[None, None, :] & m1[None, :, None] & m1[:, None, None]).reshape(-1)

    def interior_index(self) -> np.ndarray:
        return np.flatnonzero(self.interior_mask())

    def cell_dofs(self) -> np.ndarray:
        """(n^3, (k+1)^3) global node indices of every cell, local index
        a + (k+1)(b + (k+1)c), cells ordered x fastest."""
        n, k, N = self.n, self.k, self.N
        loc = np.arange(k + 1)
        c = np.arange(n)
        # global 1D indices per cell and local node
        g1 = c[:, None] * k + loc[None, :]   # (n, k+1)
        gz = g1[:, None, None, :, None, None]
        gy = g1[None, :, None, None, :, None]
        gx = g1[None, None, :, None, None, :]
        g = gx + N * (gy + N * gz)            # (cz, cy, cx, lc, lb, la)
        return g.reshape(n ** 3, (k + 1) ** 3)


def assemble_cell_loop(mesh: Mesh):
    """Full (boundary-inclusive) M and K by adding element matrices cell by
    cell (all cells are translates of each other on this mesh)."""
    Me, Ke = element_matrices_3d(mesh.k, mesh.h)
    dofs = mesh.cell_dofs()
    ncell, nl = dofs.shape
    rows = np.repeat(dofs, nl, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, nl)).reshape(-1)
    mv = np.tile(Me.reshape(-1), ncell)
    kv = np.tile(Ke.reshape(-1), ncell)
    shape = (mesh.ndofs, mesh.ndofs)
    M = sp.coo_matrix((mv, (rows, cols)), shape=shape).tocsr()
    K = sp.coo_matrix((kv, (rows, cols)), shape=shape).tocsr()
    M.sum_duplicates()
    K.sum_duplicates()
    return M, K


def global_1d(mesh: Mesh):
    """1D global mass and stiffness matrices (N x N) on the n-cell partition
    of [0,1], assembled element by element."""
    N, k, h = mesh.N, mesh.k, mesh.h
    m = np.zeros((N, N))
    a = np.zeros((N, N))
    for e in range(mesh.n):
        s = slice(e * k, e * k + k + 1)
        m[s, s] += h * mesh.el.mass
        a[s, s] += mesh.el.stiff / h
    return sp.csr_matrix(m), sp.csr_matrix(a)


def assemble_kron(mesh: Mesh):
    """Full M and K as Kronecker products of the 1D global matrices:
    M = m (x) m (x) m, K = a(x)m(x)m + m(x)a(x)m + m(x)m(x)a (z, y, x order)."""
    m, a = global_1d(mesh)
    mm = sp.kron(m, m, format="csr")
    M = sp.kron(m, mm, format="csr")
    K = (sp.kron(a, mm, format="csr") + sp.kron(m, sp.kron(a, m), format="csr")
         + sp.kron(m, sp.kron(m, a), format="csr"))
    return M.tocsr(), K.tocsr()


def restrict_interior(mesh: Mesh, A):
    idx = mesh.interior_index()
    return A[idx][:, idx].tocsr()


class Problem:
    """Interior (Dirichlet-eliminated) M and K of one mesh."""

    def __init__(self, n: int, k: int, method: str = "auto"):
        self.mesh = Mesh(n, k)
        if method == "auto":
            method = "cell" if self.mesh.ndofs * (k + 1) ** 3 <= 3e7 else "kron"
        M, K = (assemble_cell_loop if method == "cell" else assemble_kron)(self.mesh)
        self.Mfull, self.Kfull = M, K
        self.M = restrict_interior(self.mesh, M)
        self.K = restrict_interior(self.mesh, K)
        self.idx = self.mesh.interior_index()

    def to_full(self, v_int: np.ndarray) -> np.ndarray:
        """Interior vector(s) -> full N^3 grid vector(s) with zero boundary.
        Accepts shape (nint,) or (Q, nint)."""
        v_int = np.asarray(v_int)
        out = np.zeros(v_int.shape[:-1] + (self.mesh.ndofs,), dtype=v_int.dtype)
        out[..., self.idx] = v_int
        return out

    def to_int(self, v_full: np.ndarray) -> np.ndarray:
        return np.asarray(v_full)[..., self.idx]


def interpolate(mesh: Mesh, func) -> np.ndarray:
    """Nodal interpolant on the full grid: func(x, y, z) at every node."""
    x = mesh.x1d
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return func(X, Y, Z).reshape(-1)


def load_separable(mesh: Mesh, f1) -> np.ndarray:
    """G_i = int_Omega f1(x) f1(y) f1(z) phi_i, by the (k+1)^3 Gauss rule per
    cell.  For a product source the cell integral factorises exactly into
    1D Gauss sums, g = g1 (x) g1 (x) g1 with g1_i = sum_cells sum_q w_q h f1(x_q) l_i(x_q).
    Returns the full-grid vector (boundary entries are included; the caller
    restricts to the interior)."""
    k, h, N = mesh.k, mesh.h, mesh.N
    qx, qw = gauss_rule(k + 1)
    B = lagrange_values(mesh.el.nodes, qx)
    g1 = np.zeros(N)
    for e in range(mesh.n):
        xq = (e + qx) * h
        g1[e * k:e * k + k + 1] += B.T @ (qw * h * f1(xq))
    return np.einsum("z,y,x->zyx", g1, g1, g1).reshape(-1)


def prolongation_1d(mesh_c: Mesh) -> np.ndarray:
    """Global 1D prolongation (N_f x N_c) from the n-cell to the 2n-cell
    partition: P[f, c] = value of the coarse basis function c at fine node f."""
    k, Nc = mesh_c.k, mesh_c.N
    Nf = 2 * mesh_c.n * k + 1
    Pe = mesh_c.el.prolongation()          # (2k+1, k+1)
    P = np.zeros((Nf, Nc))
    for e in range(mesh_c.n):
        P[2 * e * k:2 * e * k + 2 * k + 1, e * k:e * k + k + 1] = Pe
    return P


def prolongation_3d(mesh_c: Mesh):
    """P = P1 (x) P1 (x) P1 (tensor-product basis), full grids."""
    P1 = sp.csr_matrix(prolongation_1d(mesh_c))
    return sp.kron(P1, sp.kron(P1, P1), format="csr")
