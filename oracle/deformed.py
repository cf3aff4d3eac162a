"""Finite-element matrices on a deformed (non-affine) hexahedral mesh (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

The paper works on affine meshes and names the cost of non-affine geometry
as the reason to batch stages (Sec. 3.4): the per-quadrature-point Jacobian
data is then read once for all stages.  This module defines the deformed
problem that the library's deformed-mesh operator is checked against.

Mesh: the uniform n^3 mesh of the unit cube mapped by

    Phi(x) = x + eps s(x) (1, 1, 1),   s(x) = sin(pi x1) sin(pi x2) sin(pi x3),

which is the identity on the boundary of the cube and maps the cube onto
itself (for |eps| small enough that det Phi' > 0).  Cell c with lower corner
h c is the image of the reference cube by F(xi) = Phi(h (c + xi)); the
finite-element space is {phi o F^-1} with phi the Q_k tensor Lagrange basis on
Gauss-Lobatto nodes (the same reference element as on the affine mesh).
Element integrals use the (k+1)^3-point Gauss rule, as on the affine mesh:

    M_e[i, j] = sum_q w_q det J_q  phi_i(xi_q) phi_j(xi_q),
    K_e[i, j] = sum_q w_q det J_q  (J_q^-T grad phi_i)(xi_q) . (J_q^-T grad phi_j)(xi_q),

with J_q = F'(xi_q) = h Phi'(h (c + xi_q)).  Phi' = I + eps (1,1,1)^T grad s^T
is written out analytically.  Dirichlet conditions as on the affine mesh.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .assemble import Mesh, prolongation_3d, restrict_interior
from .fe import Element1D


def phi(x, eps):
    """Phi at points x (..., 3)."""
    x = np.asarray(x, dtype=float)
    s = np.prod(np.sin(np.pi * x), axis=-1)
    return x + eps * s[..., None]


def phi_jacobian(x, eps):
    """Phi'(x) (..., 3, 3), [i, j] = d Phi_i / d x_j."""
    x = np.asarray(x, dtype=float)
    sn, cs = np.sin(np.pi * x), np.cos(np.pi * x)
    grad = np.stack([np.pi * cs[..., 0] * sn[..., 1] * sn[..., 2],
                     np.pi * sn[..., 0] * cs[..., 1] * sn[..., 2],
                     np.pi * sn[..., 0] * sn[..., 1] * cs[..., 2]], axis=-1)
    J = np.broadcast_to(np.eye(3), x.shape[:-1] + (3, 3)).copy()
    J += eps * grad[..., None, :]          # every row i gets eps * grad s
    return J


class _RefData:
    """Reference basis values and gradients at the Gauss points:
    val (nq^3, n1^3), gref (3, nq^3, n1^3) with point index qa + nq (qb + nq qc)
    and local node index a + n1 (b + n1 c), x fastest; 3D weights w (nq^3,)."""

    def __init__(self, k):
        el = Element1D(k)
        B, D, qw = el.B, el.D, el.qw
        n1 = nq = k + 1
        self.k, self.qx, self.el = k, el.qx, el
        self.w = np.einsum("a,b,c->cba", qw, qw, qw).reshape(-1)
        self.val = np.einsum("xa,yb,zc->zyxcba", B, B, B).reshape(nq ** 3, n1 ** 3)
        self.gref = np.stack([np.einsum("xa,yb,zc->zyxcba", D, B, B).reshape(nq ** 3, n1 ** 3),
                              np.einsum("xa,yb,zc->zyxcba", B, D, B).reshape(nq ** 3, n1 ** 3),
                              np.einsum("xa,yb,zc->zyxcba", B, B, D).reshape(nq ** 3, n1 ** 3)])
        # reference coordinates of the points, (nq^3, 3), point qa + nq (qb + nq qc)
        idx = np.arange(nq ** 3)
        self.xi = np.stack([self.qx[idx % nq], self.qx[(idx // nq) % nq], self.qx[idx // nq ** 2]], axis=-1)


def _point_coords(ref, n, cells=None):
    """Undeformed coordinates of the Gauss points of the given cells (index
    cx + n (cy + n cz); all cells if None): (ncells, nq^3, 3)."""
    h = 1.0 / n
    c = np.arange(n ** 3) if cells is None else np.asarray(cells)
    corner = np.stack([c % n, (c // n) % n, c // (n * n)], axis=-1).astype(float)
    return h * (corner[:, None, :] + ref.xi[None, :, :])


def cell_dofs(n, k, cells):
    """Global node indices (ncells, (k+1)^3) of the given cells, local index
    a + (k+1)(b + (k+1)c)."""
    N, n1 = n * k + 1, k + 1
    c = np.asarray(cells)
    loc = np.arange(n1 ** 3)
    a, b, cc = loc % n1, (loc // n1) % n1, loc // (n1 * n1)
    cx, cy, cz = c % n, (c // n) % n, c // (n * n)
    return ((cx[:, None] * k + a) + N * ((cy[:, None] * k + b) + N * (cz[:, None] * k + cc)))


def cell_geometry(n, k, eps, cells=None):
    """Per cell and Gauss point: w_q det J_q and the physical-gradient map
    J_q^-T, for all cells or the given cell indices (cx + n (cy + n cz))."""
    ref = _RefData(k)
    x = _point_coords(ref, n, cells)
    J = (1.0 / n) * phi_jacobian(x, eps)
    det = np.linalg.det(J)
    JinvT = np.swapaxes(np.linalg.inv(J), -1, -2)
    return ref, ref.w[None, :] * det, JinvT


def element_matrices(n, k, eps, cells=None):
    """(Me, Ke) of shape (ncells, n1^3, n1^3) for all cells or the given ones."""
    ref, wdet, JinvT = cell_geometry(n, k, eps, cells)
    # physical gradients of every basis function at every point: (ncell, nq^3, 3, n1^3)
    gphys = np.einsum("cqij,jqa->cqia", JinvT, ref.gref)
    Me = np.einsum("cq,qa,qb->cab", wdet, ref.val, ref.val)
    Ke = np.einsum("cq,cqia,cqib->cab", wdet, gphys, gphys)
    return Me, Ke


def assemble(mesh: Mesh, eps: float):
    """Full (boundary-inclusive) M and K on the deformed mesh, cell loop."""
    Me, Ke = element_matrices(mesh.n, mesh.k, eps)
    dofs = mesh.cell_dofs()
    ncell, nl = dofs.shape
    rows = np.repeat(dofs, nl, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, nl)).reshape(-1)
    shape = (mesh.ndofs, mesh.ndofs)
    M = sp.coo_matrix((Me.reshape(-1), (rows, cols)), shape=shape).tocsr()
    K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=shape).tocsr()
    M.sum_duplicates()
    K.sum_duplicates()
    return M, K


class DeformedProblem:
    """Interior (Dirichlet-eliminated) M and K of the deformed mesh."""

    def __init__(self, n: int, k: int, eps: float):
        self.mesh = Mesh(n, k)
        self.eps = eps
        self.Mfull, self.Kfull = assemble(self.mesh, eps)
        self.M = restrict_interior(self.mesh, self.Mfull)
        self.K = restrict_interior(self.mesh, self.Kfull)
        self.idx = self.mesh.interior_index()

    def to_full(self, v_int):
        v_int = np.asarray(v_int)
        out = np.zeros(v_int.shape[:-1] + (self.mesh.ndofs,), dtype=v_int.dtype)
        out[..., self.idx] = v_int
        return out

    def to_int(self, v_full):
        return np.asarray(v_full)[..., self.idx]


def sampled_rows(n, k, eps, u_full, nodes, absolute=False):
    """(M u)[node] and (K u)[node] for interior nodes (ix, iy, iz) of the full
    grid, from the element matrices of the cells around each node only (for
    meshes too large to assemble).  u_full: boundary entries are ignored.
    With absolute, the entries of the element matrices enter by magnitude
    (|M| u and |K| u, for rounding-error bounds)."""
    N = n * k + 1
    u = np.array(u_full, dtype=float).reshape(N, N, N)
    u[0], u[-1], u[:, 0], u[:, -1], u[:, :, 0], u[:, :, -1] = 0, 0, 0, 0, 0, 0
    u = u.reshape(-1)
    out_m, out_k = [], []
    n1 = k + 1
    for (ix, iy, iz) in nodes:
        cells, locs = [], []
        for cz in {max(0, (iz - 1) // k), min(n - 1, iz // k)}:
            for cy in {max(0, (iy - 1) // k), min(n - 1, iy // k)}:
                for cx in {max(0, (ix - 1) // k), min(n - 1, ix // k)}:
                    a, b, c = ix - cx * k, iy - cy * k, iz - cz * k
                    if 0 <= a <= k and 0 <= b <= k and 0 <= c <= k:
                        cells.append(cx + n * (cy + n * cz))
                        locs.append(a + n1 * (b + n1 * c))
        Me, Ke = element_matrices(n, k, eps, cells)
        if absolute:
            Me, Ke = np.abs(Me), np.abs(Ke)
        dofs = cell_dofs(n, k, cells)
        mv = sum(Me[e, locs[e]] @ u[dofs[e]] for e in range(len(cells)))
        kv = sum(Ke[e, locs[e]] @ u[dofs[e]] for e in range(len(cells)))
        out_m.append(mv)
        out_k.append(kv)
    return np.array(out_m), np.array(out_k)


class DeformedHierarchy:
    """Level matrices of the deformed mesh on every multigrid level (n, n/2,
    ... while even), each rediscretised on its own mesh mapped by the same
    Phi, with the interior prolongations of the affine hierarchy: the coarse
    space is nested in the fine one because a coarse cell's reference
    polynomials are polynomials in the reference coordinates of its fine
    cells (the fine cells are images of halves of the coarse reference cube
    under the same map).  Duck-types oracle.multigrid.Hierarchy for BlockMG."""

    def __init__(self, n: int, k: int, eps: float):
        from .multigrid import level_sizes
        self.k = k
        self.sizes = level_sizes(n)
        self.levels = [DeformedProblem(m, k, eps) for m in self.sizes]
        self.P = []
        for l in range(len(self.sizes) - 1):
            fine, coarse = self.levels[l], self.levels[l + 1]
            Pf = prolongation_3d(coarse.mesh)
            self.P.append(Pf[fine.idx][:, coarse.idx].tocsr())

    @property
    def nlevels(self):
        return len(self.levels)
