"""Single rows of the assembled operators (oracle).

Test infrastructure only: see ``oracle/__init__.py``.

For meshes too large to assemble, (M u)(node) and (K u)(node) are computed one
node at a time as the sum over the (up to 8) cells that contain the node of
the node's row of the element matrix times the cell's nodal values, which is
exactly what the cell-loop assembly adds into that row.
"""
from __future__ import annotations

import itertools

import numpy as np

from .fe import element_matrices_3d


class PointwiseOperator:
    def __init__(self, n: int, k: int):
        self.n, self.k = n, k
        self.N = n * k + 1
        self.Me, self.Ke = element_matrices_3d(k, 1.0 / n)

    def _cells_1d(self, g):
        """(cell, local index) pairs of the 1D elements that contain node g."""
        k, n = self.k, self.n
        out = []
        e, a = divmod(g, k)
        if e < n:
            out.append((e, a))
        if a == 0 and e > 0:
            out.append((e - 1, k))
        return out

    def rows(self, u, nodes, absolute=False):
        """(M u) and (K u) at the given nodes.

        u: full-grid vector (N^3,) with zero boundary entries (boundary values
        are ignored: homogeneous Dirichlet).  nodes: iterable of (ix, iy, iz).
        Boundary nodes return 0 (the Dirichlet-eliminated operator).  With
        absolute=True the entries of the element matrices are replaced by their
        absolute values (the |M| |u| bound used for rounding tolerances)."""
        Me = np.abs(self.Me) if absolute else self.Me
        Ke = np.abs(self.Ke) if absolute else self.Ke
        N, k = self.N, self.k
        u3 = np.asarray(u).reshape(N, N, N).copy()
        u3[0, :, :] = 0; u3[-1, :, :] = 0
        u3[:, 0, :] = 0; u3[:, -1, :] = 0
        u3[:, :, 0] = 0; u3[:, :, -1] = 0
        n1 = k + 1
        outM, outK = [], []
        for (ix, iy, iz) in nodes:
            if min(ix, iy, iz) == 0 or max(ix, iy, iz) == N - 1:
                outM.append(0.0); outK.append(0.0)
                continue
            sm = sk = 0.0
            for (ex, ax), (ey, ay), (ez, az) in itertools.product(
                    self._cells_1d(ix), self._cells_1d(iy), self._cells_1d(iz)):
                loc = u3[ez * k:ez * k + n1, ey * k:ey * k + n1, ex * k:ex * k + n1].reshape(-1)
                row = ax + n1 * (ay + n1 * az)
                sm += Me[row] @ loc
                sk += Ke[row] @ loc
            outM.append(sm); outK.append(sk)
        return np.array(outM), np.array(outK)
