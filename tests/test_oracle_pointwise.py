"""Pin of the oracle's single-row operator evaluation against the assembled
cell-loop matrices (brute force on small meshes)."""
import numpy as np
import pytest

from oracle.assemble import Problem
from oracle.pointwise import PointwiseOperator


@pytest.mark.parametrize("n,k", [(2, 1), (3, 2), (2, 4), (1, 6)])
def test_rows_match_assembled(n, k):
    p = Problem(n, k, "cell")
    rng = np.random.default_rng(11)
    u = p.to_full(rng.standard_normal(p.M.shape[0]))
    Mu = p.to_full(p.M @ p.to_int(u))
    Ku = p.to_full(p.K @ p.to_int(u))
    N = p.mesh.N
    nodes = [(ix, iy, iz) for iz in range(N) for iy in range(N) for ix in range(N)]
    pw = PointwiseOperator(n, k)
    m, kk = pw.rows(u, nodes)
    np.testing.assert_allclose(m, Mu, atol=1e-15 * np.abs(Mu).max() * 10)
    np.testing.assert_allclose(kk, Ku, atol=1e-13 * np.abs(Ku).max())
