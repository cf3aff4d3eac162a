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


def _cell_interior(N, k):
    """Nodes strictly inside a cell in all three directions (one cell each)."""
    inner = [g for g in range(1, N - 1) if g % k != 0]
    return [(ix, iy, iz) for iz in inner for iy in inner for ix in inner]


@pytest.mark.parametrize("n,k", [(2, 1), (3, 1)])
def test_absolute_rows_q1_equal_abs_matrix(n, k):
    """Q_1: every element mass entry is positive and every element stiffness
    entry off the diagonal is non-positive, so assembly never cancels and the
    element-wise |M_e| |u| bound equals |M| |u| (and |K| |u|) of the assembled
    matrices at every node."""
    p = Problem(n, k, "cell")
    u = p.to_full(np.random.default_rng(12).standard_normal(p.M.shape[0]))
    au = np.abs(p.to_int(u))
    Ma = p.to_full(abs(p.M) @ au)
    Ka = p.to_full(abs(p.K) @ au)
    N = p.mesh.N
    nodes = [(ix, iy, iz) for iz in range(N) for iy in range(N) for ix in range(N)]
    m, kk = PointwiseOperator(n, k).rows(np.abs(u), nodes, absolute=True)
    np.testing.assert_allclose(m, Ma, rtol=1e-13, atol=1e-17)
    np.testing.assert_allclose(kk, Ka, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("n,k", [(2, 2), (2, 3), (1, 5)])
def test_absolute_rows_bound_and_single_cell_equality(n, k):
    """Any degree: the bound is at least |M| |u| >= |M u| at every node (the
    property the rounding tolerances rely on), and at nodes inside a single
    cell, where no two cells add into the row, it equals |M| |u| of the
    assembled matrices exactly."""
    p = Problem(n, k, "cell")
    u = p.to_full(np.random.default_rng(13).standard_normal(p.M.shape[0]))
    au = np.abs(p.to_int(u))
    N = p.mesh.N
    full = [(ix, iy, iz) for iz in range(N) for iy in range(N) for ix in range(N)]
    pw = PointwiseOperator(n, k)
    m, kk = pw.rows(np.abs(u), full, absolute=True)
    Ma, Ka = p.to_full(abs(p.M) @ au), p.to_full(abs(p.K) @ au)
    Mu, Ku = np.abs(p.to_full(p.M @ p.to_int(u))), np.abs(p.to_full(p.K @ p.to_int(u)))
    assert np.all(m >= Ma * (1 - 1e-13)) and np.all(Ma >= Mu * (1 - 1e-13))
    assert np.all(kk >= Ka * (1 - 1e-13)) and np.all(Ka >= Ku * (1 - 1e-13))
    inner = _cell_interior(N, k)
    idx = [ix + N * (iy + N * iz) for ix, iy, iz in inner]
    mi, ki = pw.rows(np.abs(u), inner, absolute=True)
    np.testing.assert_allclose(mi, Ma[idx], rtol=1e-13)
    np.testing.assert_allclose(ki, Ka[idx], rtol=1e-13)
    # and the signed rows are smaller there whenever some entry cancels
    ms, _ = pw.rows(u, inner)
    assert np.all(np.abs(ms) <= mi * (1 + 1e-13))
