"""Pins of the oracle's deformed-mesh matrices: the affine case, the analytic
Jacobian, and integrals over the physical domain whose exact values are known
(volume, the energy of the coordinate functions, the mean of x_1)."""
import numpy as np
import pytest

from oracle.assemble import Mesh, Problem
from oracle.deformed import DeformedProblem, assemble, phi, phi_jacobian, sampled_rows


@pytest.mark.parametrize("n,k", [(2, 2), (3, 1), (2, 3)])
def test_zero_deformation_is_the_affine_mesh(n, k):
    p = Problem(n, k, "cell")
    M, K = assemble(Mesh(n, k), 0.0)
    assert abs(M - p.Mfull).max() <= 1e-15 * abs(p.Mfull).max()
    assert abs(K - p.Kfull).max() <= 1e-14 * abs(p.Kfull).max()


def test_jacobian_matches_finite_differences():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (50, 3))
    eps, d = 0.15, 1e-6
    J = phi_jacobian(x, eps)
    for j in range(3):
        e = np.zeros(3)
        e[j] = d
        fd = (phi(x + e, eps) - phi(x - e, eps)) / (2 * d)
        np.testing.assert_allclose(J[:, :, j], fd, atol=1e-8)


def test_boundary_is_fixed():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (40, 3))
    for d in range(3):
        for v in (0.0, 1.0):
            y = x.copy()
            y[:, d] = v
            np.testing.assert_allclose(phi(y, 0.2), y, atol=1e-15)


def _coordinate_interpolants(mesh, eps):
    """Nodal values of the physical coordinates x_1, x_2, x_3 at the mapped nodes."""
    X = np.stack(np.meshgrid(mesh.x1d, mesh.x1d, mesh.x1d, indexing="ij"), axis=-1)   # [x, y, z]
    X = X.transpose(2, 1, 0, 3).reshape(-1, 3)                                       # x fastest
    return phi(X, eps).T


@pytest.mark.parametrize("n,k", [(4, 3), (3, 4)])
def test_physical_integrals(n, k):
    """With u_d the interpolant of the physical coordinate x_d (not in the
    space on a curved mesh, but close to it): u_d^T K u_e -> delta_de |Omega| = delta_de,
    1^T M u_1 -> int x_1 = 1/2, 1^T M 1 = |Omega| = 1, K 1 = 0."""
    eps = 0.1
    mesh = Mesh(n, k)
    M, K = assemble(mesh, eps)
    U = _coordinate_interpolants(mesh, eps)
    one = np.ones(mesh.ndofs)
    assert abs(K @ one).max() <= 1e-12 * abs(K).max()
    assert abs(one @ M @ one - 1.0) <= 1e-10
    G = U @ (K @ U.T)
    np.testing.assert_allclose(G, np.eye(3), atol=2e-5)
    assert abs(one @ M @ U[0] - 0.5) <= 1e-6


def test_physical_integrals_converge():
    """The coordinate-energy error shrinks under refinement (interpolation error
    of the curved map), so the agreement above is not a coincidence."""
    eps, k = 0.15, 2
    errs = []
    for n in (2, 4, 8):
        mesh = Mesh(n, k)
        _, K = assemble(mesh, eps)
        U = _coordinate_interpolants(mesh, eps)
        errs.append(np.abs(U @ (K @ U.T) - np.eye(3)).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < errs[0] / 10


def test_matrices_symmetric_and_definite():
    p = DeformedProblem(3, 2, 0.12)
    assert abs(p.M - p.M.T).max() <= 1e-15 and abs(p.K - p.K.T).max() <= 1e-13
    assert np.linalg.eigvalsh(p.M.toarray()).min() > 0
    assert np.linalg.eigvalsh(p.K.toarray()).min() > 0


def test_sampled_rows_equal_assembled_rows():
    n, k, eps = 3, 3, 0.1
    mesh = Mesh(n, k)
    M, K = assemble(mesh, eps)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(mesh.ndofs)
    u[~mesh.interior_mask()] = 0
    N = mesh.N
    nodes = [(1, 1, 1), (3, 3, 3), (3, 5, 6), (8, 2, 7), (4, 4, 1)]
    m, kk = sampled_rows(n, k, eps, u, nodes)
    rows = [a + N * (b + N * c) for a, b, c in nodes]
    np.testing.assert_allclose(m, (M @ u)[rows], atol=1e-15)
    np.testing.assert_allclose(kk, (K @ u)[rows], atol=1e-12)



@pytest.mark.parametrize("n,k", [(2, 2), (3, 3)])
def test_sampled_absolute_rows_bound_and_single_cell_equality(n, k):
    """The |M_e| |u| bound of the sampled rows (rounding tolerances of the
    deformed-operator tests) is at least |M| |u| of the assembled deformed
    matrices everywhere, and equal to it at nodes inside a single cell, where
    no two cells add into the row."""
    eps = 0.08
    mesh = Mesh(n, k)
    M, K = assemble(mesh, eps)
    u = np.random.default_rng(7).standard_normal(mesh.ndofs)
    u[~mesh.interior_mask()] = 0
    au = np.abs(u)
    N = mesh.N
    g1 = range(1, N - 1)
    allint = [(a, b, c) for c in g1 for b in g1 for a in g1]
    inner = [(a, b, c) for (a, b, c) in allint if a % k and b % k and c % k]
    for nodes in (allint, inner):
        m, kk = sampled_rows(n, k, eps, au, nodes, absolute=True)
        rows = [a + N * (b + N * c) for a, b, c in nodes]
        Ma, Ka = (abs(M) @ au)[rows], (abs(K) @ au)[rows]
        if nodes is inner:
            np.testing.assert_allclose(m, Ma, rtol=1e-13)
            np.testing.assert_allclose(kk, Ka, rtol=1e-13)
        else:
            assert np.all(m >= Ma * (1 - 1e-13)) and np.all(kk >= Ka * (1 - 1e-13))
            assert np.all(Ma >= np.abs(M @ u)[rows] * (1 - 1e-13))
            assert np.all(Ka >= np.abs(K @ u)[rows] * (1 - 1e-13))
    # Q_1 element mass entries are all positive: no cancellation anywhere
    mesh1 = Mesh(3, 1)
    M1, _ = assemble(mesh1, eps)
    u1 = np.abs(np.random.default_rng(8).standard_normal(mesh1.ndofs))
    u1[~mesh1.interior_mask()] = 0
    nodes1 = [(1, 1, 1), (2, 1, 2), (1, 2, 1), (2, 2, 2)]
    m1, _ = sampled_rows(3, 1, eps, u1, nodes1, absolute=True)
    np.testing.assert_allclose(m1, (abs(M1) @ u1)[[a + 4 * (b + 4 * c) for a, b, c in nodes1]], rtol=1e-13)

def test_deformed_hierarchy_nested_and_affine_limit():
    """eps = 0 gives the affine hierarchy.  With eps != 0 the spaces stay
    nested (the same P), and the Galerkin product P^T M_f P differs from the
    rediscretised coarse matrix only by the quadrature error of the curved
    cells (it would be equal with exact integration)."""
    from oracle.deformed import DeformedHierarchy
    from oracle.multigrid import Hierarchy
    h0 = DeformedHierarchy(4, 2, 0.0)
    ha = Hierarchy(4, 2, "cell")
    for a, b in zip(h0.levels, ha.levels):
        assert abs(a.M - b.M).max() <= 1e-15 and abs(a.K - b.K).max() <= 1e-13
    h = DeformedHierarchy(4, 2, 0.08)
    for l in range(h.nlevels - 1):
        PtMP = h.P[l].T @ h.levels[l].M @ h.P[l]
        Mc = h.levels[l + 1].M
        # Galerkin product and rediscretisation differ only by quadrature error
        assert abs(PtMP - Mc).max() <= 0.05 * abs(Mc).max()


def test_vcycle_on_deformed_levels_contracts():
    from oracle.deformed import DeformedHierarchy
    from oracle.multigrid import BlockMG
    from oracle.tableau import RadauIIA
    tab = RadauIIA(2)
    h = DeformedHierarchy(8, 2, 0.08)
    mg = BlockMG(h, tab.lam, 0.05, degree=3)
    A = mg.A[0][0]
    n = A.shape[0]
    rng = np.random.default_rng(3)
    e = rng.standard_normal(n)
    e0 = np.sqrt(e @ (A @ e))
    for _ in range(3):
        e = e - mg.vcycle_block(0, A @ e)
    assert np.sqrt(e @ (A @ e)) < 0.2 ** 3 * e0
    b1, b2 = rng.standard_normal(n), rng.standard_normal(n)
    v1, v2 = mg.vcycle_block(1, b1), mg.vcycle_block(1, b2)
    assert abs(v1 @ b2 - b1 @ v2) < 1e-12 * abs(v1 @ b2)
