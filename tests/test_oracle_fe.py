"""Pins of the oracle's finite-element data and assembly (Sec. 5 set-up).

Closed forms (k = 1, 2 element matrices, Gauss-Lobatto points and weights),
exact integrals of polynomials, the Q_1 sine-mode spectrum, and the
cell-loop/Kronecker equivalence.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle.assemble import (Mesh, Problem, assemble_cell_loop, assemble_kron, interpolate,
                             load_separable, prolongation_1d, prolongation_3d)
from oracle.fe import Element1D, element_matrices_3d, gll_nodes

KS = [1, 2, 3, 4, 5, 6]


def test_k1_k2_element_matrices():
    e1 = Element1D(1)
    np.testing.assert_allclose(e1.mass, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    np.testing.assert_allclose(e1.stiff, [[1, -1], [-1, 1]], atol=1e-14)
    e2 = Element1D(2)
    np.testing.assert_allclose(e2.mass * 30, [[4, 2, -1], [2, 16, 2], [-1, 2, 4]], atol=1e-13)
    np.testing.assert_allclose(e2.stiff * 3, [[7, -8, 1], [-8, 16, -8], [1, -8, 7]], atol=1e-13)


def test_gll_closed_forms():
    np.testing.assert_allclose(gll_nodes(2), [0, 0.5, 1], atol=1e-16)
    s5 = 1 / np.sqrt(5)
    np.testing.assert_allclose(gll_nodes(3), [0, (1 - s5) / 2, (1 + s5) / 2, 1], atol=1e-15)
    s37 = np.sqrt(3 / 7)
    np.testing.assert_allclose(gll_nodes(4), [0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("k", KS)
def test_gll_nodes_and_weights(k):
    """Interior nodes are roots of P_k'(2x-1); the integrals of the Lagrange
    polynomials are the Gauss-Lobatto weights 1/(k(k+1) P_k(s_a)^2) on [0,1]."""
    x = gll_nodes(k)
    s = 2 * x - 1
    Pk = [0] * k + [1]
    if k > 1:
        np.testing.assert_allclose(npleg.legval(s[1:-1], npleg.legder(Pk)), 0, atol=1e-12)
    w = 1.0 / (k * (k + 1) * npleg.legval(s, Pk) ** 2)
    el = Element1D(k)
    np.testing.assert_allclose(el.mass.sum(axis=1), w, rtol=1e-13)
    np.testing.assert_allclose(x, 1 - x[::-1], atol=0)


@pytest.mark.parametrize("k", KS)
def test_element_integrals_exact_for_polynomials(k):
    """u^T mass v = int_0^1 x^i x^j and u^T stiff v = int_0^1 (x^i)'(x^j)'
    for the nodal values of monomials of degree <= k."""
    el = Element1D(k)
    x = el.nodes
    for i in range(k + 1):
        for j in range(k + 1):
            u, v = x ** i, x ** j
            assert abs(u @ el.mass @ v - 1.0 / (i + j + 1)) < 1e-13
            exact = i * j / (i + j - 1) if i > 0 and j > 0 else 0.0
            assert abs(u @ el.stiff @ v - exact) < 1e-11 * max(1, exact)
    # Lagrange property
    from oracle.fe import lagrange_values
    np.testing.assert_allclose(lagrange_values(x, x), np.eye(k + 1), atol=1e-14)


@pytest.mark.parametrize("k", KS)
def test_prolongation_interpolates_polynomials(k):
    el = Element1D(k)
    P = el.prolongation()
    xf = np.concatenate([0.5 * el.nodes, 0.5 + 0.5 * el.nodes[1:]])
    for deg in range(k + 1):
        np.testing.assert_allclose(P @ el.nodes ** deg, xf ** deg, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_3d_element_matrices_are_kronecker(k):
    h = 0.25
    Me, Ke = element_matrices_3d(k, h)
    el = Element1D(k)
    m, a = el.mass, el.stiff
    Mk = h ** 3 * np.kron(m, np.kron(m, m))
    Kk = h * (np.kron(a, np.kron(m, m)) + np.kron(m, np.kron(a, m)) + np.kron(m, np.kron(m, a)))
    np.testing.assert_allclose(Me, Mk, atol=1e-15 * np.abs(Mk).max() * 10)
    np.testing.assert_allclose(Ke, Kk, atol=1e-13 * np.abs(Kk).max())


@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (3, 2), (2, 3), (2, 4), (1, 6)])
def test_cell_loop_equals_kronecker(n, k):
    mesh = Mesh(n, k)
    M1, K1 = assemble_cell_loop(mesh)
    M2, K2 = assemble_kron(mesh)
    assert abs(M1 - M2).max() < 1e-15
    assert abs(K1 - K2).max() < 1e-12 * abs(K1).max()


@pytest.mark.parametrize("n,k", [(1, 1), (3, 1), (2, 2), (2, 4), (1, 5)])
def test_volume_and_constants(n, k):
    """Before Dirichlet elimination: 1^T M 1 = |Omega| = 1 and K 1 = 0."""
    mesh = Mesh(n, k)
    M, K = assemble_cell_loop(mesh)
    one = np.ones(mesh.ndofs)
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    assert np.abs(K @ one).max() < 1e-12 * abs(K).max()


@pytest.mark.parametrize("n,k", [(2, 2), (3, 2), (2, 3), (1, 4)])
def test_bubble_energy(n, k):
    """u = x(1-x)y(1-y)z(1-z) lies in the space for k >= 2 and vanishes on the
    boundary: u^T M u = (1/30)^3, u^T K u = 3 (1/3)(1/30)^2 = 1/900."""
    p = Problem(n, k, "cell")
    u = p.to_int(interpolate(p.mesh, lambda x, y, z: x * (1 - x) * y * (1 - y) * z * (1 - z)))
    assert abs(u @ (p.M @ u) - (1 / 30) ** 3) < 1e-16
    assert abs(u @ (p.K @ u) - 1 / 900) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 5])
def test_q1_sine_mode_spectrum(n):
    """Q_1 on the uniform mesh: the discrete sine modes are exact generalised
    eigenvectors, K s = lam M s, lam = sum_d (6/h^2)(1-cos t_d)/(2+cos t_d),
    t_d = m_d pi h."""
    p = Problem(n, 1, "cell")
    h = 1.0 / n
    for mx, my, mz in [(1, 1, 1), (1, 2, 1), (n - 1, 1, max(1, n - 2))]:
        if max(mx, my, mz) > n - 1:
            continue
        s = p.to_int(interpolate(p.mesh, lambda x, y, z: np.sin(mx * np.pi * x)
                                 * np.sin(my * np.pi * y) * np.sin(mz * np.pi * z)))
        lam = sum(6 / h ** 2 * (1 - np.cos(m * np.pi * h)) / (2 + np.cos(m * np.pi * h))
                  for m in (mx, my, mz))
        np.testing.assert_allclose(p.K @ s, lam * (p.M @ s), atol=1e-12 * lam * np.abs(p.M @ s).max())


@pytest.mark.parametrize("n,k", [(2, 1), (3, 2), (2, 4)])
def test_load_vector(n, k):
    """G_i = int f phi_i: with f = 1, sum G = |Omega| = 1; with f = 1 tested
    against the nodal interpolant of x (exact for k >= 1), sum G_i x_i = 1/2;
    for f(x)f(y)f(z), f = sin(pi x), sum G_i = (2/pi)^3 up to quadrature error."""
    mesh = Mesh(n, k)
    G = load_separable(mesh, lambda x: np.ones_like(x))
    assert abs(G.sum() - 1.0) < 1e-14
    xi = interpolate(mesh, lambda x, y, z: x)
    assert abs(G @ xi - 0.5) < 1e-14
    Gs = load_separable(mesh, lambda x: np.sin(np.pi * x))
    assert abs(Gs.sum() - (2 / np.pi) ** 3) < 0.05 * (1.0 / n) ** (2 * k)


@pytest.mark.parametrize("n,k", [(1, 2), (2, 1), (2, 3)])
def test_prolongation_3d_and_galerkin(n, k):
    """P maps the coarse interpolant of a Q_k polynomial to its fine
    interpolant; with nested spaces and exact quadrature, P^T A_f P = A_c."""
    mc, mf = Mesh(n, k), Mesh(2 * n, k)
    P = prolongation_3d(mc)
    f = lambda x, y, z: (x ** k - 0.3 * y) * (1 + z ** (k - 1)) * (2 - x * y) ** 0 + y ** k * z
    np.testing.assert_allclose(P @ interpolate(mc, f), interpolate(mf, f), atol=1e-13)
    Mc, Kc = assemble_cell_loop(mc)
    Mf, Kf = assemble_cell_loop(mf)
    assert abs(P.T @ Mf @ P - Mc).max() < 1e-15
    assert abs(P.T @ Kf @ P - Kc).max() < 1e-12 * abs(Kc).max()
    # the 1D prolongation rows at coarse vertices are unit rows
    P1 = prolongation_1d(mc)
    for e in range(n + 1):
        row = P1[2 * e * k]
        assert row[e * k] == 1.0 and np.count_nonzero(row) == 1
