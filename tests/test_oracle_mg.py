"""Pins of the oracle's Chebyshev smoother, multigrid V-cycle, block
preconditioner (eq. irk:P) and FGMRES."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.fgmres import IterativeStepper, fgmres
from oracle.multigrid import BlockMG, BlockPreconditioner, Hierarchy, chebyshev, level_sizes
from oracle.step import DirectStepper
from oracle.tableau import RadauIIA


def test_level_sizes():
    assert level_sizes(64) == [64, 32, 16, 8, 4, 2, 1]
    assert level_sizes(48) == [48, 24, 12, 6, 3]
    assert level_sizes(5) == [5]


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
@pytest.mark.parametrize("x0_zero", [True, False])
def test_chebyshev_error_is_scaled_chebyshev_polynomial(degree, x0_zero):
    """For D^-1 A with eigenvalue t in [lo, up], the Chebyshev iteration
    multiplies the error component by T_nu((theta - t)/delta) / T_nu(theta/delta)
    (closed form; T_nu the Chebyshev polynomial of the first kind)."""
    rng = np.random.default_rng(degree)
    t = np.linspace(0.05, 2.0, 40)
    d = rng.uniform(0.5, 2.0, t.size)            # Jacobi diagonal
    A = sp.diags(t * d)                           # D^-1 A = diag(t)
    xs = rng.standard_normal(t.size)
    b = A @ xs
    x0 = None if x0_zero else rng.standard_normal(t.size)
    up, lo = 2.1, 0.14
    x = chebyshev(A, 1.0 / d, b, x0, degree, up, lo)
    theta, delta = (up + lo) / 2, (up - lo) / 2
    Tn = np.polynomial.chebyshev.Chebyshev.basis(degree)
    factor = Tn((theta - t) / delta) / Tn(theta / delta)
    e0 = xs - (np.zeros_like(xs) if x0 is None else x0)
    np.testing.assert_allclose(xs - x, factor * e0, atol=1e-12)


@pytest.fixture(scope="module")
def mg8():
    tab = RadauIIA(3)
    hier = Hierarchy(8, 2)
    return tab, hier, BlockMG(hier, tab.lam, 0.05, degree=3)


def test_vcycle_linear_and_symmetric(mg8):
    tab, hier, mg = mg8
    n = hier.levels[0].M.shape[0]
    rng = np.random.default_rng(0)
    b1, b2 = rng.standard_normal(n), rng.standard_normal(n)
    for i in range(tab.Q):
        v1, v2 = mg.vcycle_block(i, b1), mg.vcycle_block(i, b2)
        np.testing.assert_allclose(mg.vcycle_block(i, 2.5 * b1 + b2), 2.5 * v1 + v2, atol=1e-12 * np.abs(v1).max())
        assert abs(v1 @ b2 - b1 @ v2) < 1e-12 * abs(v1 @ b2)


def test_vcycle_contraction(mg8):
    """As a stationary iteration x <- x + V(b - A x) the V-cycle contracts
    strongly (power iteration on I - V A)."""
    tab, hier, mg = mg8
    A0 = mg.A[0]
    rng = np.random.default_rng(1)
    for i in range(tab.Q):
        e = rng.standard_normal(A0[i].shape[0])
        rate = 0.0
        for _ in range(12):
            e_new = e - mg.vcycle_block(i, A0[i] @ e)
            rate = np.linalg.norm(e_new) / np.linalg.norm(e)
            e = e_new / np.linalg.norm(e_new)
        assert rate < 0.3, (i, rate)


def test_eig_bounds_are_upper_bounds(mg8):
    tab, hier, mg = mg8
    for l in range(hier.nlevels):
        assert mg.eig_max[l] >= mg.max_eig_exact(l) * 1.19


def test_block_preconditioner_with_exact_blocks():
    """Eq. (irk:P): with exact block solves, P^-1 inverts L (x) M + tau I (x) K."""
    tab = RadauIIA(4)
    hier = Hierarchy(2, 2)
    M, K = hier.levels[0].M, hier.levels[0].K
    tau = 0.03

    class Exact:
        def vcycle(self, b):
            return np.stack([spla.spsolve((tab.lam[i] * M + tau * K).tocsc(), b[i]) for i in range(tab.Q)])

    P = BlockPreconditioner(tab, Exact())
    n = M.shape[0]
    x = np.random.default_rng(2).standard_normal(tab.Q * n)
    Lop = sp.kron(sp.csr_matrix(tab.L), M) + tau * sp.kron(sp.identity(tab.Q), K)
    np.testing.assert_allclose(P.apply(Lop @ x), x, atol=1e-10 * np.abs(x).max())


def test_fgmres_solves_small_dense():
    rng = np.random.default_rng(5)
    A = np.eye(30) * 4 + rng.standard_normal((30, 30)) * 0.3
    b = rng.standard_normal(30)
    x, its, rr = fgmres(lambda v: A @ v, lambda v: v / 4.0, b, rtol=1e-13, restart=8)
    np.testing.assert_allclose(A @ x, b, atol=1e-11)
    assert rr < 1e-12


@pytest.mark.parametrize("Q", [2, 3])
def test_iterative_step_equals_direct(Q):
    """FGMRES on eq. (irk:A) with the eq. (irk:P) multigrid preconditioner
    reproduces the direct solve of the stage system."""
    n, k, tau = 4, 2, 0.05
    tab = RadauIIA(Q)
    st = IterativeStepper(n, k, tab, tau)
    rng = np.random.default_rng(Q)
    y = rng.standard_normal(st.M.shape[0])
    gbar = rng.standard_normal((Q, st.M.shape[0]))
    yi, its, rr = st.step(y, gbar, rtol=1e-14)
    yd, _ = DirectStepper(st.M, st.K, tab, tau).step(y, gbar)
    assert np.linalg.norm(yi - yd) / np.linalg.norm(yd) < 1e-12
    assert its < 30
