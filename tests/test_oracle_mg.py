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


def _q1_max_eig_closed_form(n, lams, tau):
    """Largest eigenvalue of D^-1 (lam M + tau K) over the blocks on the uniform
    n^3 mesh of Q_1 elements, in closed form.  The 1D matrices m (mass) and a
    (stiffness) are tridiagonal Toeplitz on the interior nodes, so the discrete
    sine modes theta_d = j_d pi / n (j_d = 1..n-1) are eigenvectors of both,
    with eigenvalues (h/3)(2 + cos theta) and (2/h)(1 - cos theta); the 3D
    matrices are Kronecker sums of them and the Jacobi diagonal is constant,
    (2h/3)^3 for M and 3 (2/h)(2h/3)^2 for K."""
    h = 1.0 / n
    th = np.arange(1, n) * np.pi / n
    mu_m = (h / 3) * (2 + np.cos(th))
    mu_a = (2 / h) * (1 - np.cos(th))
    mz, my, mx = np.meshgrid(mu_m, mu_m, mu_m, indexing="ij")
    az, ay, ax = np.meshgrid(mu_a, mu_a, mu_a, indexing="ij")
    eM = mz * my * mx
    eK = az * my * mx + mz * ay * mx + mz * my * ax
    dM = (2 * h / 3) ** 3
    dK = 3 * (2 / h) * (2 * h / 3) ** 2
    return max(float(((l * eM + tau * eK) / (l * dM + tau * dK)).max()) for l in lams)


@pytest.mark.parametrize("n,Q,tau", [(8, 3, 0.05), (24, 2, 1e-3), (6, 4, 0.7)])
def test_max_eig_exact_q1_closed_form(n, Q, tau):
    """Sec. 5.4 (one Chebyshev bound over all blocks): the oracle's largest
    eigenvalue of D^-1 A over the blocks lam_i M + tau K equals the sine-mode
    closed form on every level of a Q_1 hierarchy (the dense path for small
    levels, the sparse eigensolver for 23^3 interior unknowns)."""
    tab = RadauIIA(Q)
    hier = Hierarchy(n, 1)
    mg = BlockMG(hier, tab.lam, tau, degree=2, eig_max=[1.0] * hier.nlevels)
    for l, m in enumerate(hier.sizes):
        got = mg.max_eig_exact(l)
        if m == 1:
            assert got == 1.0          # no interior unknowns on one cell
            continue
        want = _q1_max_eig_closed_form(m, tab.lam, tau)
        assert abs(got - want) <= 1e-9 * want, (l, m, got, want)


def test_max_eig_exact_between_rayleigh_and_gershgorin(mg8):
    """Q_2 (no closed form): the largest eigenvalue of D^-1 A lies above the
    Rayleigh quotient v^T A v / v^T D v of any vector and below the largest
    Gershgorin row sum of |D^-1 A|, for every block and level."""
    tab, hier, mg = mg8
    rng = np.random.default_rng(3)
    for l in range(hier.nlevels):
        if hier.levels[l].M.shape[0] == 0:
            continue
        lam = mg.max_eig_exact(l)
        ray = gersh = 0.0
        for Ai, Di in zip(mg.A[l], mg.Dinv[l]):
            for _ in range(5):
                v = rng.standard_normal(Ai.shape[0])
                ray = max(ray, (v @ (Ai @ v)) / (v @ (v / Di)))
            gersh = max(gersh, float((abs(Ai).multiply(Di[:, None])).sum(axis=1).max()))
        assert ray <= lam * (1 + 1e-12), (l, ray, lam)
        assert lam <= gersh * (1 + 1e-12), (l, lam, gersh)


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
