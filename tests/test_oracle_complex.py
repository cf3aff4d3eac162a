"""Pins of the oracle's direct (complex) diagonalisation of A_Q^-1
(eq. irk:Ainv), the two-by-two real blocks and PRESB (Sec. 6, eqs. presb:a,
complex:twobytwo, presb:p)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.assemble import Problem
from oracle.complex_irk import (ComplexBlocks, ComplexStepper, Presb, block_operator, pair_matrix,
                                presb_matrix)
from oracle.step import DirectStepper, premultiplied_operator
from oracle.tableau import RadauIIA


def _pade_denominator_roots(Q):
    """Roots of the denominator of the (Q-1, Q) Pade approximant of exp(z),
    D(z) = sum_n (2Q-1-n)! Q! / ((2Q-1)! n! (Q-n)!) (-z)^n.  Radau IIA's
    stability function is that approximant and D(z) = det(I - z A), so its
    roots are the eigenvalues of A^-1."""
    f = math.factorial
    coef = [f(2 * Q - 1 - n) * f(Q) / (f(2 * Q - 1) * f(n) * f(Q - n)) * (-1) ** n for n in range(Q + 1)]
    return np.roots(coef[::-1])


def _key(z):
    return (round(z.real, 8), round(z.imag, 8))


@pytest.mark.parametrize("Q", range(1, 10))
def test_eigenvalues_are_pade_denominator_roots(Q):
    dec = ComplexBlocks(RadauIIA(Q))
    mine = list(dec.lam) + [np.conj(l) for l in dec.lam[:dec.npair]]
    ref = _pade_denominator_roots(Q)
    assert len(mine) == Q
    np.testing.assert_allclose(sorted(mine, key=_key), sorted(ref, key=_key), rtol=1e-9)
    assert dec.npair == Q // 2 and dec.nb == (Q + 1) // 2
    assert all(l.imag > 0 for l in dec.lam[:dec.npair])
    assert all(l.real > 0 for l in dec.lam)


@pytest.mark.parametrize("Q", range(1, 10))
def test_real_form_identities(Q):
    """T U = I and T A^-1 U = Lam_r, whose blocks are built from lam alone."""
    tab = RadauIIA(Q)
    dec = ComplexBlocks(tab)
    np.testing.assert_allclose(dec.T @ dec.U, np.eye(Q), atol=1e-11)
    scale = np.abs(dec.LamR).max()
    np.testing.assert_allclose(dec.T @ tab.Ainv @ dec.U, dec.LamR, atol=1e-10 * scale)


@pytest.mark.parametrize("Q", [2, 3, 4, 5])
def test_scalar_model_problem(Q):
    """M -> 1, K -> kappa: k = U (Lam_r + tau kappa I)^-1 T r solves
    (A^-1 + tau kappa I) k = r."""
    tab = RadauIIA(Q)
    dec = ComplexBlocks(tab)
    rng = np.random.default_rng(Q)
    r = rng.standard_normal(Q)
    for tk in (1e-3, 0.7, 40.0):
        k = dec.U @ np.linalg.solve(dec.LamR + tk * np.eye(Q), dec.T @ r)
        np.testing.assert_allclose(k, np.linalg.solve(tab.Ainv + tk * np.eye(Q), r), rtol=1e-10)


@pytest.fixture(scope="module")
def small():
    return Problem(3, 2)


@pytest.mark.parametrize("Q", [2, 3, 4])
def test_block_operator_is_complex_block(small, Q):
    """Pair slots (re, im) of (Lam_r (x) M + tau I (x) K) u equal the real and
    imaginary parts of (lam M + tau K)(u_re + i u_im); the real block is
    lam M + tau K."""
    p, tau = small, 0.03
    dec = ComplexBlocks(RadauIIA(Q))
    rng = np.random.default_rng(7)
    u = rng.standard_normal((Q, p.M.shape[0]))
    v = block_operator(dec, p.M, p.K, tau, u)
    Mc, Kc = p.M.astype(complex), p.K.astype(complex)
    for j in range(dec.nb):
        sl = dec.block_slots(j)
        lam = dec.lam[j]
        if len(sl) == 2:
            z = (lam * Mc + tau * Kc) @ (u[sl[0]] + 1j * u[sl[1]])
            np.testing.assert_allclose(v[sl[0]], z.real, atol=1e-12 * np.abs(z).max())
            np.testing.assert_allclose(v[sl[1]], z.imag, atol=1e-12 * np.abs(z).max())
            pm = pair_matrix(dec, p.M, p.K, tau, j)
            np.testing.assert_allclose(np.concatenate([v[sl[0]], v[sl[1]]]),
                                       pm @ np.concatenate([u[sl[0]], u[sl[1]]]), atol=1e-12 * np.abs(z).max())
        else:
            z = (lam.real * p.M + tau * p.K) @ u[sl[0]]
            np.testing.assert_allclose(v[sl[0]], z, atol=1e-12 * np.abs(z).max())


@pytest.mark.parametrize("Q", [1, 2, 3, 5])
def test_block_operator_similar_to_premultiplied(small, Q):
    """(U (x) I) (Lam_r (x) M + tau I (x) K) u = (A^-1 (x) M + tau I (x) K)(U (x) I) u."""
    p, tau = small, 0.2
    tab = RadauIIA(Q)
    dec = ComplexBlocks(tab)
    rng = np.random.default_rng(11)
    n = p.M.shape[0]
    u = rng.standard_normal((Q, n))
    lhs = dec.U @ block_operator(dec, p.M, p.K, tau, u)
    rhs = (premultiplied_operator(p.M, p.K, tab.Ainv, tau) @ (dec.U @ u).reshape(-1)).reshape(Q, n)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11 * np.abs(rhs).max())


def _exact_presb(dec, p, tau):
    H = [sp.csc_matrix(h * p.M + tau * p.K) for h in dec.h_shift()]
    return Presb(dec, p.M, lambda s, b: spla.spsolve(H[s], b))


@pytest.mark.parametrize("Q", [2, 3, 4])
def test_presb_factorisation(small, Q):
    """With exact inner solves, P (P^-1 r) = r for P = [[K', -M'], [M', K'+2M']]
    assembled from its definition, and the real block is solved exactly."""
    p, tau = small, 0.05
    dec = ComplexBlocks(RadauIIA(Q))
    pre = _exact_presb(dec, p, tau)
    rng = np.random.default_rng(5)
    n = p.M.shape[0]
    for j in range(dec.nb):
        sl = list(dec.block_slots(j))
        r = rng.standard_normal((len(sl), n))
        x = pre.apply_block(j, r)
        if len(sl) == 2:
            P = presb_matrix(dec, p.M, p.K, tau, j)
            np.testing.assert_allclose(P @ x.reshape(-1), r.reshape(-1), atol=1e-10 * np.abs(r).max())
        else:
            A = dec.lam[j].real * p.M + tau * p.K
            np.testing.assert_allclose(A @ x[0], r[0], atol=1e-10 * np.abs(r).max())


@pytest.mark.parametrize("Q", [2, 4])
@pytest.mark.parametrize("tau", [1e-3, 0.1])
def test_presb_spectrum_in_half_one(small, Q, tau):
    """For K' symmetric positive definite and M' symmetric positive
    semidefinite, the eigenvalues of P^-1 A (A the two-by-two block) are real
    and lie in [1/2, 1] (the PRESB bound of the method's cited analysis;
    checked here by a dense eigen-solve)."""
    p = small
    dec = ComplexBlocks(RadauIIA(Q))
    for j in range(dec.npair):
        A = pair_matrix(dec, p.M, p.K, tau, j).toarray()
        P = presb_matrix(dec, p.M, p.K, tau, j).toarray()
        ev = np.linalg.eigvals(np.linalg.solve(P, A))
        assert np.abs(ev.imag).max() < 1e-8
        assert ev.real.min() > 0.5 - 1e-10 and ev.real.max() < 1 + 1e-10


@pytest.mark.parametrize("Q", [2, 3, 4, 5])
def test_complex_step_matches_direct_step(Q):
    """The direct-diagonalisation step (per-block GMRES with PRESB and
    V-cycles) reaches the coupled system's solution."""
    n, k, tau = 4, 2, 0.02
    tab = RadauIIA(Q)
    cs = ComplexStepper(n, k, tab, tau)
    rng = np.random.default_rng(Q)
    nint = cs.M.shape[0]
    y = rng.standard_normal(nint)
    gbar = rng.standard_normal((Q, nint))
    y1, its = cs.step(y, gbar, rtol=1e-12)
    yd, _ = DirectStepper(cs.M, cs.K, tab, tau).step(y, gbar)
    np.testing.assert_allclose(y1, yd, atol=1e-10 * np.abs(yd).max())
    assert len(its) == (Q + 1) // 2 and all(0 < i < 40 for i in its)
