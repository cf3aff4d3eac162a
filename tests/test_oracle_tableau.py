"""Pins of the oracle's Radau IIA tableau and preconditioner factors.

Each test ties oracle/tableau.py to something other than itself: textbook
closed forms (Q = 1, 2, 3), order conditions, the Pade stability function,
and the statements of Sec. 2 of the paper about A_Q^-1 and its Crout factor.
"""
import math
import os

import numpy as np
import pytest

from oracle.tableau import RadauIIA, pade_exp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
QS = list(range(1, 10))


def _golden_q3():
    s6 = math.sqrt(6.0)
    vals = {}
    with open(os.path.join(GOLDEN, "radau_iia_q3.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, expr = line.split("=", 1)
            vals[name.strip()] = eval(expr, {"s6": s6})
    return vals


def test_q1_is_backward_euler_tableau():
    t = RadauIIA(1)
    assert t.A.tolist() == [[1.0]] and t.b.tolist() == [1.0] and t.c.tolist() == [1.0]


def test_q2_closed_form():
    t = RadauIIA(2)
    np.testing.assert_allclose(t.c, [1 / 3, 1.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(t.A, [[5 / 12, -1 / 12], [3 / 4, 1 / 4]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(t.b, [3 / 4, 1 / 4], rtol=0, atol=1e-15)


def test_q3_matches_textbook_table():
    g = _golden_q3()
    t = RadauIIA(3)
    np.testing.assert_allclose(t.c, [g["c1"], g["c2"], g["c3"]], rtol=0, atol=2e-15)
    A = [[g[f"a{i}{j}"] for j in (1, 2, 3)] for i in (1, 2, 3)]
    np.testing.assert_allclose(t.A, A, rtol=0, atol=2e-15)
    np.testing.assert_allclose(t.b, [g["b1"], g["b2"], g["b3"]], rtol=0, atol=2e-15)


@pytest.mark.parametrize("Q", QS)
def test_order_conditions(Q):
    """B(2Q-1): sum b_i c_i^(m-1) = 1/m; C(Q): sum_j a_ij c_j^(m-1) = c_i^m/m;
    c_Q = 1 and b equals the last row of A (stiffly accurate)."""
    t = RadauIIA(Q)
    for m in range(1, 2 * Q):
        assert abs(t.b @ t.c ** (m - 1) - 1.0 / m) < 1e-14
    for m in range(1, Q + 1):
        np.testing.assert_allclose(t.A @ t.c ** (m - 1), t.c ** m / m, rtol=0, atol=1e-14)
    assert t.c[-1] == 1.0
    np.testing.assert_allclose(t.A[-1], t.b, rtol=0, atol=1e-15)
    assert np.all(np.diff(t.c) > 0) and t.c[0] > 0


@pytest.mark.parametrize("Q", QS)
def test_stability_function_is_pade(Q):
    """R(z) = 1 + z b^T (I - zA)^-1 e equals the (Q-1, Q) Pade approximant of e^z."""
    t = RadauIIA(Q)
    zs = np.array([-0.01, -0.5, -3.0, -40.0, -1e4, 0.3 + 2j, -2.0 - 5j])
    R = t.stability(zs)
    P = np.array([pade_exp(Q - 1, Q, complex(z)) for z in zs])
    np.testing.assert_allclose(R, P, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("Q", QS)
def test_inverse_spectrum(Q):
    """Sec. 2: A_Q^-1 has floor(Q/2) complex-conjugate pairs and one real
    eigenvalue for odd Q; all lie in the right half-plane (A-stability)."""
    t = RadauIIA(Q)
    ev = np.linalg.eigvals(t.Ainv)
    ncomplex = int(np.sum(np.abs(ev.imag) > 1e-8))
    assert ncomplex == 2 * (Q // 2)
    assert int(np.sum(np.abs(ev.imag) <= 1e-8)) == Q % 2
    assert np.all(ev.real > 0)
    np.testing.assert_allclose(t.Ainv @ t.A, np.eye(Q), rtol=0, atol=1e-11)


@pytest.mark.parametrize("Q", QS)
def test_crout_factor_and_real_decomposition(Q):
    """Sec. 2: A_Q^-1 = L U with U unit-diagonal, so L^-1 A_Q^-1 is upper
    triangular with unit diagonal (all eigenvalues one); the spectral
    decomposition of L is real: L = S Lam S^-1 with real, distinct, positive
    Lam = diag(L)."""
    t = RadauIIA(Q)
    scale = np.abs(t.Ainv).max()
    assert np.allclose(np.triu(t.L, 1), 0.0)
    assert np.allclose(np.tril(t.U, -1), 0.0)
    np.testing.assert_allclose(np.diag(t.U), 1.0, rtol=0, atol=0)
    np.testing.assert_allclose(t.L @ t.U, t.Ainv, rtol=0, atol=1e-13 * scale)
    LiA = np.linalg.solve(t.L, t.Ainv)
    np.testing.assert_allclose(np.tril(LiA, -1), 0.0, atol=1e-10)
    np.testing.assert_allclose(np.diag(LiA), 1.0, atol=1e-10)
    lam = t.lam
    assert np.all(lam > 0)
    assert len(set(np.round(lam, 10))) == Q
    np.testing.assert_allclose(lam, np.diag(t.L), rtol=0, atol=0)
    rec = t.S @ np.diag(lam) @ t.Sinv
    cond = np.linalg.cond(t.S)
    np.testing.assert_allclose(rec, t.L, rtol=0, atol=1e-14 * cond * scale)
    np.testing.assert_allclose(t.S @ t.Sinv, np.eye(Q), rtol=0, atol=1e-13 * cond)


def test_q2_crout_by_hand():
    """Q = 2 by hand: A^-1 = [[3/2, 1/2], [-9/2, 5/2]]; Crout gives
    L = [[3/2, 0], [-9/2, 4]], U = [[1, 1/3], [0, 1]]; eigenvectors of L with
    unit diagonal: S = [[1, 0], [9/5, 1]]."""
    t = RadauIIA(2)
    np.testing.assert_allclose(t.Ainv, [[1.5, 0.5], [-4.5, 2.5]], atol=1e-14)
    np.testing.assert_allclose(t.L, [[1.5, 0.0], [-4.5, 4.0]], atol=1e-14)
    np.testing.assert_allclose(t.U, [[1.0, 1 / 3], [0.0, 1.0]], atol=1e-14)
    np.testing.assert_allclose(t.S, [[1.0, 0.0], [1.8, 1.0]], atol=1e-14)
    np.testing.assert_allclose(t.lam, [1.5, 4.0], atol=1e-14)
