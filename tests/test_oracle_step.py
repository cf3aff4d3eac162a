"""Pins of the oracle's Radau IIA step (Sec. 2): backward Euler at Q = 1,
the Pade stability function on an exact eigenmode, order 2Q-1 in time
against the semi-discrete exact solution, agreement of the direct and modal
solvers, and the manufactured solution of the 8^3 Q_2 workload."""
import numpy as np
import pytest

from oracle.assemble import Problem, interpolate, load_separable
from oracle.step import (DirectStepper, ModalSolver, backward_euler, premultiplied_operator,
                         premultiplied_rhs, stage_matrix, stage_rhs)
from oracle.tableau import RadauIIA, pade_exp


def _sines(p, mx, my, mz):
    return p.to_int(interpolate(p.mesh, lambda x, y, z: np.sin(mx * np.pi * x)
                                * np.sin(my * np.pi * y) * np.sin(mz * np.pi * z)))


@pytest.mark.parametrize("n,k", [(3, 1), (2, 2)])
def test_q1_is_backward_euler(n, k):
    p = Problem(n, k)
    tab = RadauIIA(1)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(p.M.shape[0])
    g = rng.standard_normal(p.M.shape[0])
    tau = 0.07
    y1, _ = DirectStepper(p.M, p.K, tab, tau).step(y, g[None, :])
    yb = backward_euler(p.M, p.K, tau, y, g)
    np.testing.assert_allclose(y1, yb, rtol=0, atol=1e-12 * np.abs(yb).max())


@pytest.mark.parametrize("Q", [1, 2, 3, 4, 5])
def test_eigenmode_step_is_pade(Q):
    """Q_1 sine mode s with K s = lam M s (closed-form lam), g = 0:
    y_1 = R(-tau lam) s with R the (Q-1, Q) Pade approximant of exp."""
    n = 4
    p = Problem(n, 1)
    h = 1.0 / n
    s = _sines(p, 1, 2, 3)
    lam = sum(6 / h ** 2 * (1 - np.cos(m * np.pi * h)) / (2 + np.cos(m * np.pi * h)) for m in (1, 2, 3))
    tab = RadauIIA(Q)
    for tau in (0.003, 0.05, 1.0):
        y1, _ = DirectStepper(p.M, p.K, tab, tau).step(s)
        R = pade_exp(Q - 1, Q, -tau * lam)
        np.testing.assert_allclose(y1, R * s, rtol=0, atol=1e-12 * np.abs(s).max())


@pytest.mark.parametrize("Q", [1, 2, 3, 4])
def test_premultiplied_form_same_stages(Q):
    """Eq. (irk:A) is eq. (stage system) multiplied by A^-1 (x) I: both give
    the same k."""
    p = Problem(2, 2)
    tab = RadauIIA(Q)
    rng = np.random.default_rng(Q)
    y = rng.standard_normal(p.M.shape[0])
    gbar = rng.standard_normal((Q, p.M.shape[0]))
    tau = 0.1
    _, k = DirectStepper(p.M, p.K, tab, tau).step(y, gbar)
    A = premultiplied_operator(p.M, p.K, tab.Ainv, tau)
    b = premultiplied_rhs(p.K, tab.Ainv, y, gbar).reshape(-1)
    np.testing.assert_allclose(A @ k.reshape(-1), b, rtol=0, atol=1e-11 * np.abs(b).max())
    S = stage_matrix(p.M, p.K, tab.A, tau)
    np.testing.assert_allclose(S @ k.reshape(-1), stage_rhs(p.K, y, gbar).reshape(-1),
                               atol=1e-11 * np.abs(gbar).max())


@pytest.mark.parametrize("n,k,Q", [(3, 2, 2), (2, 3, 3), (4, 1, 5)])
def test_modal_equals_direct(n, k, Q):
    p = Problem(n, k)
    tab = RadauIIA(Q)
    tau = 0.02
    rng = np.random.default_rng(7)
    y = rng.standard_normal(p.M.shape[0])
    gbar = rng.standard_normal((Q, p.M.shape[0]))
    yd, _ = DirectStepper(p.M, p.K, tab, tau).step(y, gbar)
    ym = ModalSolver(n, k).step(tab, tau, y, gbar)
    assert np.linalg.norm(ym - yd) / np.linalg.norm(yd) < 1e-12


@pytest.mark.parametrize("Q", [1, 2, 3])
def test_order_in_time(Q):
    """Against the semi-discrete exact solution of M y' + K y = e^{-t} G
    (per eigenmode: yhat e^{-lam t} + ghat (e^{-t} - e^{-lam t})/(lam - 1)),
    the error of n steps decays as tau^(2Q-1) (Sec. 2: order 2Q-1)."""
    n, k = 4, 2
    ms = ModalSolver(n, k)
    p = Problem(n, k)
    G = p.to_int(load_separable(p.mesh, lambda x: np.sin(np.pi * x)))
    y0 = _sines(p, 1, 2, 1)
    yh0, gh, lam = ms.to_modal(y0), ms.load_to_modal(G), ms.lam
    T = 1.0
    ye = ms.from_modal(yh0 * np.exp(-lam * T) + gh * (np.exp(-T) - np.exp(-lam * T)) / (lam - 1))
    tab = RadauIIA(Q)
    errs = []
    for nsteps in (8, 16, 32):
        tau = T / nsteps
        y, t = y0.copy(), 0.0
        for _ in range(nsteps):
            y = ms.step(tab, tau, y, np.exp(-(t + tab.c * tau))[:, None] * G[None, :])
            t += tau
        errs.append(np.linalg.norm(y - ye) / np.linalg.norm(ye))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2 * Q - 1 - 0.35), rates


def test_manufactured_8cubed_q2():
    """The 8^3 Q_2, Q = 2, tau = 0.05, 10-step workload: u = prod sin(pi x_d) e^-t,
    f = (3 pi^2 - 1) u.  The nodal error at t = 0.5 is small and drops with h."""
    tab = RadauIIA(2)
    errs = []
    for n in (4, 8):
        p = Problem(n, 2)
        G = p.to_int(load_separable(p.mesh, lambda x: np.sin(np.pi * x)))
        u = lambda t: p.to_int(interpolate(p.mesh, lambda x, y, z: np.sin(np.pi * x)
                                           * np.sin(np.pi * y) * np.sin(np.pi * z) * np.exp(-t)))
        st = DirectStepper(p.M, p.K, tab, 0.05)
        y, t = u(0.0), 0.0
        for _ in range(10):
            y, _ = st.step(y, (3 * np.pi ** 2 - 1) * np.exp(-(t + tab.c * 0.05))[:, None] * G[None, :])
            t += 0.05
        errs.append(np.linalg.norm(y - u(t)) / np.linalg.norm(u(t)))
    assert errs[1] < 1e-4 and errs[0] / errs[1] > 6, errs
