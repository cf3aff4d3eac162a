"""GPU parity of the direct (complex) diagonalisation path of Sec. 6 against
the oracle: the eigen-data of A^-1 in real slot form (eq. irk:Ainv), the
two-by-two block operator (eq. complex:twobytwo), PRESB with V-cycles on
H = (Re lam + Im lam) M + tau K (eq. presb:p), and whole steps.

Bars: eigen-data 1e-12 relative (both sides round a 50-digit or long-double
computation to fp64); operators 1e-13 relative (fp64) / 1e-5 (fp32 input and
arithmetic); PRESB 1e-12 (fp64) and 1e-4 (mixed), as for the V-cycle it is
built from; steps 1e-10 relative L2 against the exact modal step from the
same y_n (the local error of each step) at rtol 1e-12.  The stopping test is per block and relative to the block's own
right-hand side in the slot basis, so at a given rtol the error of y is
larger than with the Crout method's global test (the oracle's per-block
GMRES at rtol 1e-10 ends 7e-10 from the exact step on the 8^3 Q_2 case, the
library 6.6e-10); rtol 1e-12 leaves room below the bar.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2209_06700_amd import rk
    return rk


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _opts(R, **kw):
    return R.rk_default_options(method=R.RK_METHOD_COMPLEX, **kw)


@pytest.mark.parametrize("Q", range(1, 10))
def test_complex_setup_matches_oracle(R, Q):
    from oracle.complex_irk import ComplexBlocks
    from oracle.tableau import RadauIIA
    dec = ComplexBlocks(RadauIIA(Q))
    ctx = R.rk_create(2, 1, Q, 0.1, _opts(R))
    try:
        info = R.rk_info(ctx)
    finally:
        R.rk_destroy(ctx)
    assert info["n_blocks"] == dec.nb and info["n_pairs"] == dec.npair
    np.testing.assert_allclose(np.array(info["clam"]), dec.lam, rtol=1e-12)
    T, U = np.array(info["T"]), np.array(info["U"])
    np.testing.assert_allclose(T @ U, np.eye(Q), atol=1e-12)
    # spectral projectors of the blocks do not depend on the eigenvector scaling
    for j in range(dec.nb):
        sl = list(dec.block_slots(j))
        want = dec.U[:, sl] @ dec.T[sl, :]
        np.testing.assert_allclose(U[:, sl] @ T[sl, :], want, atol=1e-12 * max(1.0, np.abs(want).max()))


@pytest.mark.parametrize("n,k,Q,tau", [(4, 2, 2, 0.03), (3, 3, 3, 0.01), (2, 4, 4, 0.2), (4, 1, 5, 0.05),
                                       (2, 6, 2, 0.002)])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_cblocks_operator_parity(R, n, k, Q, tau, dtype):
    from oracle.assemble import Problem
    from oracle.complex_irk import ComplexBlocks, block_operator
    from oracle.tableau import RadauIIA
    from paper_2209_06700_amd.synthetic import random_vector
    print(f"cblocks n={n} k={k} Q={Q} {dtype}", flush=True)
    p = Problem(n, k)
    dec = ComplexBlocks(RadauIIA(Q))
    N = n * k + 1
    u_np = random_vector((Q, N ** 3), seed=21 + Q, zero_boundary_N=N)
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    if dtype == "fp32":
        u_np = u_np.astype(np.float32).astype(np.float64)
    ctx = R.rk_create(n, k, Q, tau, _opts(R), eig_max=[1.0] * R.n_levels(n))
    try:
        u = torch.tensor(u_np, device="cuda", dtype=tdt)
        v = torch.full_like(u, float("nan"))
        R.rk_apply_operator(ctx, R.RK_OP_CBLOCKS, u, v)
        torch.cuda.synchronize()
        got = v.double().cpu().numpy().reshape(Q, -1)
    finally:
        R.rk_destroy(ctx)
    want = block_operator(dec, p.M, p.K, tau, np.stack([p.to_int(x) for x in u_np]))
    got_int = np.stack([p.to_int(x) for x in got])
    tol = 1e-13 if dtype == "fp64" else 1e-5
    assert np.abs(got_int - want).max() <= tol * np.abs(want).max()
    assert not np.stack([x[~p.mesh.interior_mask()] for x in got]).any()


def test_cblocks_similar_to_premultiplied_on_gpu(R):
    """(U (x) I) B u = A (U (x) I) u with both operators applied by the library."""
    from paper_2209_06700_amd.synthetic import random_vector
    n, k, Q, tau = 4, 3, 4, 0.02
    N = n * k + 1
    ctx = R.rk_create(n, k, Q, tau, _opts(R), eig_max=[1.0] * R.n_levels(n))
    try:
        U = torch.tensor(R.rk_info(ctx)["U"], dtype=torch.float64, device="cuda")
        u = torch.tensor(random_vector((Q, N ** 3), seed=2, zero_boundary_N=N), device="cuda")
        Bu = torch.empty_like(u)
        R.rk_apply_operator(ctx, R.RK_OP_CBLOCKS, u, Bu)
        Uu = (U @ u.view(Q, -1)).contiguous()
        AUu = torch.empty_like(Uu)
        R.rk_apply_operator(ctx, R.RK_OP_CALA, Uu, AUu)
        lhs = U @ Bu.view(Q, -1)
        torch.cuda.synchronize()
        assert float((lhs - AUu).abs().max()) <= 1e-12 * float(AUu.abs().max())
    finally:
        R.rk_destroy(ctx)


def _oracle_presb(n, k, Q, tau, deg, cdeg):
    from oracle.complex_irk import ComplexBlocks, Presb
    from oracle.multigrid import BlockMG, Hierarchy
    from oracle.tableau import RadauIIA
    dec = ComplexBlocks(RadauIIA(Q))
    hier = Hierarchy(n, k)
    mg = BlockMG(hier, dec.h_shift(), tau, degree=deg, coarse_degree=cdeg, cheb_range=15.0)
    pre = Presb(dec, hier.levels[0].M, lambda s, b: mg.vcycle_block(s, b))
    return dec, hier, mg, pre


# (n, k, Q, tau, smoother degree, coarse degree): odd and even Q (with and
# without a real block), single-level and multilevel hierarchies
PCASES = [(8, 2, 2, 0.05, 3, 3), (4, 3, 3, 0.01, 2, 4), (6, 2, 5, 0.02, 3, 3), (2, 4, 4, 0.003, 3, 2),
          (5, 2, 1, 0.05, 3, 3), (4, 4, 3, 0.01, 1, 2)]


@pytest.mark.parametrize("n,k,Q,tau,deg,cdeg", PCASES)
@pytest.mark.parametrize("mode", ["batched", "per_stage"])
def test_presb_parity_fp64(R, n, k, Q, tau, deg, cdeg, mode):
    from paper_2209_06700_amd.synthetic import random_vector
    print(f"presb fp64 n={n} k={k} Q={Q} {mode}", flush=True)
    dec, hier, mg, pre = _oracle_presb(n, k, Q, tau, deg, cdeg)
    fine = hier.levels[0]
    N = n * k + 1
    opts = _opts(R, cheb_degree=deg, coarse_cheb_degree=cdeg, cheb_range=15.0,
                 mode=R.RK_BATCHED if mode == "batched" else R.RK_PER_STAGE)
    ctx = R.rk_create(n, k, Q, tau, opts, eig_max=list(mg.eig_max))
    try:
        r_np = random_vector((Q, N ** 3), seed=31 + n, zero_boundary_N=N)
        r = torch.tensor(r_np, device="cuda")
        z = torch.full_like(r, float("nan"))
        R.rk_apply_preconditioner(ctx, r, z)
        torch.cuda.synchronize()
        got = z.cpu().numpy()
    finally:
        R.rk_destroy(ctx)
    want = np.stack([fine.to_full(x) for x in pre.apply(np.stack([fine.to_int(x) for x in r_np]))])
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-12 * scale, np.abs(got - want).max() / scale


@pytest.mark.parametrize("n,k,Q,tau", [(8, 2, 2, 0.05), (4, 4, 3, 0.01)])
def test_presb_mixed_precision(R, n, k, Q, tau):
    from paper_2209_06700_amd.synthetic import random_vector
    dec, hier, mg, pre = _oracle_presb(n, k, Q, tau, 3, 3)
    fine = hier.levels[0]
    N = n * k + 1
    ctx = R.rk_create(n, k, Q, tau, _opts(R, precision=R.RK_PREC_MIXED), eig_max=list(mg.eig_max))
    try:
        r_np = random_vector((Q, N ** 3), seed=41, zero_boundary_N=N)
        z = torch.empty(Q * N ** 3, dtype=torch.float64, device="cuda")
        R.rk_apply_preconditioner(ctx, torch.tensor(r_np, device="cuda").view(-1), z)
        torch.cuda.synchronize()
        got = z.cpu().numpy().reshape(Q, -1)
    finally:
        R.rk_destroy(ctx)
    want = np.stack([fine.to_full(x) for x in pre.apply(np.stack([fine.to_int(x) for x in r_np]))])
    assert np.abs(got - want).max() <= 1e-4 * np.abs(want).max()


PREC = {"fp64": 0, "mixed": 1}


@pytest.mark.parametrize("n,k,Q,tau,mode,prec", [
    (8, 2, 2, 0.05, "batched", "fp64"),
    (16, 2, 3, 0.01, "batched", "fp64"),
    (16, 2, 3, 0.01, "per_stage", "mixed"),
    (8, 4, 5, 0.002, "batched", "mixed"),
    (12, 3, 4, 0.005, "batched", "mixed"),
    (6, 3, 1, 0.1, "batched", "fp64"),
])
def test_complex_step_vs_modal_oracle(R, n, k, Q, tau, mode, prec):
    from oracle.assemble import Problem
    from oracle.step import ModalSolver
    from oracle.tableau import RadauIIA
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    print(f"complex step n={n} k={k} Q={Q} {mode} {prec}", flush=True)
    solver = R.RadauIIA(n, k, Q, tau, method=R.RK_METHOD_COMPLEX, precision=PREC[prec], rtol=1e-12,
                        mode=R.RK_BATCHED if mode == "batched" else R.RK_PER_STAGE)
    x1 = grid_coords(solver.info["nodes"], n)
    y0 = fourier_field(x1, seed=1)
    ms = ModalSolver(n, k)
    p = Problem(n, k, "kron")
    y = torch.tensor(y0, device="cuda")
    tab = RadauIIA(Q)
    for s in range(3):
        y_ref = ms.step(tab, tau, p.to_int(y.cpu().numpy()))
        stats = solver.step(s * tau, y)
        assert _rel(p.to_int(y.cpu().numpy()), y_ref) <= 1e-10
        nb = (Q + 1) // 2
        its = stats["block_iterations"]
        assert all(i > 0 for i in its[:nb]) and not any(its[nb:])
        assert stats["iterations"] == max(its[:nb])
        assert stats["rel_residual"] <= 1e-12
    solver.close()


def test_complex_step_q7_as_accurate_as_oracle(R):
    """Q = 7: the eigenvector basis of A^-1 has condition number ~2e3, and
    with the per-block stopping test the oracle's own complex step ends
    5e-9 from the exact step at rtol 1e-12 on this case.  Bar: three times
    the oracle's error on the same data."""
    from oracle.assemble import Problem
    from oracle.complex_irk import ComplexStepper
    from oracle.step import ModalSolver
    from oracle.tableau import RadauIIA
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    n, k, Q, tau = 4, 2, 7, 0.05
    solver = R.RadauIIA(n, k, Q, tau, method=R.RK_METHOD_COMPLEX, rtol=1e-12)
    y0 = fourier_field(grid_coords(solver.info["nodes"], n), seed=1)
    p = Problem(n, k, "kron")
    tab = RadauIIA(Q)
    exact = ModalSolver(n, k).step(tab, tau, p.to_int(y0))
    y_or, _ = ComplexStepper(n, k, tab, tau).step(p.to_int(y0), rtol=1e-12)
    err_or = _rel(y_or, exact)
    y = torch.tensor(y0, device="cuda")
    stats = solver.step(0.0, y)
    assert stats["rel_residual"] <= 1e-12
    assert _rel(p.to_int(y.cpu().numpy()), exact) <= 3 * err_or, err_or
    solver.close()


def test_complex_step_with_source_vs_direct(R):
    """g(t) = gamma(t) G with a seeded load vector, against the oracle's
    direct solve of the coupled stage system; block iteration counts close
    to the oracle's per-block GMRES with PRESB."""
    from oracle.assemble import Problem
    from oracle.complex_irk import ComplexStepper
    from oracle.step import DirectStepper
    from oracle.tableau import RadauIIA
    from paper_2209_06700_amd.synthetic import random_vector
    n, k, Q, tau = 4, 2, 4, 0.02
    N = n * k + 1
    p = Problem(n, k)
    tab = RadauIIA(Q)
    y0 = random_vector(N ** 3, seed=8, zero_boundary_N=N)
    G = random_vector(N ** 3, seed=9, zero_boundary_N=N)
    gam = [0.3 + 0.1 * i for i in range(Q)]
    cs = ComplexStepper(n, k, tab, tau)
    solver = R.RadauIIA(n, k, Q, tau, method=R.RK_METHOD_COMPLEX, rtol=1e-12, eig_max=list(cs.mg.eig_max))
    y = torch.tensor(y0, device="cuda")
    stats = solver.step(0.0, y, torch.tensor(G, device="cuda"), gam)
    gbar = np.array(gam)[:, None] * p.to_int(G)[None, :]
    want, _ = DirectStepper(p.M, p.K, tab, tau).step(p.to_int(y0), gbar)
    assert _rel(p.to_int(y.cpu().numpy()), want) < 1e-10
    _, its_ref = cs.step(p.to_int(y0), gbar, rtol=1e-12)
    got = stats["block_iterations"][:len(its_ref)]
    assert all(abs(a - b) <= 2 for a, b in zip(got, its_ref)), (got, its_ref)
    solver.close()


def test_complex_batched_equals_per_stage(R):
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    n, k, Q, tau = 8, 3, 5, 0.01
    outs = []
    for mode in (R.RK_BATCHED, R.RK_PER_STAGE):
        solver = R.RadauIIA(n, k, Q, tau, method=R.RK_METHOD_COMPLEX, mode=mode,
                            precision=R.RK_PREC_MIXED, eig_max=[2.0, 2.1, 2.2, 2.3])
        y = torch.tensor(fourier_field(grid_coords(solver.info["nodes"], n), seed=3), device="cuda")
        solver.step(0.0, y)
        torch.cuda.synchronize()
        outs.append(y.cpu())
        solver.close()
    assert torch.equal(outs[0], outs[1])


def test_complex_full_size_32cubed_q4(R):
    """32^3 cells, Q_4 (129^3 nodes), Q = 4, tau = 5e-4, mixed precision,
    batched, rtol 1e-11: two steps against the modal oracle."""
    from oracle.step import ModalSolver
    from oracle.tableau import RadauIIA
    from paper_2209_06700_amd.synthetic import fourier_field, grid_coords
    n, k, Q, tau = 32, 4, 4, 5e-4
    print("complex 32^3 Q_4 Q=4 mixed", flush=True)
    solver = R.RadauIIA(n, k, Q, tau, method=R.RK_METHOD_COMPLEX, precision=R.RK_PREC_MIXED, rtol=1e-11)
    y0 = fourier_field(grid_coords(solver.info["nodes"], n), seed=0)
    ms = ModalSolver(n, k)
    y = torch.tensor(y0, device="cuda")
    N = n * k + 1
    inner = np.zeros((N, N, N), dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    y_ref = y0.reshape(N, N, N)[inner]
    for s in range(2):
        solver.step(s * tau, y)
        y_ref = ms.step(RadauIIA(Q), tau, y_ref)
        got = y.cpu().numpy().reshape(N, N, N)[inner]
        assert _rel(got, y_ref) <= 1e-8
    solver.close()
