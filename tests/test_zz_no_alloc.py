"""rk_apply_operator_static (no context, no allocation: the mixed input sits in
the library's static device scratch) against rk_apply_operator on a context
with the same mesh, degree, Q and tau.  Both run the same kernels, so the
results must agree bitwise; two calls in a row, the second on a smaller mesh
(the scratch keeps the first call's contents), and the size limit."""
import pytest
import torch

from paper_2209_06700_amd import rk as R

pytestmark = pytest.mark.gpu

CASES = [  # (n_cells, degree, Q, tau): first call, then a smaller one
    ((6, 4, 3, 1e-3), (3, 2, 2, 0.05)),
    ((5, 3, 5, 2e-2), (2, 5, 4, 1e-3)),
]
FORMS = [R.RK_OP_CALA, R.RK_OP_STAGE, R.RK_OP_BLOCKS, R.RK_OP_K, R.RK_OP_M]


def _ref(n, k, Q, tau, form, u, prec):
    s = R.RadauIIA(n, k, Q, tau, precision=prec, restart=2, autotune=0, eig_max=[1.0] * R.n_levels(n))
    v = torch.empty_like(u)
    s.apply_operator(form, u, v)
    torch.cuda.synchronize()
    s.close()
    return v


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("pair", CASES)
def test_static_matches_context(pair, form, dtype):
    torch.manual_seed(7)
    prec = R.RK_PREC_FP64 if dtype == torch.float64 else R.RK_PREC_MIXED
    outs = []
    for n, k, Q, tau in pair:
        N = n * k + 1
        ns = 1 if form in (R.RK_OP_K, R.RK_OP_M) else Q
        u = torch.randn(ns * N ** 3, dtype=dtype, device="cuda")
        v = torch.full_like(u, float("nan"))
        R.rk_apply_operator_static(n, k, Q, tau, form, u, v)
        outs.append((u, v, (n, k, Q, tau)))
    torch.cuda.synchronize()
    for u, v, (n, k, Q, tau) in outs:
        want = _ref(n, k, Q, tau, form, u, prec)
        assert torch.equal(v, want), (n, k, Q, tau, form, (v - want).abs().max().item())


def test_static_on_a_side_stream_and_limit():
    n, k, Q, tau = 4, 4, 4, 5e-4
    N = n * k + 1
    u = torch.randn(Q * N ** 3, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        R.rk_apply_operator_static(n, k, Q, tau, R.RK_OP_CALA, u, v, stream=st)
    st.synchronize()
    assert torch.equal(v, _ref(n, k, Q, tau, R.RK_OP_CALA, u, R.RK_PREC_FP64))
    # Q N^3 fp64 values beyond the static scratch: rejected before any launch
    nb = 33  # N = 133, Q = 4: 75 MB > 64 MiB
    assert Q * (nb * k + 1) ** 3 * 8 > R.RK_STATIC_SCRATCH_BYTES
    big = torch.empty(Q * (nb * k + 1) ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RKError, match="static scratch"):
        R.rk_apply_operator_static(nb, k, Q, tau, R.RK_OP_CALA, big, torch.empty_like(big))
    # the forms without a stage mix need no scratch and take any size
    R.rk_apply_operator_static(nb, k, Q, tau, R.RK_OP_BLOCKS, big, torch.empty_like(big))
    torch.cuda.synchronize()
