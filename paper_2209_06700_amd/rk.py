"""Python binding of the stage-parallel Radau IIA library (same names as the C ABI).

All arithmetic runs in the HIP library; these functions check shapes and
dtypes of torch CUDA tensors and pass raw device pointers.  Vectors are
contiguous tensors holding the full N^3 grid (x fastest), Q-stage vectors
have shape (Q, N, N, N) or (Q * N^3,).  See include/rk.h for the contract.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (LIB, RK_BATCHED, RK_ENOCONV, RK_FP32, RK_FP64, RK_METHOD_COMPLEX, RK_METHOD_CROUT, RK_OK,
                   RK_OP_BLOCKS, RK_OP_CALA, RK_OP_CBLOCKS, RK_MAX_Q, RK_OP_K, RK_OP_M, RK_OP_STAGE,
                   RK_PER_STAGE, RK_PREC_FP64, RK_PREC_MIXED, RK_STATIC_SCRATCH_BYTES, rk_info_t, rk_mesh,
                   rk_options, rk_stats)

__all__ = ["RKError", "rk_default_options", "rk_workspace_bytes", "rk_create", "rk_destroy", "rk_info",
           "rk_apply_operator_batch",
           "rk_step", "rk_step_batch", "rk_apply_operator", "rk_vcycle", "rk_apply_preconditioner",
           "rk_last_error", "rk_deformed_geometry_bytes", "rk_deformed_geometry", "rk_deformed_apply",
           "rk_apply_operator_static", "RK_STATIC_SCRATCH_BYTES", "DeformedOperator",
           "RadauIIA", "RK_FP64", "RK_FP32", "RK_PREC_FP64", "RK_PREC_MIXED", "RK_BATCHED",
           "RK_PER_STAGE", "RK_OP_CALA", "RK_OP_STAGE", "RK_OP_BLOCKS", "RK_OP_K", "RK_OP_M",
           "RK_OP_CBLOCKS", "RK_METHOD_CROUT", "RK_METHOD_COMPLEX"]


class RKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rk error {code}: {msg}")
        self.code = code


@dataclass
class Context:
    handle: C.c_void_p
    workspace: torch.Tensor
    N: int
    Q: int
    precision: int
    stream: torch.cuda.Stream | None
    _eig: object = None     # keeps an eig_max array alive during create


def rk_last_error(ctx: Context | None = None) -> str:
    msg = LIB.rk_last_error(ctx.handle if ctx is not None else None)
    return msg.decode() if msg else ""


def _check(rc: int, ctx: Context | None = None):
    if rc != RK_OK:
        raise RKError(rc, rk_last_error(ctx))


def rk_default_options(**kw) -> rk_options:
    """Options struct with the library defaults, overridden by keywords
    (precision, mode, rtol, max_iter, restart, cheb_degree, coarse_cheb_degree,
    cheb_range, eig_safety, eig_iterations, timing, method, deform, autotune,
    deform_mg, vc_streams, z_chunk, tile_shape, tail_nodes; eig_max is set by
    rk_create)."""
    o = rk_options()
    LIB.rk_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "eig_max":
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def rk_workspace_bytes(n_cells: int, degree: int, Q: int, opts: rk_options | None = None,
                       length: float = 1.0) -> int:
    mesh = rk_mesh(n_cells, length)
    out = C.c_size_t(0)
    _check(LIB.rk_workspace_bytes(C.byref(mesh), degree, Q, C.byref(opts) if opts else None, C.byref(out)))
    return out.value


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return RK_FP64
    if t.dtype == torch.float32:
        return RK_FP32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _vec(t: torch.Tensor, numel: int, name: str, dtype=None) -> C.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return C.c_void_p(t.data_ptr())


def n_levels(n_cells: int) -> int:
    """Number of multigrid levels: n_cells is halved while it is even."""
    count, m = 1, int(n_cells)
    while m % 2 == 0 and count < _lib.RK_MAX_LEVELS:
        m //= 2
        count += 1
    return count


def rk_create(n_cells: int, degree: int, Q: int, tau: float, opts: rk_options | None = None,
              eig_max=None, device: str | torch.device = "cuda",
              stream: torch.cuda.Stream | None = None, length: float = 1.0) -> Context:
    """Allocate the workspace (torch) and create a context on `stream`
    (default: the current stream of `device`) for the cube [0, length]^3."""
    opts = opts if opts is not None else rk_default_options()
    eig_arr = None
    if eig_max is not None:
        vals = [float(v) for v in eig_max]
        if len(vals) != n_levels(n_cells):
            raise ValueError(f"eig_max needs {n_levels(n_cells)} values (one per level)")
        eig_arr = (C.c_double * len(vals))(*vals)
        opts.eig_max = C.cast(eig_arr, C.POINTER(C.c_double))
    nbytes = rk_workspace_bytes(n_cells, degree, Q, opts, length)
    dev = torch.device(device)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    # The workspace is used on the context stream only: allocate it there, so
    # that the caching allocator orders its reuse after that stream's work.
    with torch.cuda.stream(st):
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    mesh = rk_mesh(n_cells, length)
    h = C.c_void_p()
    rc = LIB.rk_create(C.byref(mesh), degree, Q, float(tau), C.byref(opts), C.c_void_p(ws.data_ptr()),
                       nbytes, C.c_void_p(st.cuda_stream), C.byref(h))
    opts.eig_max = None
    _check(rc)
    return Context(h, ws, n_cells * degree + 1, Q, opts.precision, st, eig_arr)


def rk_destroy(ctx: Context):
    if ctx.handle:
        LIB.rk_destroy(ctx.handle)
        ctx.handle = C.c_void_p()


def rk_info(ctx: Context) -> dict:
    i = rk_info_t()
    _check(LIB.rk_info(ctx.handle, C.byref(i)), ctx)
    Q, nl = i.Q, i.n_levels
    mat = lambda a: [[a[r * Q + c] for c in range(Q)] for r in range(Q)]
    return dict(N=i.N, n_cells=i.n_cells, degree=i.degree, Q=Q, n_levels=nl,
                level_cells=list(i.level_cells[:nl]), tau=i.tau, h=i.h,
                A=mat(i.A), b=list(i.b[:Q]), c=list(i.c[:Q]), Ainv=mat(i.Ainv), L=mat(i.L),
                S=mat(i.S), Sinv=mat(i.Sinv), lam=list(i.lambda_[:Q]),
                eig_max=list(i.eig_max[:nl]), nodes=list(i.nodes[:i.degree + 1]),
                n_blocks=i.n_blocks, n_pairs=i.n_pairs,
                clam=[complex(i.clam_re[j], i.clam_im[j]) for j in range(i.n_blocks)],
                T=mat(i.T), U=mat(i.U), level_cz=list(i.level_cz[:nl]), krylov_cz=i.krylov_cz,
                level_ts=list(i.level_ts[:nl]), level_cz_store=list(i.level_cz_store[:nl]),
                level_ts_store=list(i.level_ts_store[:nl]), tail_level=i.tail_level)


def rk_step(ctx: Context, t_n: float, y: torch.Tensor, G: torch.Tensor | None = None,
            gamma=None, raise_on_noconv: bool = True) -> dict:
    """One Radau IIA step in place on y (fp64, N^3).  g(t) = gamma(t) G with
    gamma given at the Q stage times t_n + c_i tau.  Returns the stats."""
    N3 = ctx.N ** 3
    yp = _vec(y, N3, "y", torch.float64)
    gp = None
    garr = None
    if G is not None:
        gp = _vec(G, N3, "G", torch.float64)
        if gamma is None or len(gamma) != ctx.Q:
            raise ValueError("gamma must hold Q values")
        garr = (C.c_double * ctx.Q)(*[float(g) for g in gamma])
    st = rk_stats()
    rc = LIB.rk_step(ctx.handle, float(t_n), yp, gp, garr, C.byref(st))
    if rc != RK_OK and not (rc == RK_ENOCONV and not raise_on_noconv):
        raise RKError(rc, rk_last_error(ctx))
    return _stats_dict(rc, st)


def _stats_dict(rc, st):
    return dict(code=rc, iterations=st.iterations, vcycles=st.vcycles, rel_residual=st.rel_residual,
                t_rhs=st.t_rhs, t_vmult=st.t_vmult, t_basis=st.t_basis, t_blocks=st.t_blocks,
                t_rest=st.t_rest, block_iterations=list(st.block_iterations))


def rk_step_batch(ctxs, t_n, ys, Gs=None, gammas=None, threads: int = 0, raise_on_error: bool = True):
    """One step of each context (rk_step_batch): ctxs, t_n, ys (fp64 N_i^3
    tensors) and optionally Gs / gammas are sequences of equal length.
    Returns the per-entry stats dicts (with the entry's code)."""
    m = len(ctxs)
    if not (len(t_n) == len(ys) == m) or (Gs is not None and len(Gs) != m):
        raise ValueError("batch sequences must have equal lengths")
    handles = (C.c_void_p * m)(*[c.handle for c in ctxs])
    tarr = (C.c_double * m)(*[float(t) for t in t_n])
    yarr = (C.c_void_p * m)(*[_vec(y, c.N ** 3, "y", torch.float64) for c, y in zip(ctxs, ys)])
    garr = None
    gam = (C.c_double * (m * RK_MAX_Q))()
    if Gs is not None:
        garr = (C.c_void_p * m)(*[None if G is None else _vec(G, c.N ** 3, "G", torch.float64)
                                  for c, G in zip(ctxs, Gs)])
        for i, (c, G) in enumerate(zip(ctxs, Gs)):
            if G is not None:
                if gammas is None or gammas[i] is None or len(gammas[i]) != c.Q:
                    raise ValueError(f"entry {i}: gamma must hold Q values")
                for q, g in enumerate(gammas[i]):
                    gam[i * RK_MAX_Q + q] = float(g)
    st = (rk_stats * m)()
    codes = (C.c_int * m)()
    rc = LIB.rk_step_batch(handles, m, tarr, yarr, garr, gam, st, codes, int(threads))
    out = [_stats_dict(codes[i], st[i]) for i in range(m)]
    if rc != RK_OK and raise_on_error:
        bad = next(i for i in range(m) if codes[i] != RK_OK)
        raise RKError(rc, f"entry {bad}: {rk_last_error(ctxs[bad])}")
    return out


def rk_apply_operator(ctx: Context, form: int, u: torch.Tensor, v: torch.Tensor):
    ns = 1 if form in (RK_OP_K, RK_OP_M) else ctx.Q
    n = ns * ctx.N ** 3
    up = _vec(u, n, "u")
    vp = _vec(v, n, "v", u.dtype)
    _check(LIB.rk_apply_operator(ctx.handle, int(form), _dtype_code(u), up, vp), ctx)


def rk_apply_operator_batch(ctxs, form: int, us, vs, stream: torch.cuda.Stream | None = None):
    """v_i = op_i(u_i) for several contexts in work-list launches
    (rk_apply_operator_batch; forms RK_OP_BLOCKS, RK_OP_K, RK_OP_M), on
    `stream` (default: the current stream)."""
    m = len(ctxs)
    if not (len(us) == len(vs) == m) or m == 0:
        raise ValueError("batch sequences must have one or more entries of equal length")
    dt = us[0].dtype
    sizes = [(1 if form in (RK_OP_K, RK_OP_M) else c.Q) * c.N ** 3 for c in ctxs]
    handles = (C.c_void_p * m)(*[c.handle for c in ctxs])
    uarr = (C.c_void_p * m)(*[_vec(u, n, "u", dt) for u, n in zip(us, sizes)])
    varr = (C.c_void_p * m)(*[_vec(v, n, "v", dt) for v, n in zip(vs, sizes)])
    st = stream if stream is not None else torch.cuda.current_stream(us[0].device)
    _check(LIB.rk_apply_operator_batch(handles, m, int(form), _dtype_code(us[0]), uarr, varr,
                                       C.c_void_p(st.cuda_stream)))


def rk_vcycle(ctx: Context, b: torch.Tensor, x: torch.Tensor):
    n = ctx.Q * ctx.N ** 3
    bp = _vec(b, n, "b")
    xp = _vec(x, n, "x", b.dtype)
    _check(LIB.rk_vcycle(ctx.handle, _dtype_code(b), bp, xp), ctx)


def rk_apply_preconditioner(ctx: Context, r: torch.Tensor, z: torch.Tensor):
    n = ctx.Q * ctx.N ** 3
    _check(LIB.rk_apply_preconditioner(ctx.handle, _vec(r, n, "r", torch.float64),
                                       _vec(z, n, "z", torch.float64)), ctx)


def _dtype_from_torch(dtype) -> int:
    if dtype == torch.float64:
        return RK_FP64
    if dtype == torch.float32:
        return RK_FP32
    raise TypeError(f"unsupported dtype {dtype}")


def rk_deformed_geometry_bytes(n_cells: int, degree: int, dtype=torch.float64) -> int:
    out = C.c_size_t(0)
    _check(LIB.rk_deformed_geometry_bytes(C.byref(rk_mesh(n_cells)), degree, _dtype_from_torch(dtype),
                                          C.byref(out)))
    return out.value


def rk_deformed_geometry(n_cells: int, degree: int, eps: float, geometry: torch.Tensor,
                         stream: torch.cuda.Stream | None = None):
    """Fill `geometry` (a CUDA tensor of the operator dtype and
    rk_deformed_geometry_bytes bytes) for the map with amplitude eps."""
    nbytes = rk_deformed_geometry_bytes(n_cells, degree, geometry.dtype)
    if not geometry.is_cuda or not geometry.is_contiguous() or geometry.numel() * geometry.element_size() != nbytes:
        raise ValueError(f"geometry must be a contiguous CUDA tensor of {nbytes} bytes")
    st = stream if stream is not None else torch.cuda.current_stream(geometry.device)
    _check(LIB.rk_deformed_geometry(C.byref(rk_mesh(n_cells)), degree, float(eps),
                                    _dtype_from_torch(geometry.dtype), C.c_void_p(geometry.data_ptr()),
                                    C.c_void_p(st.cuda_stream)))


def rk_deformed_apply(n_cells: int, degree: int, alpha, beta, geometry: torch.Tensor, u: torch.Tensor,
                      v: torch.Tensor, stream: torch.cuda.Stream | None = None):
    """v_s = alpha[s] M u_s + beta[s] K u_s on the deformed mesh, Q = len(alpha)
    stages of N^3 entries each; u, v, geometry of one dtype."""
    Q = len(alpha)
    if len(beta) != Q:
        raise ValueError("alpha and beta need the same length")
    N = n_cells * degree + 1
    up = _vec(u, Q * N ** 3, "u")
    vp = _vec(v, Q * N ** 3, "v", u.dtype)
    if geometry.dtype != u.dtype or not geometry.is_cuda:
        raise TypeError("geometry must be a CUDA tensor of the vectors' dtype")
    st = stream if stream is not None else torch.cuda.current_stream(u.device)
    a = (C.c_double * Q)(*[float(x) for x in alpha])
    b = (C.c_double * Q)(*[float(x) for x in beta])
    _check(LIB.rk_deformed_apply(C.byref(rk_mesh(n_cells)), degree, Q, a, b, _dtype_code(u),
                                 C.c_void_p(geometry.data_ptr()), up, vp, C.c_void_p(st.cuda_stream)))


def rk_apply_operator_static(n_cells: int, degree: int, Q: int, tau: float, form: int, u: torch.Tensor,
                             v: torch.Tensor, stream: torch.cuda.Stream | None = None, length: float = 1.0):
    """v = op(u) without a context or any allocation (the library's static
    scratch holds the mixed input of RK_OP_CALA / RK_OP_STAGE)."""
    ns = 1 if form in (RK_OP_K, RK_OP_M) else Q
    n = ns * (n_cells * degree + 1) ** 3
    up = _vec(u, n, "u")
    vp = _vec(v, n, "v", u.dtype)
    st = stream if stream is not None else torch.cuda.current_stream(u.device)
    _check(LIB.rk_apply_operator_static(C.byref(rk_mesh(n_cells, length)), degree, Q, float(tau), int(form),
                                        _dtype_code(u), up, vp, C.c_void_p(st.cuda_stream)))


class DeformedOperator:
    """The deformed-mesh operator with its geometry array (torch-allocated)."""

    def __init__(self, n_cells, degree, eps, dtype=torch.float64, device="cuda", stream=None):
        self.n, self.k, self.eps, self.dtype = n_cells, degree, eps, dtype
        self.N = n_cells * degree + 1
        nbytes = rk_deformed_geometry_bytes(n_cells, degree, dtype)
        esize = torch.tensor([], dtype=dtype).element_size()
        self.geometry = torch.empty(nbytes // esize, dtype=dtype, device=device)
        self.stream = stream
        rk_deformed_geometry(n_cells, degree, eps, self.geometry, stream)

    def apply(self, u, v, alpha, beta):
        rk_deformed_apply(self.n, self.k, alpha, beta, self.geometry, u, v, self.stream)


class RadauIIA:
    """Owner of one context: ``RadauIIA(n_cells, degree, Q, tau, **options)``."""

    def __init__(self, n_cells, degree, Q, tau, eig_max=None, device="cuda", stream=None, length=1.0,
                 **options):
        self.opts = rk_default_options(**options)
        self.ctx = rk_create(n_cells, degree, Q, tau, self.opts, eig_max=eig_max, device=device,
                             stream=stream, length=length)
        self.info = rk_info(self.ctx)
        self.N, self.Q = self.ctx.N, Q

    def step(self, t_n, y, G=None, gamma=None, **kw):
        return rk_step(self.ctx, t_n, y, G, gamma, **kw)

    def apply_operator(self, form, u, v):
        rk_apply_operator(self.ctx, form, u, v)

    def vcycle(self, b, x):
        rk_vcycle(self.ctx, b, x)

    def apply_preconditioner(self, r, z):
        rk_apply_preconditioner(self.ctx, r, z)

    def close(self):
        rk_destroy(self.ctx)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
