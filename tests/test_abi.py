"""The C-ABI library loads, exports every entry point declared in
include/rk.h, and its host-only calls (options, workspace sizing, argument
validation) behave as documented.  No GPU is touched here."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rk_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_api():
    names = _declared()
    for n in ["rk_create", "rk_step", "rk_apply_operator", "rk_vcycle", "rk_workspace_bytes",
              "rk_destroy", "rk_info", "rk_last_error", "rk_default_options", "rk_apply_preconditioner"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2209_06700_amd import _lib
    lib = C.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == _declared()


def test_default_options():
    from paper_2209_06700_amd import rk as R
    o = R.rk_default_options()
    assert (o.precision, o.mode, o.rtol, o.restart, o.cheb_degree, o.cheb_range) == (0, 0, 1e-10, 30, 3, 15.0)
    o = R.rk_default_options(precision=R.RK_PREC_MIXED, restart=12)
    assert o.precision == 1 and o.restart == 12
    with pytest.raises(TypeError):
        R.rk_default_options(bogus=1)


def test_default_method_and_bad_method():
    from paper_2209_06700_amd import rk as R
    assert R.rk_default_options().method == R.RK_METHOD_CROUT
    assert R.rk_default_options().autotune == 1 and R.rk_default_options().deform == 0.0
    for kw in (dict(autotune=2), dict(deform=0.2)):
        with pytest.raises(R.RKError):
            R.rk_workspace_bytes(4, 2, 2, R.rk_default_options(**kw))
    with pytest.raises(R.RKError):
        R.rk_workspace_bytes(4, 2, 2, R.rk_default_options(method=7))
    assert R.rk_workspace_bytes(4, 2, 3, R.rk_default_options(method=R.RK_METHOD_COMPLEX)) > 0


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layout_matches_header(tmp_path):
    """sizeof and every field offset of the ABI structs, as a C compiler lays
    them out from include/rk.h, equal the ctypes mirrors in the binding."""
    from paper_2209_06700_amd import _lib
    structs = {"rk_options": _lib.rk_options, "rk_stats": _lib.rk_stats, "rk_info_t": _lib.rk_info_t}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rk.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            cf = "lambda" if f == "lambda_" else f
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {cf}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        name, field, val = line.split()
        cls = structs[name]
        want = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(val) == want, line


def test_workspace_bytes_scale_with_problem():
    from paper_2209_06700_amd import rk as R
    a = R.rk_workspace_bytes(8, 2, 2)
    b = R.rk_workspace_bytes(16, 2, 2)
    c = R.rk_workspace_bytes(8, 2, 4)
    assert 0 < a < b and a < c
    mixed = R.rk_workspace_bytes(32, 4, 3, R.rk_default_options(precision=R.RK_PREC_MIXED))
    fp64 = R.rk_workspace_bytes(32, 4, 3)
    assert mixed < fp64
    # at least the Krylov bases: (2 restart + 1) fp64 vectors of Q N^3
    N = 32 * 4 + 1
    assert fp64 > (2 * 30 + 1) * 3 * N ** 3 * 8


@pytest.mark.parametrize("args", [(0, 2, 2), (4, 0, 2), (4, 7, 2), (4, 2, 0), (4, 2, 10)])
def test_invalid_sizes_rejected(args):
    from paper_2209_06700_amd import rk as R
    with pytest.raises(R.RKError) as e:
        R.rk_workspace_bytes(*args)
    assert e.value.code == R._lib.RK_EINVAL


def test_invalid_options_rejected():
    from paper_2209_06700_amd import rk as R
    for kw in [dict(precision=5), dict(mode=3), dict(rtol=0.0), dict(restart=0), dict(cheb_degree=0),
               dict(cheb_range=1.0)]:
        with pytest.raises(R.RKError):
            R.rk_workspace_bytes(4, 2, 2, R.rk_default_options(**kw))


def test_create_rejects_missing_workspace_without_touching_the_gpu():
    from paper_2209_06700_amd import _lib
    lib = _lib.LIB
    mesh = _lib.rk_mesh(4)
    out = C.c_void_p()
    rc = lib.rk_create(C.byref(mesh), 2, 2, 0.1, None, None, 0, None, C.byref(out))
    assert rc == _lib.RK_EWORKSPACE and not out.value
    assert b"workspace" in lib.rk_last_error(None)
    rc = lib.rk_create(C.byref(mesh), 2, 2, -1.0, None, None, 0, None, C.byref(out))
    assert rc == _lib.RK_EINVAL


def test_step_batch_argument_checks_without_the_gpu():
    """rk_step_batch validates its arguments before any context is touched:
    an empty batch succeeds, NULL entries are rejected."""
    from paper_2209_06700_amd import _lib
    L = _lib.LIB
    assert L.rk_step_batch(None, 0, None, None, None, None, None, None, 0) == _lib.RK_OK
    ctx = (C.c_void_p * 1)(None)
    t = (C.c_double * 1)(0.0)
    y = (C.c_void_p * 1)(None)
    assert L.rk_step_batch(ctx, 1, t, y, None, None, None, None, 1) == _lib.RK_EINVAL
    assert L.rk_step_batch(ctx, -1, t, y, None, None, None, None, 1) == _lib.RK_EINVAL


def test_operator_batch_argument_checks_without_the_gpu():
    """rk_apply_operator_batch rejects empty or NULL batches, NULL entries,
    dense forms and bad dtypes before any context or vector is touched."""
    from paper_2209_06700_amd import _lib
    L = _lib.LIB
    ctx = (C.c_void_p * 1)(None)
    u = (C.c_void_p * 1)(None)
    v = (C.c_void_p * 1)(None)
    assert L.rk_apply_operator_batch(ctx, 0, _lib.RK_OP_BLOCKS, _lib.RK_FP32, u, v, None) == _lib.RK_EINVAL
    assert L.rk_apply_operator_batch(None, 1, _lib.RK_OP_BLOCKS, _lib.RK_FP32, u, v, None) == _lib.RK_EINVAL
    assert L.rk_apply_operator_batch(ctx, 1, _lib.RK_OP_BLOCKS, _lib.RK_FP32, u, v, None) == _lib.RK_EINVAL
    assert b"NULL context" in L.rk_last_error(None)
    for form in (_lib.RK_OP_CALA, _lib.RK_OP_STAGE, _lib.RK_OP_CBLOCKS, 6):
        assert L.rk_apply_operator_batch(ctx, 1, form, _lib.RK_FP32, u, v, None) == _lib.RK_EINVAL
    assert L.rk_apply_operator_batch(ctx, 1, _lib.RK_OP_K, 7, u, v, None) == _lib.RK_EINVAL


def test_mesh_length_checked_without_the_gpu():
    """rk_mesh.length must be finite and > 0, and 1 for deformed meshes."""
    from paper_2209_06700_amd import _lib
    from paper_2209_06700_amd import rk as R
    lib = _lib.LIB
    out = C.c_size_t(0)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        assert lib.rk_workspace_bytes(C.byref(_lib.rk_mesh(4, bad)), 2, 2, None, C.byref(out)) == _lib.RK_EINVAL
    assert lib.rk_workspace_bytes(C.byref(_lib.rk_mesh(4, 3.0)), 2, 2, None, C.byref(out)) == 0 and out.value > 0
    opts = R.rk_default_options(deform=0.05)
    assert lib.rk_workspace_bytes(C.byref(_lib.rk_mesh(4, 2.0)), 2, 2, C.byref(opts), C.byref(out)) == _lib.RK_EINVAL
    assert b"unit cube" in lib.rk_last_error(None)
    assert lib.rk_deformed_geometry_bytes(C.byref(_lib.rk_mesh(4, 2.0)), 2, _lib.RK_FP64,
                                          C.byref(out)) == _lib.RK_EINVAL
