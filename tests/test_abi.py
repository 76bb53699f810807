"""The C-ABI library loads, exports every function include/cmtcs.h declares, and rejects bad
arguments on the host before any HIP call (no GPU needed for any of this)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2310_00420_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmtcs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cmtcs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("cmtcs_create", "cmtcs_destroy", "cmtcs_estep", "cmtcs_mstep", "cmtcs_em_iter",
              "cmtcs_mstep_pi", "cmtcs_solve", "cmtcs_apply", "cmtcs_profile", "cmtcs_rhs", "cmtcs_grad", "cmtcs_tiles", "cmtcs_last_error",
              "cmtcs_version"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version():
    assert _lib.load().cmtcs_version().startswith(b"cmtcs")


def _problem(**over):
    T = over.pop("T", 2)
    row_off = over.pop("row_off", np.array([0, 4, 8], np.int64))
    p = dict(T=T, C=2, D=32, row_off=row_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
             phi=1, phi_dtype=_lib.CMTCS_F32, phi_resid=None, y=1, beta=1.0,
             math=_lib.CMTCS_MATH_F64, max_rhs=34, max_iters=10, max_K=16)
    p.update(over)
    return _lib.Problem(**p), row_off


@pytest.mark.parametrize("over,frag", [
    (dict(D=30), "multiple of 16"),
    (dict(D=0), "multiple of 16"),
    (dict(T=0), "T and C"),
    (dict(C=0), "T and C"),
    (dict(beta=0.0), "beta"),
    (dict(max_iters=0), "max_iters"),
    (dict(max_rhs=0), "max_rhs"),
    (dict(max_rhs=20), "max_rhs"),
    (dict(phi=None), "phi and y"),
    (dict(row_off=np.array([0, 5, 3], np.int64)), "non-decreasing"),
    (dict(row_off=np.array([1, 5, 8], np.int64)), "row_off[0]"),
    (dict(math=_lib.CMTCS_MATH_MIXED), "MATH_MIXED"),
    (dict(math=_lib.CMTCS_MATH_MIXED, phi_dtype=_lib.CMTCS_BF16, D=48), "multiple of 32"),
    (dict(phi_dtype=_lib.CMTCS_BF16), "phi_dtype F32"),
    (dict(phi_resid=1), "phi_resid"),
    (dict(math=9), "unknown math mode"),
    (dict(phi_dtype=9), "phi_dtype F32"),
    (dict(math=_lib.CMTCS_MATH_MIXED, phi_dtype=-1), "BF16 or F16"),
    (dict(math=_lib.CMTCS_MATH_F32, phi_resid=1), "phi_resid"),
    (dict(D=16384, row_off=np.array([0, 4, 65540], np.int64)), "Phi block"),
    (dict(D=16384, max_rhs=40000), "column slots"),
])
def test_create_rejects_bad_problems(over, frag):
    lib = _lib.load()
    p, keep = _problem(**over)
    h = ctypes.c_void_p(123)
    rc = lib.cmtcs_create(ctypes.byref(h), ctypes.byref(p), None)
    assert rc in (_lib.CMTCS_E_INVALID, _lib.CMTCS_E_UNSUPPORTED)
    assert h.value is None
    assert frag in lib.cmtcs_last_error().decode()


@pytest.mark.parametrize("over,frag", [
    (dict(op=7), "unknown sensing operator"),
    (dict(op=_lib.CMTCS_OP_PARTIAL_FOURIER, freq=1, math=_lib.CMTCS_MATH_F32), "MATH_F64"),
    (dict(op=_lib.CMTCS_OP_PARTIAL_FOURIER, freq=1, D=48), "power of two"),
    (dict(op=_lib.CMTCS_OP_PARTIAL_FOURIER, freq=1, D=8192), "power of two"),
    (dict(op=_lib.CMTCS_OP_PARTIAL_FOURIER, freq=None, D=64), "freq and y"),
])
def test_create_rejects_bad_fourier_problems(over, frag):
    test_create_rejects_bad_problems(over, frag)


def test_apply_noalloc_rejects_on_the_host():
    """Argument errors and problems beyond the static scratch array are reported before any
    HIP call."""
    lib = _lib.load()
    cc = (ctypes.c_int32 * 64)()
    assert lib.cmtcs_apply_noalloc(None, 1, 1, cc, 1, 1, None) == _lib.CMTCS_E_INVALID
    p, keep = _problem()
    assert lib.cmtcs_apply_noalloc(ctypes.byref(p), None, 1, cc, 1, 1, None) == \
        _lib.CMTCS_E_INVALID
    p, keep = _problem(op=_lib.CMTCS_OP_PARTIAL_FOURIER, D=64)
    assert lib.cmtcs_apply_noalloc(ctypes.byref(p), 1, 1, cc, 1, 1, None) == \
        _lib.CMTCS_E_UNSUPPORTED
    for over in (dict(op=5), dict(math=7), dict(math=_lib.CMTCS_MATH_MIXED)):
        p, keep = _problem(**over)
        assert lib.cmtcs_apply_noalloc(ctypes.byref(p), 1, 1, cc, 1, 1, None) == \
            _lib.CMTCS_E_UNSUPPORTED
    p, keep = _problem(phi_dtype=4)
    assert lib.cmtcs_apply_noalloc(ctypes.byref(p), 1, 1, cc, 1, 1, None) == \
        _lib.CMTCS_E_INVALID
    # 720 column slots x 16384 x 8 bytes of padded right-hand sides alone exceed 64 MiB
    R = 600
    big = (ctypes.c_int32 * R)()
    p, keep = _problem(T=1, D=16384, row_off=np.array([0, 8], np.int64))
    assert lib.cmtcs_apply_noalloc(ctypes.byref(p), 1, R, big, 1, 1, None) == \
        _lib.CMTCS_E_INVALID
    assert "too large" in lib.cmtcs_last_error().decode()


def test_null_arguments():
    lib = _lib.load()
    assert lib.cmtcs_create(None, None, None) == _lib.CMTCS_E_INVALID
    h = ctypes.c_void_p()
    assert lib.cmtcs_create(ctypes.byref(h), None, None) == _lib.CMTCS_E_INVALID
    o = _lib.Opts(K=1, max_iters=1)
    assert lib.cmtcs_estep(None, None, None, ctypes.byref(o), None, None, None, None, None,
                           None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_mstep(None, None, None, None, ctypes.byref(o), None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_mstep_pi(None, None, None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_em_iter(None, None, None, ctypes.byref(o), None, None, None, None,
                             None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_solve(None, None, 1, None, None, None, None, None, ctypes.byref(o),
                           None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_apply(None, None, 1, None, None, None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_profile(None, 1, None, None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_rhs(None, None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_tiles(None, None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_grad(None, 1, None, None, None, 0.0, None, None) == _lib.CMTCS_E_INVALID
    assert lib.cmtcs_destroy(None) == _lib.CMTCS_OK


def test_error_raises_from_python():
    with pytest.raises(_lib.CmtcsError) as e:
        _lib.check(_lib.load().cmtcs_create(None, None, None))
    assert e.value.code == _lib.CMTCS_E_INVALID


def test_comparison_initial_alpha_follows_the_workload_recipe():
    """The support-difference comparison draws alpha^0 as the synthetic workloads do (Alg. 2
    initialisation, U(0, 1) per (c, d), float32), so its fits start where the oracle's would."""
    import synth
    from paper_2310_00420_amd.experiments import _alpha0
    for C, D in ((1, 512), (2, 512), (3, 77)):
        a = _alpha0(C, D, synth.INIT_SEED)
        assert a.dtype == np.float32
        assert np.array_equal(a.astype(np.float64), synth.draw_alpha0(C, D, synth.INIT_SEED))
