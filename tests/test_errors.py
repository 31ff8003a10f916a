"""Host-side validation of the C ABI (runs without a GPU: arguments are checked first)."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_04634_amd", "libnullspace.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _init(**kw):
    from paper_2407_04634_amd import _lib

    lib = _lib.load()
    p = _lib.default_params(**{k: v for k, v in kw.items() if k in dict(_lib.Params._fields_)})
    h = ctypes.c_void_p()
    m, n = kw.get("m", 100), kw.get("n", 100)
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    st = lib.nullspace_init(ctypes.byref(h), m, n, kw.get("nnz", 10), kw.get("rowptr", dummy), dummy,
                            dummy, None, None, ctypes.byref(p), None)
    return st, lib.nullspace_last_error().decode(), h


@pytest.mark.parametrize("kw,msg", [
    (dict(eps=0.0), "eps"),
    (dict(eps=float("nan")), "eps"),
    (dict(d=3), "d must be"),
    (dict(d=4, max_dim=66), "multiple of d"),
    (dict(d=4, max_dim=8), "at least 3d"),
    (dict(max_dim=100), "must not exceed n"),
    (dict(m=0), "m and n"),
    (dict(nnz=-1), "nnz"),
    (dict(max_matvec=0), "max_matvec"),
    (dict(prec=7), "precision"),
    (dict(op=5), "op must be"),
    (dict(reorder=3), "reorder"),
    (dict(precond=3), "precond must be"),
    (dict(precond=2, ic_droptol=-1.0), "ic_droptol"),
    (dict(precond=2, ic_diagcomp=float("nan")), "ic_diagcomp"),
    (dict(op=1, m=120, n=100), "square"),
])
def test_invalid_arguments_are_rejected(kw, msg):
    from paper_2407_04634_amd import _lib

    st, err, h = _init(**kw)
    assert st == _lib.NSP_ERR_ARG
    assert msg in err
    assert not h.value


def test_null_context_calls_fail_cleanly():
    from paper_2407_04634_amd import _lib

    lib = _lib.load()
    assert lib.lanczos_run(None, None) == _lib.NSP_ERR_ARG
    assert lib.extract_basis(None, None, 0) == _lib.NSP_ERR_ARG
    lib.nullspace_destroy(None)
