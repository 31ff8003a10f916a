"""The C-ABI library loads and exports every symbol include/nullspace.h declares (CPU-only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2407_04634_amd", "libnullspace.so")
HEADER = os.path.join(ROOT, "include", "nullspace.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:nsp_status|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("nullspace_init", "apply_op", "lanczos_run", "extract_basis", "backward",
                 "nullspace_destroy", "nullspace_last_error"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (binds the HIP runtime torch ships before the library)

    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_params_and_binding_symbols():
    from paper_2407_04634_amd import _lib

    p = _lib.default_params()
    assert p.d == 1 and p.max_dim == 64 and abs(p.eps - 1e-3) < 1e-18 and p.refine == 1
    assert set(_lib.EXPORTS) <= set(_declared()) | {"nsp_default_params"}
