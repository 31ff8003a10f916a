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


def test_binding_structs_match_the_header_layout(tmp_path):
    """Offsets and sizes of nsp_params / nsp_stats as the C compiler lays them out."""
    import shutil
    import subprocess

    from paper_2407_04634_amd import _lib

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "nullspace.h"', "int main(void) {"]
    for cname, py in (("nsp_params", _lib.Params), ("nsp_stats", _lib.Stats)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in (("nsp_params", _lib.Params), ("nsp_stats", _lib.Stats)):
        assert got[(cname, "size")] == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
