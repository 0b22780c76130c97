"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mtp.h")
LIB = os.path.join(ROOT, "paper_2510_00193_amd", "libmtp.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mtp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("mtp_create", "mtp_destroy", "mtp_compute", "mtp_grade", "mtp_neighbors", "mtp_param_grad",
                 "mtp_sizes", "mtp_last_error", "mtp_set_params", "mtp_levels"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmtp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmtp.so not built")
def test_levels_query_without_gpu():
    from paper_2510_00193_amd import compiled_levels
    levels = compiled_levels()
    assert 10 in levels and 16 in levels


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2510_00193_amd import _lib
    with pytest.raises(RuntimeError, match="missing"):
        _lib.open_library(str(tmp_path / "nope.so"))


def test_ctypes_structures_match_the_header_layout(tmp_path):
    """The binding's structures have the size and field offsets the C compiler gives the
    header's structures (a field added on one side only would shift every later field)."""
    import shutil
    import subprocess
    from paper_2510_00193_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mtp_params": _lib.MtpParams, "mtp_system": _lib.MtpSystem, "mtp_nlist": _lib.MtpNlist}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mtp.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
