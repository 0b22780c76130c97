"""Host (CPU) build of the generated level programs, checked against central differences.

The device code generator emits plain templated C++; compiled for the host it
must agree with finite differences of its own value functions (tangents of the
moments, contractions, products and adjoints) and with the plain definition of
the adjoint pair sums.
"""
import os
import shutil
import subprocess

import pytest

from paper_2510_00193_amd.codegen.emit import emit_level

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
@pytest.mark.parametrize("level,groups,budget", [(6, 1, None), (10, 1, None), (10, 2, None), (12, 3, None),
                                                 (14, 1, None), (14, 2, None), (12, 1, 140), (14, 2, 200)])
def test_generated_tangents_match_differences(tmp_path, level, groups, budget):
    """budget: a register budget small enough to cut the reverse-tangent program into several
    parts (stores of first touches, additions of later ones, zeros of untouched entries)."""
    hdr = tmp_path / f"L{level}.inc"
    text = emit_level(level, groups) if budget is None else emit_level(level, groups, rtan_budget=budget)
    if budget is not None:
        assert int(text.split("NRTPART = ")[1].split(";")[0]) > 1, "budget too large for a split"
    hdr.write_text(text)
    exe = tmp_path / "harness"
    cmd = ["g++", "-O1", "-std=c++17", f'-DMTP_LEVEL_HEADER="{hdr}"', f"-DMTP_LEVEL_STRUCT=Lv{level}",
           f"-DMTP_NGROUP={groups}", os.path.join(HERE, "host_harness.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    errs = {line.split()[0]: float(line.split()[1]) for line in out.strip().splitlines()}
    assert errs["fwd_value"] == 0.0
    assert errs["products_cb"] == 0.0
    for k in ("tan_moments", "fwd_tan", "products_out", "products_cbd", "rev_tan", "pair_grad"):
        assert errs[k] < 1e-7, (k, errs)
    assert errs["adj_pair_S"] < 1e-13 and errs["adj_pair_A"] < 1e-13, errs
