"""The C-ABI library loads and exports every entry point that include/lsmg.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsmg.h")
LIB = os.path.join(ROOT, "paper_1902_07029_amd", "liblsmg.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lsmg_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("lsmg_build_hierarchy", "lsmg_newton_cn_step", "lsmg_vcycle"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblsmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblsmg.so not built")
def test_default_params_follow_the_paper():
    from paper_1902_07029_amd import lsmg
    p = lsmg.default_params()
    # eq. (dataeq) and tau_s = 0.9 (section 3.5.1)
    assert (p.a, p.d, p.m_s, p.m_c, p.alpha, p.beta, p.tau_s) == (1e4, 0.1, 64.06, 100.09, 0.01, 0.1, 0.9)
    assert p.precision == 0 and p.newton_tol == 1e-10


@pytest.mark.parametrize("struct", ["lsmg_params", "lsmg_step_stats"])
def test_binding_structs_match_the_header(tmp_path, struct):
    # the binding's ctypes structures have the header's field offsets and sizes
    # (compiled on the host with gcc; the header is plain C)
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    from paper_1902_07029_amd import lsmg
    cls = {"lsmg_params": lsmg.Params, "lsmg_step_stats": lsmg.StepStats}[struct]
    fields = [f for f, _ in cls._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text(f'#include <stddef.h>\n#include <stdio.h>\n#include "lsmg.h"\n'
                   f'int main(void) {{\n{body}    printf("%zu\\n", sizeof({struct}));\n    return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[:-1] == [getattr(cls, f).offset for f in fields]
    assert out[-1] == ctypes.sizeof(cls)
