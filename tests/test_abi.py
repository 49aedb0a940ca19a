"""The C-ABI library loads on the CPU and exports every function include/ebamg.h declares.

No compute call is made here (no GPU in CPU-only runs)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebamg.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = "\n".join(line for line in text.splitlines() if not line.lstrip().startswith("typedef"))
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def libpath():
    from paper_2204_06083_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2204_06083_amd import build
        build.build(jobs=4)
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("eb_assemble_diag", "eb_assemble_rhs", "stencil_apply", "amg_setup", "pcg_solve",
                     "amg_free", "eb_strerror", "eb_last_error"):
        assert required in names, required


def test_every_declared_symbol_is_exported(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(_declared_functions()) <= exported


def test_binding_covers_exports_and_host_only_calls(libpath):
    from paper_2204_06083_amd import _lib
    L = _lib.lib()
    assert set(_lib.EXPORTS) == set(_declared_functions())
    assert L.eb_abi_version() == 1
    assert L.eb_strerror(_lib.EB_EDOMAIN).decode().startswith("domain")
    # host-side validation rejects bad arguments before any device work
    g = _lib.EbGrid()
    g.dim = 5
    nu, nc = ctypes.c_int64(), ctypes.c_int64()
    rc = L.eb_assemble_diag(ctypes.byref(g), None, None, None, None, 0, ctypes.byref(nu), ctypes.byref(nc), None)
    assert rc == _lib.EB_EINVAL
    assert b"grid" in L.eb_last_error()
    h = ctypes.c_void_p()
    rc = L.amg_setup(None, None, None, 0.0, None, ctypes.byref(h), None)
    assert rc == _lib.EB_EINVAL and not h.value
    assert L.amg_num_levels(None) == 0


def test_struct_layouts_match_header():
    from paper_2204_06083_amd import _lib
    assert ctypes.sizeof(_lib.EbGrid) == 48
    assert ctypes.sizeof(_lib.AmgParams) == 48
    assert ctypes.sizeof(_lib.PcgParams) == 24
    assert ctypes.sizeof(_lib.PcgResult) == 48
    assert _lib.CUT_DTYPE.itemsize == 56
    assert ctypes.sizeof(_lib.LevelInfo) == 72 + 12 * 8


def test_struct_layouts_against_a_c_compiler(tmp_path):
    """sizeof / offsetof of the header's structs as a C compiler lays them out,
    against the ctypes declarations of the binding."""
    from paper_2204_06083_amd import _lib
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ebamg.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(eb_grid_t), sizeof(amg_params_t),\n'
        "         offsetof(amg_params_t, alloc), offsetof(amg_params_t, free), offsetof(amg_params_t, alloc_ctx),\n"
        "         sizeof(pcg_params_t), sizeof(eb_cut_t));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P = _lib.AmgParams
    assert vals == [ctypes.sizeof(_lib.EbGrid), ctypes.sizeof(P), P.alloc.offset, P.free.offset,
                    P.alloc_ctx.offset, ctypes.sizeof(_lib.PcgParams), _lib.CUT_DTYPE.itemsize]
