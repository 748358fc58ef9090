"""Host-side checks of the C interface (no GPU): the shared library loads and
exports every entry point the header declares, and the binding's constants
match the header's."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ocpamg.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("typedef", "void", "const", "int")))


def _lib_or_skip():
    from paper_2102_03515_amd import capi
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libocpamg.so not built")
    return capi


def test_header_declares_the_interface():
    names = _declared_functions()
    for must in ("fe_assemble", "amg_setup", "pcg_solve", "ocp_ctx_create", "amg_vcycle", "ocp_spmv"):
        assert must in names


def test_library_exports_every_declared_symbol():
    capi = _lib_or_skip()
    import ctypes
    L = ctypes.CDLL(capi.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(L, name), f"{name} declared in the header but not exported"
    assert set(capi.exported_symbols()) == set(_declared_functions())


def test_constants_match_header():
    capi = _lib_or_skip()
    src = open(HEADER).read()
    defs = dict(re.findall(r"#define (OCP_\w+) \(?(-?\d+)\)?", src))
    assert int(defs["OCP_OK"]) == capi.OK
    assert int(defs["OCP_MAXIT"]) == capi.MAXIT
    assert int(defs["OCP_ERR_INVALID_ARG"]) == capi.ERR_INVALID_ARG
    assert int(defs["OCP_ERR_BAD_MESH"]) == capi.ERR_BAD_MESH
    assert int(defs["OCP_ERR_BREAKDOWN"]) == capi.ERR_BREAKDOWN
    assert int(defs["OCP_ERR_UNSUPPORTED"]) == capi.ERR_UNSUPPORTED
    assert int(defs["OCP_PREC_MIXED"]) == capi.PREC_MIXED
    assert int(defs["OCP_STOP_PRECOND"]) == capi.STOP_PRECOND
    assert int(defs["OCP_TARGET_BOX"]) == capi.TARGET_BOX
    assert int(defs["OCP_KEEP_KM"]) == capi.KEEP_KM
    assert int(defs["OCP_NO_LOAD"]) == capi.NO_LOAD
    assert int(defs["OCP_AMG_REDBLACK"]) == capi.AMG_REDBLACK


def test_struct_layouts():
    """ctypes structures have the sizes the C compiler gives the header's structs."""
    capi = _lib_or_skip()
    import ctypes
    assert ctypes.sizeof(capi._Mesh) == 4 + 4 + 3 * 8
    assert ctypes.sizeof(capi._Target) == 4 + 4 + 8 + 8 + 8 + 48 + 8
    assert ctypes.sizeof(capi.SolveInfo) == 8 + 5 * 8
    assert ctypes.sizeof(capi._AmgParams) == 5 * 4 + 4 + 3 * 8 + 8


def test_package_has_no_cpu_fallback():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2102_03515_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that gcc gives the header's struct (compiled here from the header)."""
    import ctypes
    import shutil
    import subprocess
    capi = _lib_or_skip()
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    pairs = [("ocp_mesh", capi._Mesh), ("ocp_target", capi._Target), ("ocp_system_view", capi._SystemView),
             ("ocp_amg_params", capi._AmgParams), ("ocp_level_view", capi._LevelView),
             ("ocp_solve_info", capi.SolveInfo)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ocpamg.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for cname, cls in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
