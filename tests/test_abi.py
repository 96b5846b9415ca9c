"""CPU checks of the C ABI: the library loads, exports what include/pac.h declares,
and rejects bad arguments before touching a device."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2603_15023_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(A.LIB_PATH):
        from paper_2603_15023_amd import build
        build.build()
    return A.load()


def test_library_exports_every_declared_function(lib):
    declared = A.header_functions()
    assert set(declared) == set(A.EXPORTS), "binding and header disagree"
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in declared if f not in exported]
    assert not missing, f"not exported: {missing}"
    for f in declared:
        assert hasattr(lib, f)


def test_library_holds_gfx950_code():
    # the device code object bundle in .hip_fatbin names its target triple
    with open(A.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_version_and_null_arguments(lib):
    assert lib.pac_version() == 1
    assert lib.pac_ctx_create(0, None) == -1
    assert b"null" in lib.pac_last_error()
    assert lib.pac_ctx_destroy(None) == 0
    assert lib.pac_check(None, None, None) == -1
    assert lib.pac_hash_mask(None, None, None, 0, 0, 64, 0, None) == -1
    inp = A.AggInput()
    st = A.AggState()
    assert lib.pac_group_aggregate(None, None, C.byref(inp), 64, 0, 0, 0, C.byref(st)) == -1
    params = A.FinalizeParams(1.0 / 128, 1, -1, 1)
    assert lib.pac_finalize(None, None, C.byref(st), 64, 1, 0, 0, None, 0, C.byref(params), None, None, None, None,
                            None) == -1


def test_struct_sizes_match_header():
    # pac_cell is 16 bytes, pac_finalize_params 24, the input struct has the documented field order
    assert C.sizeof(A.Cell) == 16
    assert C.sizeof(A.FinalizeParams) == 24
    assert A.AggInput.n_cols.offset < A.AggInput.cols.offset < A.AggInput.col_type.offset


def test_ctypes_layout_matches_c_header(tmp_path):
    """Compile a probe against include/pac.h with gcc and compare every field offset."""
    structs = {"pac_agg_input": A.AggInput, "pac_agg_state": A.AggState, "pac_cell": A.Cell,
               "pac_finalize_params": A.FinalizeParams, "pac_lift_op": A.LiftOp}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pac.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_product_code_does_not_use_the_oracle():
    """The package and the shared input generators neither import nor build
    anything under oracle/ (only the tests, smoke() and the CPU-baseline leg
    of bench.py may), and the HIP sources include nothing from it."""
    import ast

    offenders = []
    for sub in ("paper_2603_15023_amd", "workloads"):
        for dirpath, _, files in os.walk(os.path.join(ROOT, sub)):
            for f in files:
                path = os.path.join(dirpath, f)
                if f.endswith(".py"):
                    tree = ast.parse(open(path).read(), path)
                    for node in ast.walk(tree):
                        names = []
                        if isinstance(node, ast.Import):
                            names = [a.name for a in node.names]
                        elif isinstance(node, ast.ImportFrom) and node.level == 0:
                            names = [node.module or ""]
                        if any(n == "oracle" or n.startswith("oracle.") for n in names):
                            offenders.append(f"{path}:{node.lineno}")
                elif f.endswith((".hip", ".h", ".cpp", ".c")):
                    for i, line in enumerate(open(path), 1):
                        if line.lstrip().startswith("#include") and "oracle" in line:
                            offenders.append(f"{path}:{i}")
    assert not offenders, f"product code reaches the oracle: {offenders}"
