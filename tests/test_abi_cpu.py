"""Host-side checks of the C ABI: the library loads and exports every function
include/kbnb.h declares, and the Python binding mirrors the C structures.
No compute calls are made (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2605_22188_amd as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kbnb.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ["create_problem", "destroy_problem", "submit_nodes", "poll_bounds",
                     "branch_and_bound", "last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(K.LIB_PATH), reason="libkbnb.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(K.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(K.EXPORTS)


STRUCTS = {"kbnb_problem_desc": K.ProblemDesc, "kbnb_node_desc": K.NodeDesc,
           "kbnb_tune_options": K.TuneOptions, "kbnb_tune_result": K.TuneResult,
           "kbnb_bound_result": K.BoundResult, "kbnb_bnb_options": K.BnbOptions,
           "kbnb_bnb_result": K.BnbResult}


def test_struct_layouts_match_header(tmp_path):
    """Compile a C program against include/kbnb.h and compare every field offset."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "kbnb.h"', "int main(void){"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    for line in filter(None, out):
        cname, field, val = line.split()
        py = STRUCTS[cname]
        got = ctypes.sizeof(py) if field == "size" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)


@pytest.mark.skipif(not os.path.exists(K.LIB_PATH), reason="libkbnb.so not built")
def test_null_handle_errors_without_device():
    lib = K.load()
    assert lib.destroy_problem(None) == -5
    assert lib.submit_nodes(None, None, 0) == -5
    assert "NULL" in K.last_error()


def test_autotune_rejects_bad_candidates_before_any_device_call():
    X = np.zeros((4, 3), np.float32)
    y = np.ones(4)
    for kw in [dict(widths=[0]), dict(widths=[8192]), dict(periods=[0]), dict(widths=[]),
               dict(nodes=[([5], [])] * 0 + [([0], [1])], widths=[64], periods=[-1])]:
        with pytest.raises(K.KbnbError) as e:
            K.autotune(X, y, 1, 0, 1.0, 1.0, dtype="f32", **kw)
        assert e.value.code == -1, kw


def test_header_constants_match_binding():
    text = open(os.path.join(ROOT, "include", "kbnb.h")).read()
    defs = dict((m.group(1), int(m.group(2))) for m in
                re.finditer(r"#define KBNB_(\w+) \(?(-?\d+)\)?", text))
    pairs = {"OK": "OK", "TIMEOUT": "TIMEOUT", "CONVERGED": "CONVERGED", "PRUNED": "PRUNED",
             "MAXITER": "MAXITER", "DTYPE_F64": "DTYPE_F64", "DTYPE_F32": "DTYPE_F32",
             "DTYPE_BF16": "DTYPE_BF16", "ITER_AUTO": "ITER_AUTO", "ITER_F32": "ITER_F32",
             "ITER_F64": "ITER_F64", "ITER_ANCHORED": "ITER_ANCHORED",
             "MEM_HOST_COPY": "MEM_HOST_COPY",
             "MEM_DEVICE_COPY": "MEM_DEVICE_COPY"}
    for hname, pname in pairs.items():
        assert defs[hname] == getattr(K, pname), hname
