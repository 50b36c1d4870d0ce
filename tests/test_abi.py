"""CPU-side checks of the C ABI library: it loads, exports every declared
entry point, and its own 64 -> 16 table agrees with the oracle's (both derived
independently from the class definitions).  No compute call needs a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import tc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_0-9]+)\s*\(", text)))


def test_library_loads():
    assert os.path.exists(tc.LIB_PATH), "libtc.so not built"
    tc.load()


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(tc.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_binding_covers_every_declared_symbol():
    assert sorted(tc.SIGNATURES) == declared_functions()


def test_library_table_matches_oracle_table():
    assert tc.tc_class_table().tolist() == oracle.table().tolist()


def test_status_strings():
    lib = tc.load()
    for code in range(-7, 1):
        s = lib.tc_status_string(code)
        assert s and s != b"unknown status"
    assert lib.tc_status_string(-99) == b"unknown status"


def test_null_arguments_rejected_without_device():
    lib = tc.load()
    assert lib.tc_class_table(None) == tc.TC_ERR_ARG
    assert lib.tc_context_create(0, 0, None, None) == tc.TC_ERR_ARG
    assert lib.tc_context_destroy(None) == tc.TC_ERR_ARG
    assert lib.tc_census(None, None, None) == tc.TC_ERR_ARG
    assert lib.tc_poll(None, 1, None, None) == tc.TC_ERR_ARG


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(tc, "_lib", None)
    monkeypatch.setattr(tc, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        tc.load()


def test_struct_layouts_match_header(tmp_path):
    """Every field of the binding's structures sits at the offset the C
    compiler gives it in include/tc.h, and the sizes agree."""
    structs = {name: getattr(tc, name) for name in ("tc_graph_info", "tc_tuning", "tc_kernel_stats",
                                                    "tc_serve_stats")}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "tc.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        name, key, value = line.split()
        cls = structs[name]
        got = ctypes.sizeof(cls) if key == "size" else getattr(cls, key).offset
        assert got == int(value), (name, key, got, value)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())
