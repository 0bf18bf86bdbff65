"""The C-ABI library loads and exports every function declared in include/ib.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ib.h")
LIB = os.path.join(ROOT, "paper_2309_03600_amd", "libibwave.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ib_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2309_03600_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_declares_the_same_functions():
    from paper_2309_03600_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()


def test_abi_version_and_error_text(lib):
    lib.ib_abi_version.restype = ctypes.c_int32
    assert lib.ib_abi_version() == 4
    lib.ib_last_error.restype = ctypes.c_char_p
    assert lib.ib_last_error() is not None


def test_argument_errors_without_gpu(lib):
    # null arguments are rejected on the host before any device call
    lib.ib_build_weights.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.ib_build_weights(None, None, None, None, ctypes.byref(out)) == -1
    lib.ib_step.restype = ctypes.c_int
    assert lib.ib_step(None, 1, None, 0, None, 0, None) == -1


def test_struct_layouts_match_the_header(tmp_path):
    # the binding's ctypes structures against the header, compiled by the host C compiler
    import shutil
    import subprocess

    from paper_2309_03600_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"ib_grid": _lib.ib_grid, "ib_params": _lib.ib_params, "ib_stats": _lib.ib_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ib.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            name, field, val = line.split()
            got[(name, field)] = int(val)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


def test_forcing_rejects_a_null_state_without_gpu(lib):
    lib.ib_state_set_forcing.restype = ctypes.c_int
    assert lib.ib_state_set_forcing(None, None, 0, None, 0, None) == -1
