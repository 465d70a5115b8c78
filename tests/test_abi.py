"""The C-ABI library loads and exports every symbol the header declares.
CPU only: no call that needs a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctrace.h")
LIB = os.path.join(ROOT, "paper_2010_08482_amd", "libctrace.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("ctr_create", "ctr_destroy", "ctr_set_impurity", "ctr_trace", "ctr_trace_batch",
                 "ctr_trace_batch_device", "ctr_trace_lazy_batch", "ctr_bound", "ctr_strings",
                 "ctr_status_string", "ctr_last_error", "ctr_version", "ctr_synchronize",
                 "ctr_arena_resident_bytes", "ctr_trace_histogram"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libctrace.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libctrace.so not built")
def test_status_strings_and_argument_errors_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.ctr_status_string.restype = ctypes.c_char_p
    assert lib.ctr_status_string(0) == b"CTR_OK"
    assert lib.ctr_status_string(-2) == b"CTR_ERR_OOM"
    lib.ctr_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.ctr_version()
    # null output pointer is rejected before any device call
    lib.ctr_create.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.ctr_create(0, None, 0, None, None) == -1
    assert lib.ctr_status_string(-8) == b"CTR_ERR_BUSY"
    # server: bad arguments are rejected before any thread or device work
    lib.ctr_server_create.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p()
    assert lib.ctr_server_create(None, 1, None, ctypes.byref(out)) == -1 and not out.value


def test_binding_names_match_header():
    src = open(os.path.join(ROOT, "paper_2010_08482_amd", "ctrace.py")).read()
    for name in declared_functions():
        assert f"def {name}(" in src, name


STRUCTS = ("ctr_value", "ctr_opts", "ctr_impurity", "ctr_mc_opts", "ctr_server_opts", "ctr_result")


def test_binding_struct_layouts_match_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets, as a C compiler lays them out (gcc on the header alone)."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler on this host")
    from paper_2010_08482_amd import ctrace

    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ctrace.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for name, _ in getattr(ctrace, s)._fields_:
            lines.append(f'  printf("{s} {name} %zu\\n", offsetof({s}, {name}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for s in STRUCTS:
        st = getattr(ctrace, s)
        assert got[(s, "size")] == ctypes.sizeof(st), s
        for name, _ in st._fields_:
            assert got[(s, name)] == getattr(st, name).offset, (s, name)


def test_markov_step_rejects_uniforms_of_the_wrong_shape():
    """The library reads n_chains x 6 uniforms: the binding refuses any other
    shape before the call (no chain set is needed to see it)."""
    import numpy as np

    from paper_2010_08482_amd import ctrace

    for shape in [(4, 5), (3, 6), (24,)]:
        with pytest.raises(ValueError):
            ctrace.ctr_mc_step(None, np.zeros(shape), n_chains=4)
