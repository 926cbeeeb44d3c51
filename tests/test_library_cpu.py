"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wfa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wfa_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["wfa_ctx_create", "wfa_ctx_destroy", "wfa_align_batch", "wfa_copy_last_cigars",
              "wfa_strerror", "wfa_server_open", "wfa_server_submit", "wfa_server_poll",
              "wfa_server_close"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2204_02085_amd as wfa

    lib = ctypes.CDLL(wfa.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} not exported"
    assert sorted(wfa.EXPORTED) == declared_functions()


def test_strerror_and_null_context():
    import paper_2204_02085_amd as wfa

    assert wfa.wfa_strerror(wfa.WFA_E_CAPACITY).decode().startswith("CIGAR buffer")
    assert wfa.wfa_strerror(12345) == b"unknown status"
    assert wfa.wfa_set_options(None, None) == wfa.WFA_E_INVAL
    needed = ctypes.c_size_t(7)
    bad = ctypes.c_int64(7)
    rc = wfa.wfa_align_batch(None, None, None, None, 0, 0, 0, wfa.wfa_penalties(4, 6, 2), 1, None,
                             None, 0, None, ctypes.byref(needed), ctypes.byref(bad), None)
    assert rc == wfa.WFA_E_INVAL and bad.value == -1
    assert wfa.wfa_copy_last_cigars(None, None, 0, None) == wfa.WFA_E_INVAL
    assert wfa.wfa_server_close(None) == wfa.WFA_E_INVAL


def test_pair_descriptor_layout(tmp_path):
    """The binding's structures match the header's, field by field (sizes and
    offsets printed by a C program compiled against include/wfa.h)."""
    import subprocess

    import paper_2204_02085_amd as wfa

    structs = {"wfa_pair": None, "wfa_penalties": wfa.wfa_penalties,
               "wfa_options": wfa.wfa_options, "wfa_stats": wfa.wfa_stats,
               "wfa_ends_free": wfa.wfa_ends_free}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "wfa.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        if cls is not None:
            for f, _ in cls._fields_:
                lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    assert int(got["wfa_pair"]) == wfa.PAIR_DTYPE.itemsize == 24
    for name, cls in structs.items():
        if cls is None:
            continue
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"


def test_noalloc_constants_and_null_context():
    """The allocation-free entry point's limits in the binding match the
    header, and it rejects a missing context before touching a device."""
    import paper_2204_02085_amd as wfa

    src = open(os.path.join(ROOT, "include", "wfa.h")).read()
    assert "#define WFA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)" in src
    assert "#define WFA_NOALLOC_MAX_PAIRS ((uint32_t)1 << 18)" in src
    assert wfa.WFA_NOALLOC_SCRATCH_BYTES == 128 << 20 and wfa.WFA_NOALLOC_MAX_PAIRS == 1 << 18
    needed = ctypes.c_size_t(7)
    bad = ctypes.c_int64(7)
    rc = wfa.wfa_align_batch_noalloc(None, None, None, None, 0, 0, wfa.wfa_penalties(4, 6, 2), 1,
                                     None, None, 0, None, ctypes.byref(needed), ctypes.byref(bad),
                                     None)
    assert rc == wfa.WFA_E_INVAL and bad.value == -1 and needed.value == 0
