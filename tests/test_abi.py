"""The C-ABI library loads and exports every entry point include/m4.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2607_12074_amd as m4

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for mt in re.finditer(r"\b(m4_[a-z0-9_]+)\s*\(", text):
            names.add(mt.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("m4_count_motifs4", "m4_count_motifs4_ex", "m4_ctx_create", "m4_count_batch",
                 "m4_server_create", "m4_edge_triangles", "m4_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = m4.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_strerror_without_device():
    L = m4.lib()
    for code in range(8):
        assert L.m4_strerror(code)
    assert b"64 bits" in L.m4_strerror(m4.M4_EOVERFLOW)


def test_struct_layout_matches_header():
    # sizes of the ABI structs as laid out by a C compiler for x86-64
    assert ctypes.sizeof(m4.Csr) == 40
    assert ctypes.sizeof(m4.Opts) == 48
    assert ctypes.sizeof(m4.Batch) == 48


def test_signature_keys_distinguish_masks():
    # Two states with the same frontier slot but different adjacency or
    # non-adjacency requirements must never share a cache key (Section III-C).
    L = m4.lib()
    f = L.m4_internal_sig_key
    f.argtypes = [ctypes.c_uint32] * 4
    f.restype = ctypes.c_uint32
    keys = {}
    for j in (1, 2, 3):
        for mp in range(16):
            for mm in range(16):
                if mp & mm:
                    continue
                k = f(j, 123, mp, mm)
                assert k not in keys, (j, mp, mm, keys.get(k))
                keys[k] = (j, mp, mm)
    assert f(2, 5, 3, 0) != f(2, 5, 1, 2)  # adjacent to both vs to exactly one
    assert f(2, 5, 3, 0) != f(2, 6, 3, 0)


def test_missing_library_fails_loudly(monkeypatch):
    # no fallback: without the built HIP library every call raises
    import paper_2607_12074_amd as m4
    monkeypatch.setattr(m4, "LIB_PATH", "/nonexistent/libm4.so")
    monkeypatch.setattr(m4, "_lib", None)
    with pytest.raises(m4.M4Error) as e:
        m4.lib()
    assert e.value.code == m4.M4_EDEVICE
    assert "missing" in str(e.value)


def test_struct_sizes_match_a_c_compiler(tmp_path):
    # every ABI struct as a C compiler lays it out from include/m4.h, against
    # the binding's ctypes mirror (field offsets of the two largest structs too)
    import subprocess
    src = tmp_path / "sizes.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "m4.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(m4_csr), sizeof(m4_opts),
         sizeof(m4_stats), sizeof(m4_batch), sizeof(m4_tuning), sizeof(m4_result),
         offsetof(m4_stats, ms_kernel), offsetof(m4_stats, device_bytes),
         offsetof(m4_result, t_submit_ms));
  return 0;
}
''')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(m4.Csr), ctypes.sizeof(m4.Opts), ctypes.sizeof(m4.Stats),
            ctypes.sizeof(m4.Batch), ctypes.sizeof(m4.Tuning), ctypes.sizeof(m4.Result),
            m4.Stats.ms_kernel.offset, m4.Stats.device_bytes.offset,
            m4.Result.t_submit_ms.offset]
    assert got == want
