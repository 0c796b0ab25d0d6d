"""The C-ABI library on the CPU: it loads, exports every function that
include/d2.h declares, its structs have the layout the binding assumes, and
host-side validation answers without touching a GPU.  Also checks that the
product package never reaches the oracle."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "d2.h")
PKG = os.path.join(ROOT, "paper_1302_0435_amd")


@pytest.fixture(scope="module")
def ffi():
    from paper_1302_0435_amd import _ffi
    if not os.path.exists(_ffi.LIB_PATH):
        pytest.fail("libd2.so is not built (run __graft_entry__.build())")
    _ffi.lib()
    return _ffi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(d2_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    from paper_1302_0435_amd import _ffi
    assert declared_functions() == sorted(_ffi.EXPORTS)


def test_library_exports_every_declared_symbol(ffi):
    out = subprocess.run(["nm", "-D", "--defined-only", ffi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in syms, name
        assert hasattr(ffi.lib(), name)


def test_struct_layout_matches_c(ffi, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "d2.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(d2_set), offsetof(d2_set, offsets),
         offsetof(d2_set, points), offsetof(d2_set, weights), offsetof(d2_set, max_support),
         sizeof(d2_opts), offsetof(d2_opts, opt_tol), offsetof(d2_opts, bland_after));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                       check=True).stdout.split()))
    S, O = ffi.d2_set, ffi.d2_opts
    want = [ctypes.sizeof(S), S.offsets.offset, S.points.offset, S.weights.offset,
            S.max_support.offset, ctypes.sizeof(O), O.opt_tol.offset, O.bland_after.offset]
    assert got == want


def test_constants_and_strings(ffi):
    L = ffi.lib()
    assert L.d2_max_support() == 64
    assert L.d2_version().decode().startswith("d2-mi355x")
    for code in range(7):
        assert L.d2_status_string(code).decode() != "unknown status"
    assert L.d2_status_string(99).decode() == "unknown status"


def test_null_handle_is_rejected_without_a_gpu(ffi):
    L = ffi.lib()
    s = ffi.d2_set(0, 3, ffi.D2_F64, None, None, None, 1, 0)
    o = ffi.d2_opts(0, 0, 0, 0, 0.0)
    r = ctypes.byref
    assert L.d2_assign(None, r(s), r(s), r(o), None, None, None, None, None, 0, None) == ffi.D2_EINVAL
    assert L.d2_pairwise(None, r(s), r(o), None, None, None, 0, None) == ffi.D2_EINVAL
    assert L.d2_emd_batch(None, r(s), r(s), None, 0, r(o), None, None, None, None, None, None,
                          None, None, 0, None) == ffi.D2_EINVAL
    assert L.d2_cost_tiles(None, r(s), r(s), None, 0, 0, None, None, None, 0, None) == ffi.D2_EINVAL
    assert L.d2_workspace_bytes(None, 2, r(s), r(s), 0, r(o)) == 0
    assert L.d2_create(None, 0) == ffi.D2_EINVAL
    assert L.d2_destroy(None) == ffi.D2_OK


def test_product_path_never_reaches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("oracles", ""), f
                assert "import synth" not in text and "from synth" not in text, f


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1302_0435_amd import _ffi
    monkeypatch.setattr(_ffi, "_lib", None)
    monkeypatch.setattr(_ffi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(_ffi.LibraryMissing):
        _ffi.lib()
