"""The C ABI on the host: the library loads, exports what include/fab.h declares, and the
ctypes mirrors of its structs have the C layout (checked with the system C compiler)."""
import os
import re
import subprocess

import pytest

from paper_2503_22631_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(_lib.HEADER).read()
    return sorted(set(re.findall(r"^(?:fab_status|const char\*)\s+(fab_\w+)\s*\(", src, re.M)))


def test_header_declares_expected_api():
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfab.so not built")
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fab_\w+)", out))
    assert set(_declared()) <= exported


def test_status_strings_and_null_argument_checks():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfab.so not built")
    lib = _lib.load()
    for code in _lib.STATUS:
        assert lib.fab_status_string(code)
    import ctypes
    # validation happens before any HIP call
    assert lib.fab_create(None, None) == -1
    assert lib.fab_csr_create(None, 10, 10, None, None, None, 0, None) == -1
    assert lib.fab_op_destroy(None) == -1
    assert lib.fab_destroy(None) == -1
    p = _lib.fab_params(20, 2, 80, 8, 1, 1e-10, 10, 0, 0, 0.0, 0.0)
    assert lib.fab_workspace_size(None, ctypes.byref(p), 1, None) == -1
    flag = ctypes.c_int32(7)
    assert lib.fab_op_store_policy(None, 0, ctypes.byref(flag)) == -1 and flag.value == 7
    assert lib.fab_op_index_bytes(None, ctypes.byref(flag)) == -1
    assert lib.fab_batch_group(None, 4) == -1
    assert lib.fab_timing_enable(None, 1) == -1


def test_ctypes_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "lay.c"
    prog.write_text(f'''#include <stdio.h>
#include <stddef.h>
#include "{_lib.HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(fab_params), offsetof(fab_params, seed), offsetof(fab_params, tol),
         offsetof(fab_params, spec_lo), sizeof(fab_info), offsetof(fab_info, est_rel_update));
  return 0; }}''')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-std=c99", str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P, I = _lib.fab_params, _lib.fab_info
    want = [ctypes_size(P), P.seed.offset, P.tol.offset, P.spec_lo.offset, ctypes_size(I), I.est_rel_update.offset]
    assert got == want


def ctypes_size(t):
    import ctypes
    return ctypes.sizeof(t)


def test_package_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
