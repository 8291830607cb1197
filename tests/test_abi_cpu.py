"""The C-ABI library loads and exports every symbol include/sdd.h declares,
the binding's struct layouts match the header, and the product package does
not reach the oracle.  No compute calls (no GPU here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1603_09311_amd import sdd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdd_[a-z_]+)\s*\(", text)))


def test_header_declares_what_binding_binds():
    assert declared_functions() == sorted(sdd.EXPORTED)


@pytest.mark.skipif(not os.path.exists(sdd.LIB_PATH), reason="libsdd.so not built")
def test_library_exports_every_declared_symbol():
    L = C.CDLL(sdd.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", sdd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (sdd_[a-z_]+)$", nm, flags=re.M))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(sdd.LIB_PATH), reason="libsdd.so not built")
def test_library_has_no_unresolved_own_symbols():
    """Every function of the library's own namespace is defined in it (a
    shared object links with undefined symbols and fails only when loaded)."""
    nm = subprocess.run(["nm", "-D", "--undefined-only", sdd.LIB_PATH], capture_output=True, text=True).stdout
    own = [ln for ln in nm.splitlines() if "3sdd" in ln or " sdd_" in ln]
    assert not own, own


def test_status_strings_and_errors_without_gpu():
    L = sdd.lib()
    assert L.sdd_status_string(0) == b"ok"
    assert L.sdd_status_string(-2) == b"workspace exhausted"
    h = C.c_void_p()
    # a NULL workspace is rejected before any device call
    assert L.sdd_create(0, None, 0, None, C.byref(h)) == sdd.SDD_E_INVALID
    assert b"workspace" in L.sdd_last_error()
    assert L.sdd_destroy(None) == sdd.SDD_E_INVALID


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "sdd.h"\nint main(void){\n'
                   'printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(sdd_region), sizeof(sdd_model_desc),'
                   ' sizeof(sdd_request), sizeof(sdd_result), sizeof(sdd_path_record), sizeof(sdd_tuning),'
                   ' sizeof(sdd_tune_trial), sizeof(sdd_stats));\n'
                   'printf("%zu %zu %zu %zu\\n", offsetof(sdd_request, dt), offsetof(sdd_request, target_rel_se),'
                   ' offsetof(sdd_result, path_records), offsetof(sdd_model_desc, regions));\n'
                   'printf("%zu %zu %zu %zu\\n", sizeof(sdd_kappa_request), offsetof(sdd_kappa_request, g_tables),'
                   ' offsetof(sdd_kappa_request, dt), offsetof(sdd_kappa_request, precision));\n'
                   'printf("%zu %zu %zu %zu\\n", sizeof(sdd_diag), offsetof(sdd_diag, flags), offsetof(sdd_diag, g_norm),'
                   ' offsetof(sdd_result, diag));\n'
                   'printf("%u\\n", (unsigned)SDD_NOALLOC_SCRATCH_BYTES);\nreturn 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    a, b, c, d, e = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")[:5]
    want = [C.sizeof(t) for t in (sdd.sdd_region, sdd.sdd_model_desc, sdd.sdd_request, sdd.sdd_result,
                                  sdd.sdd_path_record, sdd.sdd_tuning, sdd.sdd_tune_trial, sdd.sdd_stats)]
    assert [int(x) for x in a.split()] == want
    offs = [sdd.sdd_request.dt.offset, sdd.sdd_request.target_rel_se.offset, sdd.sdd_result.path_records.offset,
            sdd.sdd_model_desc.regions.offset]
    assert [int(x) for x in b.split()] == offs
    K = sdd.sdd_kappa_request
    assert [int(x) for x in c.split()] == [C.sizeof(K), K.g_tables.offset, K.dt.offset, K.precision.offset]
    D = sdd.sdd_diag
    assert [int(x) for x in d.split()] == [C.sizeof(D), D.flags.offset, D.g_norm.offset, sdd.sdd_result.diag.offset]
    assert int(e) == sdd.SDD_NOALLOC_SCRATCH_BYTES


def test_product_path_never_reaches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1603_09311_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h", ".hpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "workloads.py" and "oracle" not in re.sub(
                    r'""".*?"""', "", text, flags=re.S).lower(), f


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sdd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sdd, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        sdd.lib()
