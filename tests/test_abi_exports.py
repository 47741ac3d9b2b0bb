"""The C-ABI library loads and exports every entry point that include/kgf.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kgf.h")
LIB = os.path.join(ROOT, "paper_1109_1205_amd", "libkgf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kgf_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kgf_sector_create", "kgf_apply_h", "kgf_apply_c", "kgf_ground_state",
                     "kgf_propagate", "kgf_greens_eq", "kgf_greens_neq"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkgf.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkgf.so not built")
def test_abi_version_matches_header_and_binding():
    """kgf_version (no device needed) reports the header's KGF_ABI_VERSION,
    and the binding loads only a library of the version it was written for."""
    from paper_1109_1205_amd import _lib
    m = re.search(r"#define\s+KGF_ABI_VERSION\s+(\d+)", open(HEADER).read())
    assert m
    lib = ctypes.CDLL(LIB)
    assert lib.kgf_version() == int(m.group(1)) == _lib.ABI_VERSION


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkgf.so not built")
def test_binding_signatures_cover_header():
    from paper_1109_1205_amd import _lib
    assert set(_lib.exported_symbols()) == set(declared_functions())


def test_handles_skip_native_destroy_once_their_context_is_closed(monkeypatch):
    """Model and sector destroys synchronise on their context's stream, so
    the binding calls them only while the context exists (finalisers of a
    reference cycle run in any order at interpreter shutdown)."""
    import ctypes
    from types import SimpleNamespace
    from paper_1109_1205_amd import _lib as L
    calls = []
    stub = SimpleNamespace(kgf_model_destroy=lambda h: calls.append(("model", h.value)),
                           kgf_sector_destroy=lambda h: calls.append(("sector", h.value)))
    monkeypatch.setattr(L, "_lib", stub)
    live = SimpleNamespace(handle=ctypes.c_void_p(0x10))
    gone = SimpleNamespace(handle=None)
    for cls, kind in ((L.Model, "model"), (L.Sector, "sector")):
        for ctx, expect in ((live, [(kind, 0x20)]), (gone, [])):
            calls.clear()
            obj = object.__new__(cls)
            obj.ctx, obj.handle = ctx, ctypes.c_void_p(0x20)
            obj.close()
            assert calls == expect and obj.handle is None
            obj.close()                      # idempotent
            assert calls == expect


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus N > 1 exits with a message and
    touches no device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=root, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
