"""The C-ABI library loads and exports every entry point include/pinv.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2410_06129_amd", "libpinv.so")


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pinv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pinv_[a-z_]+)\s*\(", text)))


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2410_06129_amd import build
        build.build()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("pinv_context_create", "pinv_build", "pinv_plan_wait", "pinv_apply",
              "pinv_apply_grouped", "pinv_forward", "pinv_plan_release"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    ensure_built()
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    ensure_built()
    from paper_2410_06129_amd import pinv
    assert sorted(declared_symbols()) == sorted(pinv.EXPORTED)


def test_status_strings_without_device():
    ensure_built()
    from paper_2410_06129_amd import pinv
    assert pinv.pinv_status_string(pinv.ERR_NOT_PD).startswith("shifted Gram")
    assert pinv.pinv_status_string(0) == "ok"
