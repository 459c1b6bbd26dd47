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


def test_build_options_without_device():
    """pinv_encoding_key validates build options and sizes the plan on the host.
    A factor-only plan (FLAG_NO_R) has its own cache key and needs neither W nor
    R: 2 * 8 * N * M bytes less for FP32 plans."""
    ensure_built()
    from paper_2410_06129_amd import pinv, synth
    enc = synth.small_case(seed=5, nx=12, ny=10, C=2, K=300, F=1).enc
    k_r, b_r = pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32)
    k_n, b_n = pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32, flags=pinv.FLAG_NO_R)
    assert k_r != k_n
    assert b_r - b_n == 2 * 8 * enc.N * enc.M
    for prec, flags in ((pinv.BF16X3, pinv.FLAG_NO_R), (pinv.FP32, 64)):
        try:
            pinv.pinv_encoding_key(enc, 1e-3, prec=prec, flags=flags)
        except pinv.PinvError as e:
            assert e.status == pinv.ERR_INVALID
        else:
            raise AssertionError(f"prec {prec} flags {flags} accepted")


def test_right_pseudoinverse_options_without_device():
    """Fewer samples than unknowns: the plan is sized on the M x M samples' Gram
    (Sec. 2.2); lambda = 0 is accepted (minimum-norm solution); factor-only,
    full-Gram and BF16X3 plans are refused."""
    ensure_built()
    from paper_2410_06129_amd import pinv, synth
    enc = synth.small_case(seed=6, nx=16, ny=12, C=2, K=40, F=1).enc     # M = 80 < N = 192
    N, M = enc.N, enc.M
    _, b = pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32)
    G = 16 * M * M
    assert b == 3 * G + 8 * M * M + 3 * 8 * N * M + (64 << 20)
    pinv.pinv_encoding_key(enc, 0.0, lambda_mode=pinv.LAMBDA_ABS, prec=pinv.FP64)
    for prec, flags, want in ((pinv.FP32, pinv.FLAG_NO_R, pinv.ERR_INVALID),
                              (pinv.FP32, pinv.FLAG_GRAM_FULL, pinv.ERR_INVALID),
                              (pinv.BF16X3, 0, pinv.ERR_UNSUPPORTED)):
        try:
            pinv.pinv_encoding_key(enc, 1e-3, prec=prec, flags=flags)
        except pinv.PinvError as e:
            assert e.status == want
        else:
            raise AssertionError(f"prec {prec} flags {flags} accepted")
