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


def _expect(pinv, want, fn):
    try:
        fn()
    except pinv.PinvError as e:
        assert e.status == want, (e.status, want, str(e))
    else:
        raise AssertionError("accepted")


def test_product_gram_and_r_forms_without_device():
    """Build options are validated and sized on the host: the complex-product
    form, the Gram form (PSF needs no off-resonance map), the block size (64
    only) and the FP64-formed R of FP32 plans (W held in FP64: 8 N M more bytes).
    Each form has its own cache key."""
    ensure_built()
    from paper_2410_06129_amd import pinv, synth
    enc = synth.small_case(seed=5, nx=12, ny=10, C=2, K=300, F=1).enc
    encb0 = synth.small_case(seed=6, nx=12, ny=10, C=2, K=300, F=1, b0=True).enc
    N, M = enc.N, enc.M
    keys = {pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32, cprod=c, gram=g)[0]
            for c in (pinv.CPROD_3M, pinv.CPROD_4M) for g in (pinv.GRAM_PSF, pinv.GRAM_SHARED, pinv.GRAM_FULL)}
    assert len(keys) == 6
    # AUTO resolves to 3M for FP32 plans and to the PSF form without B0
    assert (pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32)[0]
            == pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32, cprod=pinv.CPROD_3M, gram=pinv.GRAM_PSF)[0])
    assert (pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP64)[0]
            == pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP64, cprod=pinv.CPROD_4M)[0])
    assert (pinv.pinv_encoding_key(enc, 1e-3, flags=pinv.FLAG_GRAM_FULL)[0]
            == pinv.pinv_encoding_key(enc, 1e-3, gram=pinv.GRAM_FULL)[0])
    _, b32 = pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32)
    k64r, b64r = pinv.pinv_encoding_key(enc, 1e-3, prec=pinv.FP32, flags=pinv.FLAG_R_FP64)
    assert b64r - b32 == 8 * N * M
    # nb: 0 resolves to 128 (two-level); 64 is a different factorisation order
    k0 = pinv.pinv_encoding_key(enc, 1e-3)[0]
    assert k0 == pinv.pinv_encoding_key(enc, 1e-3, nb=128)[0]
    assert k0 != pinv.pinv_encoding_key(enc, 1e-3, nb=64)[0]
    pinv.pinv_encoding_key(encb0, 1e-3, gram=pinv.GRAM_SHARED)
    for want, kw, e in ((pinv.ERR_INVALID, dict(gram=pinv.GRAM_PSF), encb0),
                        (pinv.ERR_INVALID, dict(gram=9), enc),
                        (pinv.ERR_INVALID, dict(flags=pinv.FLAG_GRAM_FULL, gram=pinv.GRAM_PSF), enc),
                        (pinv.ERR_INVALID, dict(cprod=3), enc),
                        (pinv.ERR_INVALID, dict(prec=pinv.BF16X3, cprod=pinv.CPROD_3M), enc),
                        (pinv.ERR_UNSUPPORTED, dict(nb=96), enc),
                        (pinv.ERR_UNSUPPORTED, dict(nb=256), enc),
                        (pinv.ERR_INVALID, dict(prec=pinv.FP64, flags=pinv.FLAG_R_FP64), enc),
                        (pinv.ERR_INVALID, dict(flags=pinv.FLAG_R_FP64 | pinv.FLAG_NO_R), enc)):
        _expect(pinv, want, lambda: pinv.pinv_encoding_key(e, 1e-3, **kw))


def test_voxel_mask_without_device():
    """A voxel mask (Sec. 3.1, Sec. 4.4) shrinks the unknowns to N = S * nvox:
    the plan is sized on that N; unsorted or out-of-grid lists are refused."""
    ensure_built()
    import numpy as np
    from paper_2410_06129_amd import pinv, synth
    base = synth.small_case(seed=7, nx=16, ny=14, C=2, K=500, F=1).enc
    vox = synth.circular_mask(16, 14)
    masked = synth.Encoding(base.nx, base.ny, base.k, coil=base.coil, voxels=vox)
    assert masked.N == len(vox) < base.N
    k0, b0 = pinv.pinv_encoding_key(base, 1e-3, flags=pinv.FLAG_NO_R, gram=pinv.GRAM_SHARED)
    k1, b1 = pinv.pinv_encoding_key(masked, 1e-3, flags=pinv.FLAG_NO_R, gram=pinv.GRAM_SHARED)
    assert k0 != k1
    assert b0 - b1 == (3 * 16 + 8) * (base.N ** 2 - masked.N ** 2)
    for bad in (vox[::-1].copy(), np.array([0, 5, 5], np.int32), np.array([0, 16 * 14], np.int32)):
        e = synth.Encoding(base.nx, base.ny, base.k, coil=base.coil)
        e.voxels = np.ascontiguousarray(bad, dtype=np.int32)   # bypass the generator's own checks
        _expect(pinv, pinv.ERR_INVALID, lambda: pinv.pinv_encoding_key(e, 1e-3))


def test_binding_checks_tensors_before_the_call():
    """The C-ABI sees bare pointers; the binding refuses a tensor of the wrong
    dtype, shape or layout, or one not on the GPU, before calling it."""
    ensure_built()
    import pytest
    import torch
    from paper_2410_06129_amd import pinv
    info = {"prec": pinv.FP32, "N": 6, "M": 10}
    d = torch.zeros((3, 10), dtype=torch.complex64)
    x = torch.zeros((3, 6), dtype=torch.complex64)
    cases = [
        (d.to(torch.complex128), x, "dtype"),                       # FP64 data for an FP32 plan
        (torch.zeros((3, 11), dtype=torch.complex64), x, "shape"),  # wrong M
        (d, torch.zeros((2, 6), dtype=torch.complex64), "shape"),   # image frames differ
        (torch.zeros((10, 3), dtype=torch.complex64).t(), x, "contiguous"),   # transposed view
        (d, x, "not on the GPU"),                                   # host tensors
        (d.numpy(), x, "torch tensor"),                             # not a tensor
        (d[0], x, "2-D tensor"),                                    # one frame without the F axis
    ]
    for data, image, msg in cases:
        with pytest.raises(ValueError) as ei:
            pinv.check_frames("pinv_apply", info, data, image)
        assert msg in str(ei.value), (msg, str(ei.value))
    with pytest.raises(ValueError) as ei:
        pinv.check_frames("pinv_apply", dict(info, prec=pinv.FP64), d, x)
    assert "complex128" in str(ei.value)


def test_eigen_route_options_without_device():
    """The eigenvalue route (Eq. 7) with truncation (Eq. 4): options validated on
    the host; the truncation's kind and value are part of the cache key."""
    ensure_built()
    from paper_2410_06129_amd import pinv, synth
    enc = synth.small_case(seed=5, nx=12, ny=10, C=2, K=300, F=1).enc
    under = synth.small_case(seed=6, nx=16, ny=12, C=2, K=40, F=1).enc   # M < N
    E = pinv.ROUTE_EIGEN
    k1 = pinv.pinv_encoding_key(enc, 0.0, pinv.LAMBDA_ABS, route=E, trunc=pinv.TRUNC_KAPPA,
                                trunc_value=30.0)[0]
    k2 = pinv.pinv_encoding_key(enc, 0.0, pinv.LAMBDA_ABS, route=E, trunc=pinv.TRUNC_KAPPA,
                                trunc_value=40.0)[0]
    k3 = pinv.pinv_encoding_key(enc, 0.0, pinv.LAMBDA_ABS, route=E, trunc=pinv.TRUNC_ENERGY,
                                trunc_value=0.95)[0]
    k4 = pinv.pinv_encoding_key(enc, 1e-3, route=E)[0]
    k5 = pinv.pinv_encoding_key(enc, 1e-3)[0]
    assert len({k1, k2, k3, k4, k5}) == 5
    for want, kw, e in ((pinv.ERR_INVALID, dict(trunc=pinv.TRUNC_KAPPA, trunc_value=30.0), enc),
                        (pinv.ERR_INVALID, dict(route=E, trunc=pinv.TRUNC_KAPPA, trunc_value=0.5), enc),
                        (pinv.ERR_INVALID, dict(route=E, trunc=pinv.TRUNC_ENERGY, trunc_value=0.0), enc),
                        (pinv.ERR_INVALID, dict(route=E, trunc=pinv.TRUNC_ENERGY, trunc_value=1.5), enc),
                        (pinv.ERR_INVALID, dict(route=E, trunc=5), enc),
                        (pinv.ERR_INVALID, dict(route=2), enc),
                        (pinv.ERR_UNSUPPORTED, dict(route=E, prec=pinv.BF16X3), enc),
                        (pinv.ERR_INVALID, dict(route=E, flags=pinv.FLAG_NO_R), enc),
                        (pinv.ERR_UNSUPPORTED, dict(route=E), under)):
        _expect(pinv, want, lambda: pinv.pinv_encoding_key(e, 1e-3, **kw))
