"""Thin ctypes binding of libpinv (include/pinv.h): argument marshalling only.

Every function here forwards to the C entry point of the same name.  Device
buffers are passed as torch tensors (their data_ptr) and streams as
torch.cuda streams; torch only provides device memory and streams.  There is
no fallback: importing this module raises if libpinv.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpinv.so")

OK, ERR_INVALID, ERR_NOMEM, ERR_NOT_PD, ERR_DEVICE, ERR_BUSY, ERR_UNSUPPORTED = range(7)
FP64, FP32, BF16X3 = 0, 1, 2
LAMBDA_ABS, LAMBDA_REL_MEAN_DIAG = 0, 1
FLAG_KEEP_GRAM = 1
FLAG_UNCACHED = 2
FLAG_GRAM_FULL = 4
FLAG_NO_R = 8
FLAG_R_FP64 = 16
CPROD_AUTO, CPROD_3M, CPROD_4M = 0, 1, 2
GRAM_AUTO, GRAM_PSF, GRAM_SHARED, GRAM_FULL = 0, 1, 2, 3
ROUTE_CHOLESKY, ROUTE_EIGEN = 0, 1
TRUNC_NONE, TRUNC_KAPPA, TRUNC_ENERGY = 0, 1, 2
BUF_R, BUF_LINV, BUF_GRAM = 0, 1, 2
METRIC_DIAG, METRIC_FULL = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first "
                      "(python -c 'import __graft_entry__ as g; g.build()')")
_lib = ctypes.CDLL(LIB_PATH)

_dp = ctypes.POINTER(ctypes.c_double)


class pinv_encoding(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nk", ctypes.c_int64),
                ("k", _dp), ("t", _dp), ("ncoil", ctypes.c_int32), ("coil", _dp),
                ("b0_hz", _dp), ("nspecies", ctypes.c_int32), ("species_hz", _dp),
                ("voxels", ctypes.POINTER(ctypes.c_int32)), ("nvox", ctypes.c_int32)]


class pinv_build_opts(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("lambda_mode", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("flags", ctypes.c_int32), ("cprod", ctypes.c_int32),
                ("nb", ctypes.c_int32), ("gram", ctypes.c_int32), ("route", ctypes.c_int32),
                ("trunc", ctypes.c_int32), ("trunc_value", ctypes.c_double)]


class pinv_plan_info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("M", ctypes.c_int64), ("lambda_abs", ctypes.c_double),
                ("prec", ctypes.c_int32), ("ready", ctypes.c_int32), ("key", ctypes.c_uint64),
                ("device_bytes", ctypes.c_size_t), ("stage_ms", ctypes.c_float * 4),
                ("has_r", ctypes.c_int32), ("gram_order", ctypes.c_int64),
                ("ncoil", ctypes.c_int32), ("cprod", ctypes.c_int32), ("nk", ctypes.c_int64),
                ("gram_form", ctypes.c_int32), ("r_fp64", ctypes.c_int32),
                ("route", ctypes.c_int32), ("rank", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class pinv_apply_item(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("data", ctypes.c_void_p), ("image", ctypes.c_void_p),
                ("F", ctypes.c_int64)]


class pinv_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_group", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("max_builds", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class pinv_request(ctypes.Structure):
    _fields_ = [("enc", ctypes.POINTER(pinv_encoding)), ("opts", pinv_build_opts),
                ("data", ctypes.c_void_p), ("image", ctypes.c_void_p), ("F", ctypes.c_int64),
                ("refine_steps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tag", ctypes.c_uint64)]


class pinv_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("built", ctypes.c_int32), ("t_arrival", ctypes.c_double),
                ("t_dispatch", ctypes.c_double), ("t_done", ctypes.c_double)]


class pinv_server_stats(ctypes.Structure):
    _fields_ = [("builds", ctypes.c_uint64), ("build_failures", ctypes.c_uint64),
                ("evictions", ctypes.c_uint64), ("hits", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("items", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("invariant_violations", ctypes.c_uint64),
                ("used", ctypes.c_size_t), ("peak_used", ctypes.c_size_t),
                ("budget", ctypes.c_size_t), ("cached_plans", ctypes.c_int32),
                ("pending", ctypes.c_int32), ("running", ctypes.c_int32)]


_vp = ctypes.c_void_p
_sigs = {
    "pinv_context_create": [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_vp)],
    "pinv_context_destroy": [_vp],
    "pinv_build": [_vp, ctypes.POINTER(pinv_encoding), ctypes.POINTER(pinv_build_opts), _vp,
                   ctypes.POINTER(_vp)],
    "pinv_plan_wait": [_vp],
    "pinv_apply": [_vp, _vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, _vp],
    "pinv_apply_grouped": [_vp, ctypes.c_int32, ctypes.POINTER(pinv_apply_item), ctypes.c_int32, _vp],
    "pinv_apply_noalloc": [_vp, _vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, _vp],
    "pinv_forward": [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp],
    "pinv_srf": [_vp, _vp, ctypes.c_int32, _vp, _vp],
    "pinv_noise": [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp],
    "pinv_plan_info_get": [_vp, ctypes.POINTER(pinv_plan_info)],
    "pinv_spectrum": [_vp, _vp, _vp, _vp],
    "pinv_plan_buffers": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
    "pinv_plan_copy_buffer": [_vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp],
    "pinv_plan_release": [_vp],
    "pinv_cache_trim": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "pinv_context_usage": [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                           ctypes.POINTER(ctypes.c_int32)],
    "pinv_plan_query": [_vp],
    "pinv_context_trim": [_vp],
    "pinv_encoding_key": [ctypes.POINTER(pinv_encoding), ctypes.POINTER(pinv_build_opts),
                          ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_size_t)],
    "pinv_server_create": [_vp, ctypes.c_int, ctypes.POINTER(pinv_server_opts), ctypes.POINTER(_vp)],
    "pinv_server_submit": [_vp, ctypes.POINTER(pinv_request), ctypes.POINTER(ctypes.c_uint64)],
    "pinv_server_poll": [_vp, ctypes.POINTER(pinv_completion), ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_int32)],
    "pinv_server_drain": [_vp, ctypes.c_double],
    "pinv_server_stats_get": [_vp, ctypes.POINTER(pinv_server_stats)],
    "pinv_server_destroy": [_vp],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.pinv_status_string.argtypes = [ctypes.c_int]
_lib.pinv_status_string.restype = ctypes.c_char_p
_lib.pinv_last_error.argtypes = []
_lib.pinv_last_error.restype = ctypes.c_char_p

EXPORTED = sorted(list(_sigs) + ["pinv_status_string", "pinv_last_error"])


class PinvError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.pinv_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.pinv_status_string(status).decode()} ({msg})")


def _check(st: int, where: str):
    if st != OK:
        raise PinvError(st, where)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


# ----------------------------------------------------------------------------
# host-side argument checks.  The C-ABI receives bare device pointers and
# cannot see a tensor's dtype, shape, layout or device, so a mismatch (a
# complex64 tensor for an FP64 plan, a transposed view, a short buffer) would
# make the kernels read or write past the end of device memory.  Every call
# that passes tensors checks them here first and raises ValueError.
# ----------------------------------------------------------------------------

_ctx_device = {}     # context handle -> HIP device index


def _complex_dtype(prec: int):
    import torch
    return torch.complex128 if prec == FP64 else torch.complex64


def _real_dtype(prec: int):
    import torch
    return torch.float64 if prec == FP64 else torch.float32


def _check_layout(where: str, name: str, t, shape, dtype) -> None:
    if not hasattr(t, "data_ptr") or not hasattr(t, "is_contiguous"):
        raise ValueError(f"{where}: {name} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{where}: {name} has dtype {t.dtype}, the plan needs {dtype}")
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{where}: {name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{where}: {name} must be contiguous (row-major); call .contiguous()")


def _check_device(where: str, name: str, t, device: Optional[int]) -> None:
    if not t.is_cuda:
        raise ValueError(f"{where}: {name} is on {t.device}, not on the GPU")
    if device is not None and t.device.index is not None and t.device.index != device:
        raise ValueError(f"{where}: {name} is on cuda:{t.device.index}, the context on cuda:{device}")


def check_tensor(where: str, name: str, t, shape, dtype, device: Optional[int]) -> None:
    """Raise ValueError unless `t` is a contiguous tensor of `dtype` and `shape`
    on HIP device `device` (any device when None)."""
    _check_layout(where, name, t, shape, dtype)
    _check_device(where, name, t, device)


def check_frames(where: str, info: dict, data, image, device: Optional[int] = None) -> int:
    """data [F, M] and image [F, N] in the plan's complex type; returns F."""
    cdt = _complex_dtype(info["prec"])
    if not hasattr(data, "shape") or len(data.shape) != 2:
        raise ValueError(f"{where}: data must be a 2-D tensor [F, M]")
    F = int(data.shape[0])
    _check_layout(where, "data", data, (F, info["M"]), cdt)
    _check_layout(where, "image", image, (F, info["N"]), cdt)
    _check_device(where, "data", data, device)
    _check_device(where, "image", image, device)
    return F


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------

def pinv_context_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    out = _vp()
    _check(_lib.pinv_context_create(device, hbm_budget_bytes, ctypes.byref(out)), "pinv_context_create")
    _ctx_device[out.value] = device
    return out.value


def pinv_context_destroy(ctx: int) -> None:
    _check(_lib.pinv_context_destroy(ctx), "pinv_context_destroy")
    _ctx_device.pop(ctx, None)


def _encoding_struct(enc):
    """Marshal an encoding (synth.Encoding-like object) into pinv_encoding.
    Returns the struct and the arrays it points into (keep them alive)."""
    k = np.ascontiguousarray(enc.k, dtype=np.float64)
    keep = [k]
    t = None if enc.t is None else np.ascontiguousarray(enc.t, dtype=np.float64)
    coil = None
    if enc.coil is not None:
        c = np.ascontiguousarray(enc.coil, dtype=np.complex128)
        coil = np.ascontiguousarray(c.view(np.float64))
    b0 = None if enc.b0_hz is None else np.ascontiguousarray(enc.b0_hz, dtype=np.float64)
    sp = None if enc.species_hz is None else np.ascontiguousarray(enc.species_hz, dtype=np.float64)
    vox = getattr(enc, "voxels", None)
    vox = None if vox is None else np.ascontiguousarray(vox, dtype=np.int32)
    keep += [t, coil, b0, sp, vox]
    s = pinv_encoding(nx=enc.nx, ny=enc.ny, nk=k.shape[0], k=_ptr(k), t=_ptr(t),
                      ncoil=1 if coil is None else enc.coil.shape[0], coil=_ptr(coil),
                      b0_hz=_ptr(b0), nspecies=1 if sp is None else len(sp), species_hz=_ptr(sp),
                      voxels=None if vox is None else vox.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      nvox=0 if vox is None else len(vox))
    return s, keep


def _opts(lam, lambda_mode, prec, flags, cprod, nb, gram, route=ROUTE_CHOLESKY, trunc=TRUNC_NONE,
          trunc_value=0.0):
    return pinv_build_opts(lambda_=lam, lambda_mode=lambda_mode, prec=prec, flags=flags,
                           cprod=cprod, nb=nb, gram=gram, route=route, trunc=trunc,
                           trunc_value=trunc_value)


def pinv_build(ctx: int, enc, lam: float, lambda_mode: int = LAMBDA_REL_MEAN_DIAG,
               prec: int = FP32, flags: int = 0, stream=None, cprod: int = CPROD_AUTO, nb: int = 0,
               gram: int = GRAM_AUTO, route: int = ROUTE_CHOLESKY, trunc: int = TRUNC_NONE,
               trunc_value: float = 0.0) -> int:
    s, keep = _encoding_struct(enc)
    o = _opts(lam, lambda_mode, prec, flags, cprod, nb, gram, route, trunc, trunc_value)
    out = _vp()
    st = _lib.pinv_build(ctx, ctypes.byref(s), ctypes.byref(o), _stream_ptr(stream), ctypes.byref(out))
    del keep
    _check(st, "pinv_build")
    return out.value


def pinv_plan_wait(plan: int) -> None:
    _check(_lib.pinv_plan_wait(plan), "pinv_plan_wait")


def pinv_plan_wait_status(plan: int) -> int:
    return _lib.pinv_plan_wait(plan)


def pinv_apply(ctx: int, plan: int, data, image, refine_steps: int = 0, stream=None) -> None:
    """data: device tensor [F, M], image: device tensor [F, N] (complex64 or complex128)."""
    F = check_frames("pinv_apply", pinv_plan_info_get(plan), data, image, _ctx_device.get(ctx))
    _check(_lib.pinv_apply(ctx, plan, data.data_ptr(), F, image.data_ptr(), refine_steps,
                           _stream_ptr(stream)), "pinv_apply")


def pinv_apply_noalloc(ctx: int, plan: int, data, image, refine_steps: int = 0, stream=None) -> None:
    """pinv_apply with its scratch from the library's fixed per-GPU region (no
    device allocation); calls on one GPU must not overlap."""
    F = check_frames("pinv_apply_noalloc", pinv_plan_info_get(plan), data, image,
                     _ctx_device.get(ctx))
    _check(_lib.pinv_apply_noalloc(ctx, plan, data.data_ptr(), F, image.data_ptr(), refine_steps,
                                   _stream_ptr(stream)), "pinv_apply_noalloc")


def pinv_apply_grouped(ctx: int, items: Sequence[tuple], refine_steps: int = 0, stream=None) -> None:
    """items: sequence of (plan, data tensor, image tensor)."""
    arr = (pinv_apply_item * len(items))()
    dev = _ctx_device.get(ctx)
    for i, (plan, d, x) in enumerate(items):
        F = check_frames(f"pinv_apply_grouped item {i}", pinv_plan_info_get(plan), d, x, dev)
        arr[i] = pinv_apply_item(plan, d.data_ptr(), x.data_ptr(), F)
    _check(_lib.pinv_apply_grouped(ctx, len(items), arr, refine_steps, _stream_ptr(stream)),
           "pinv_apply_grouped")


def pinv_forward(ctx: int, plan: int, image, data, stream=None) -> None:
    """data = E image (Eq. 1): image [F, N] -> data [F, M], in the plan's type."""
    info = pinv_plan_info_get(plan)
    if not hasattr(image, "shape") or len(image.shape) != 2:
        raise ValueError("pinv_forward: image must be a 2-D tensor [F, N]")
    F = int(image.shape[0])
    cdt = _complex_dtype(info["prec"])
    dev = _ctx_device.get(ctx)
    check_tensor("pinv_forward", "image", image, (F, info["N"]), cdt, dev)
    check_tensor("pinv_forward", "data", data, (F, info["M"]), cdt, dev)
    _check(_lib.pinv_forward(ctx, plan, image.data_ptr(), F, data.data_ptr(),
                             _stream_ptr(stream)), "pinv_forward")


def pinv_srf(ctx: int, plan: int, out, mode: int = METRIC_DIAG, stream=None) -> None:
    """SRF = R E (Eq. 9): its diagonal (mode METRIC_DIAG, out [N]) or the
    full matrix (METRIC_FULL, out [N, N]); complex, in the plan's precision."""
    info = pinv_plan_info_get(plan)
    N = info["N"]
    if mode in (METRIC_DIAG, METRIC_FULL):   # other modes: the library reports INVALID
        shape = (N,) if mode == METRIC_DIAG else (N, N)
        check_tensor("pinv_srf", "out", out, shape, _complex_dtype(info["prec"]), _ctx_device.get(ctx))
    _check(_lib.pinv_srf(ctx, plan, mode, out.data_ptr(), _stream_ptr(stream)), "pinv_srf")


def pinv_noise(ctx: int, plan: int, out, coil_cov=None, mode: int = METRIC_DIAG,
               stream=None) -> None:
    """Noise matrix X = R (Psi_c kron I) R^H (Eq. 10): diag(X) (METRIC_DIAG, real
    out [N]) or X (METRIC_FULL, complex out [N, N]).  coil_cov: [C, C] Hermitian
    positive definite, or None for white noise."""
    info = pinv_plan_info_get(plan)
    N = info["N"]
    if mode == METRIC_DIAG:
        check_tensor("pinv_noise", "out", out, (N,), _real_dtype(info["prec"]), _ctx_device.get(ctx))
    elif mode == METRIC_FULL:
        check_tensor("pinv_noise", "out", out, (N, N), _complex_dtype(info["prec"]),
                     _ctx_device.get(ctx))
    cov = None
    if coil_cov is not None:
        cov = np.ascontiguousarray(np.asarray(coil_cov, dtype=np.complex128))
        C = info["ncoil"]
        if cov.shape != (C, C):
            raise ValueError(f"pinv_noise: coil_cov must be [{C}, {C}] (the plan's coils), "
                             f"got {cov.shape}")
    _check(_lib.pinv_noise(ctx, plan, None if cov is None else cov.ctypes.data, mode,
                           out.data_ptr(), _stream_ptr(stream)), "pinv_noise")


def pinv_plan_info_get(plan: int) -> dict:
    i = pinv_plan_info()
    _check(_lib.pinv_plan_info_get(plan, ctypes.byref(i)), "pinv_plan_info_get")
    return dict(N=i.N, M=i.M, lambda_abs=i.lambda_abs, prec=i.prec, ready=bool(i.ready),
                key=i.key, device_bytes=i.device_bytes, stage_ms=list(i.stage_ms),
                has_r=bool(i.has_r), gram_order=i.gram_order, ncoil=i.ncoil, cprod=i.cprod,
                nk=i.nk, gram_form=i.gram_form, r_fp64=bool(i.r_fp64), route=i.route,
                rank=i.rank, sweeps=i.sweeps)


def pinv_spectrum(ctx: int, plan: int, out, stream=None) -> None:
    """Eigenvalues of E^H E, largest first, of an eigenvalue-route plan: out is
    a device float64 tensor [N]."""
    import torch
    info = pinv_plan_info_get(plan)
    check_tensor("pinv_spectrum", "out", out, (info["N"],), torch.float64, _ctx_device.get(ctx))
    _check(_lib.pinv_spectrum(ctx, plan, out.data_ptr(), _stream_ptr(stream)), "pinv_spectrum")


def pinv_plan_buffers(plan: int):
    r, l, g = _vp(), _vp(), _vp()
    _check(_lib.pinv_plan_buffers(plan, ctypes.byref(r), ctypes.byref(l), ctypes.byref(g)),
           "pinv_plan_buffers")
    return r.value, l.value, g.value


def pinv_plan_copy_buffer(plan: int, which: int, dst, stream=None) -> None:
    """Copy R, L^-1 or the Gram into `dst` (contiguous device tensor of exactly
    the buffer's size; the library checks the byte count)."""
    if not hasattr(dst, "is_contiguous") or not dst.is_contiguous() or not dst.is_cuda:
        raise ValueError("pinv_plan_copy_buffer: dst must be a contiguous GPU tensor")
    nbytes = dst.numel() * dst.element_size()
    _check(_lib.pinv_plan_copy_buffer(plan, which, dst.data_ptr(), nbytes, _stream_ptr(stream)),
           "pinv_plan_copy_buffer")


def pinv_plan_release(plan: int) -> None:
    _check(_lib.pinv_plan_release(plan), "pinv_plan_release")


def pinv_cache_trim(ctx: int) -> int:
    f = ctypes.c_size_t()
    _check(_lib.pinv_cache_trim(ctx, ctypes.byref(f)), "pinv_cache_trim")
    return f.value


def pinv_context_usage(ctx: int):
    u, b, n = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int32()
    _check(_lib.pinv_context_usage(ctx, ctypes.byref(u), ctypes.byref(b), ctypes.byref(n)),
           "pinv_context_usage")
    return u.value, b.value, n.value


def pinv_status_string(s: int) -> str:
    return _lib.pinv_status_string(s).decode()


def pinv_last_error() -> str:
    return _lib.pinv_last_error().decode(errors="replace")


def pinv_plan_query(plan: int) -> int:
    """Non-blocking build state: OK, ERR_BUSY, or the failure status."""
    return _lib.pinv_plan_query(plan)


def pinv_context_trim(ctx: int) -> None:
    _check(_lib.pinv_context_trim(ctx), "pinv_context_trim")


def pinv_encoding_key(enc, lam: float, lambda_mode: int = LAMBDA_REL_MEAN_DIAG, prec: int = FP32,
                      flags: int = 0, cprod: int = CPROD_AUTO, nb: int = 0, gram: int = GRAM_AUTO,
                      route: int = ROUTE_CHOLESKY, trunc: int = TRUNC_NONE, trunc_value: float = 0.0):
    s, keep = _encoding_struct(enc)
    o = _opts(lam, lambda_mode, prec, flags, cprod, nb, gram, route, trunc, trunc_value)
    k, b = ctypes.c_uint64(), ctypes.c_size_t()
    st = _lib.pinv_encoding_key(ctypes.byref(s), ctypes.byref(o), ctypes.byref(k), ctypes.byref(b))
    del keep
    _check(st, "pinv_encoding_key")
    return k.value, b.value


# ----------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------

def pinv_server_create(ctx: int, device: int = 0, hbm_budget_bytes: int = 0, max_group: int = 32,
                       max_inflight: int = 2, max_builds: int = 1) -> int:
    o = pinv_server_opts(hbm_budget_bytes=hbm_budget_bytes, max_group=max_group,
                         max_inflight=max_inflight, max_builds=max_builds, reserved=0)
    out = _vp()
    _check(_lib.pinv_server_create(ctx, device, ctypes.byref(o), ctypes.byref(out)), "pinv_server_create")
    return out.value


def pinv_server_submit(server: int, enc, data, image, lam: float = 1e-3,
                       lambda_mode: int = LAMBDA_REL_MEAN_DIAG, prec: int = FP32, flags: int = 0,
                       refine_steps: int = 0, tag: int = 0, cprod: int = CPROD_AUTO,
                       gram: int = GRAM_AUTO) -> int:
    """data/image: device tensors [F, M] / [F, N], kept alive by the caller until completion."""
    check_frames("pinv_server_submit", {"prec": prec, "N": enc.N, "M": enc.M}, data, image)
    s, keep = _encoding_struct(enc)
    o = _opts(lam, lambda_mode, prec, flags, cprod, 0, gram)
    r = pinv_request(enc=ctypes.pointer(s), opts=o, data=data.data_ptr(), image=image.data_ptr(),
                     F=data.shape[0], refine_steps=refine_steps, reserved=0, tag=tag)
    t = ctypes.c_uint64()
    st = _lib.pinv_server_submit(server, ctypes.byref(r), ctypes.byref(t))
    del keep
    _check(st, "pinv_server_submit")
    return t.value


def pinv_server_poll(server: int, max_n: int = 256):
    arr = (pinv_completion * max_n)()
    n = ctypes.c_int32()
    _check(_lib.pinv_server_poll(server, arr, max_n, ctypes.byref(n)), "pinv_server_poll")
    return [dict(ticket=c.ticket, tag=c.tag, status=c.status, built=bool(c.built),
                 t_arrival=c.t_arrival, t_dispatch=c.t_dispatch, t_done=c.t_done)
            for c in arr[:n.value]]


def pinv_server_drain(server: int, timeout_s: float = 0.0) -> int:
    return _lib.pinv_server_drain(server, timeout_s)


def pinv_server_stats_get(server: int) -> dict:
    s = pinv_server_stats()
    _check(_lib.pinv_server_stats_get(server, ctypes.byref(s)), "pinv_server_stats_get")
    return {f: getattr(s, f) for f, _ in pinv_server_stats._fields_}


def pinv_server_destroy(server: int) -> None:
    _check(_lib.pinv_server_destroy(server), "pinv_server_destroy")
