"""ctypes binding of libpinv_schedsim.so: the serving scheduler on a
simulated device with a virtual clock (CPU only; used by the tests)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpinv_schedsim.so")
STAT_FIELDS = ["builds", "build_failures", "evictions", "hits", "batches", "items", "completed",
               "invariant_violations", "used", "peak_used", "budget", "use_after_release"]


def _load():
    if not os.path.exists(LIB_PATH):
        from . import build
        build.build_sim()
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, sz, d = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
    lib.sim_create.argtypes = [sz, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.sim_create.restype = vp
    lib.sim_submit.argtypes = [vp, u64, sz, sz, d, d, ctypes.c_int, u64]
    lib.sim_submit.restype = u64
    lib.sim_advance.argtypes = [vp, d]
    lib.sim_idle.argtypes = [vp]
    lib.sim_now.argtypes = [vp]
    lib.sim_now.restype = d
    P = ctypes.POINTER
    lib.sim_completions.argtypes = [vp, P(u64), P(u64), P(ctypes.c_int), P(ctypes.c_int), P(d),
                                    P(d), P(d), ctypes.c_int]
    lib.sim_stats.argtypes = [vp, P(u64)]
    lib.sim_destroy.argtypes = [vp]
    return lib


_lib = _load()


class Sim:
    def __init__(self, budget, max_group=32, max_inflight=2, max_builds=1):
        self.h = _lib.sim_create(budget, max_group, max_inflight, max_builds)

    def submit(self, key, footprint, resident, build_s, apply_s, fail=False, tag=0):
        return _lib.sim_submit(self.h, key, footprint, resident, build_s, apply_s, int(fail), tag)

    def advance(self, dt):
        _lib.sim_advance(self.h, dt)

    @property
    def now(self):
        return _lib.sim_now(self.h)

    def idle(self):
        return bool(_lib.sim_idle(self.h))

    def completions(self, max_n=4096):
        u = (ctypes.c_uint64 * max_n)
        i = (ctypes.c_int * max_n)
        f = (ctypes.c_double * max_n)
        t, g, st, b, a, dsp, dn = u(), u(), i(), i(), f(), f(), f()
        n = _lib.sim_completions(self.h, t, g, st, b, a, dsp, dn, max_n)
        return [dict(ticket=t[k], tag=g[k], status=st[k], built=bool(b[k]), t_arrival=a[k],
                     t_dispatch=dsp[k], t_done=dn[k]) for k in range(n)]

    def stats(self):
        out = (ctypes.c_uint64 * len(STAT_FIELDS))()
        _lib.sim_stats(self.h, out)
        return dict(zip(STAT_FIELDS, list(out)))

    def close(self):
        if self.h:
            _lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
