"""Python binding of libpfmi (argument marshalling only).

Every function here forwards to the C ABI of the same name (include/pfmi.h);
all computation runs in the library's HIP kernels.  The library must be built
(``python -m paper_2511_10508_amd.build``); importing raises if it is missing
— there is no CPU fallback.

PyTorch, when importable, is imported first so that the process holds one HIP
runtime: libpfmi then binds to the libamdhip64 that torch already loaded, and
torch tensors and streams can be handed to pf_create_on.
"""
import ctypes
import os

import numpy as np

try:  # one HIP runtime per process: let torch load it first when present
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional for the binding
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libpfmi.so")

PF_OK, PF_ERR_ARG, PF_ERR_UNSTABLE, PF_ERR_NOMEM, PF_ERR_DEVICE = 0, 1, 2, 3, 4
PF_ERR_STATE, PF_ERR_UNSUPPORTED, PF_ERR_BUSY, PF_ERR_NOTFOUND = 5, 6, 7, 8
PF_AC, PF_CH, PF_GS, PF_MC, PF_MH = 1, 2, 3, 4, 5
PF_FP64, PF_FP32 = 0, 1
PF_ALLOW_UNSTABLE, PF_USE_GRAPH, PF_REDUCE_EACH_STEP, PF_FORCE_GENERIC = 1, 2, 4, 8
PF_BIHARMONIC_DIRECT = 16
PF_SPECTRAL = 32
PF_IC_UNIFORM, PF_IC_GS_CUBES, PF_IC_CONST = 1, 2, 3
PF_RED_MASS0, PF_RED_MASS1, PF_RED_ENERGY, PF_RED_NONFINITE = 0, 1, 2, 3


class pf_desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("kind", ctypes.c_int32),
                ("nfields", ctypes.c_int32), ("ndim", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("order", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("nparams", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("params", ctypes.c_double * 8)]


class pf_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("mass", ctypes.c_double * 2),
                ("energy", ctypes.c_double), ("nonfinite", ctypes.c_int64),
                ("steps_done", ctypes.c_int64)]


class PfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


_P = ctypes.POINTER
_vp, _i32, _i64, _u32, _u64, _d = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
_pd, _pi64, _pi32 = _P(_d), _P(_i64), _P(_i32)

# name: (restype, argtypes) — the whole exported surface of include/pfmi.h
SIGNATURES = {
    "pf_abi_version": (_i32, []),
    "pf_last_error": (ctypes.c_char_p, []),
    "pf_status_str": (ctypes.c_char_p, [_i32]),
    "pf_weights": (_i32, [_i32, _pd]),
    "pf_weights4": (_i32, [_i32, _pd]),
    "pf_weights1": (_i32, [_i32, _pd]),
    "pf_stability": (_i32, [_P(pf_desc), _pd]),
    "pf_footprint_bytes": (_u64, [_P(pf_desc)]),
    "pf_buffer_elems": (_i64, [_P(pf_desc)]),
    "pf_create": (_i32, [_P(pf_desc), _vp, _P(_vp)]),
    "pf_create_on": (_i32, [_P(pf_desc), _vp, _P(_vp), _i32, _P(_vp)]),
    "pf_destroy": (None, [_vp]),
    "pf_init": (_i32, [_vp, _i32, _u64, _pd, _i32]),
    "pf_set_field": (_i32, [_vp, _i32, _pd, _i64]),
    "pf_get_field": (_i32, [_vp, _i32, _pd, _i64]),
    "pf_get_window": (_i32, [_vp, _i32, _pi64, _pi64, _pd]),
    "pf_field_device": (_i32, [_vp, _i32, _P(_vp), _pi64, _pi32]),
    "pf_step": (_i32, [_vp, _i64]),
    "pf_step_noalloc": (_i32, [_P(pf_desc), _vp, _P(_vp), _i32, _i32, _i64, _vp]),
    "pf_reduce": (_i32, [_vp, _i32, _pd, _pd]),
    "pf_reduce_history": (_i32, [_vp, _i32, _pd, _pd, _i64]),
    "pf_sync": (_i32, [_vp]),
    "pf_steps_done": (_i64, [_vp]),
    "pf_set_steps_done": (_i32, [_vp, _i64]),
    "pf_stream": (_i32, [_vp, _P(_vp)]),
    "pf_set_tile": (_i32, [_vp, _i32]),
    "pf_get_tile": (_i32, [_vp, _pi32, _pi32]),
    "pf_set_time_block": (_i32, [_vp, _i32]),
    "pf_get_time_block": (_i32, [_vp]),
    "pf_set_tile_rows": (_i32, [_vp, _i32]),
    "pf_get_tile_rows": (_i32, [_vp]),
    "pf_set_passes": (_i32, [_vp, _i32]),
    "pf_get_passes": (_i32, [_vp]),
    "pf_autotune": (_i32, [_vp, _i32]),
    "pf_timing_enable": (_i32, [_vp, _i32]),
    "pf_timing_read": (_i32, [_vp, _pd, _pi64, _pi64]),
    "pf_copy_probe": (_i32, [_vp, _vp, _u64, _vp, _i32, _pd]),
    "pf_server_create": (_i32, [_i32, _u64, _i32, _i32, _P(_vp)]),
    "pf_server_submit": (_i32, [_vp, _P(pf_desc), _i32, _u64, _pd, _i32, _i64, _P(_u64)]),
    "pf_server_poll": (_i32, [_vp, _P(pf_result), _i32, _pi32]),
    "pf_server_fetch": (_i32, [_vp, _u64, _i32, _pd, _i64]),
    "pf_server_release": (_i32, [_vp, _u64]),
    "pf_server_cancel": (_i32, [_vp, _u64]),
    "pf_server_drain": (_i32, [_vp, _d]),
    "pf_server_stats": (_i32, [_vp, _pi64, _pi64, _pi64, _pi64]),
    "pf_server_destroy": (None, [_vp]),
}

_lib = None


def hip_runtimes_mapped():
    """Paths of libamdhip64 images mapped into this process."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 6 and "libamdhip64" in parts[5]:
                paths.add(os.path.realpath(parts[5]))
    return sorted(paths)


def lib():
    """Load libpfmi.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError("libpfmi.so is not built: run python -m paper_2511_10508_amd.build")
    L = ctypes.CDLL(LIBPATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    rt = hip_runtimes_mapped()
    if len(rt) > 1:
        raise ImportError("more than one HIP runtime mapped: %s" % rt)
    _lib = L
    return L


def check(status):
    if status != PF_OK:
        raise PfError(status, lib().pf_last_error().decode())
    return status


def make_desc(kind, n, dx=1.0, dt=0.01, order=2, precision=PF_FP64, params=None, flags=0):
    """Fill a pf_desc.  n = (nx,), (nx, ny) or (nx, ny, nz); params default to the paper's unit constants."""
    n = list(n)
    ndim = len(n)
    while len(n) < 3:
        n.append(1)
    if params is None:
        params = {PF_GS: [0.2, 0.1, 0.04, 0.06], PF_MC: [1.0, 1.0, 0.5],
                  PF_MH: [1.0, 1.0, 0.5]}.get(kind, [1.0, 1.0])
    d = pf_desc()
    d.struct_size = ctypes.sizeof(pf_desc)
    d.kind = kind
    d.nfields = 1 + ndim if kind == PF_MH else 2 if kind in (PF_GS, PF_MC) else 1
    d.ndim = ndim
    for a in range(3):
        d.n[a] = int(n[a])
    d.dx, d.dt, d.order, d.precision = float(dx), float(dt), int(order), int(precision)
    d.nparams = len(params)
    for i, p in enumerate(params):
        d.params[i] = float(p)
    d.flags = int(flags)
    return d


def _dp(a):
    return a.ctypes.data_as(_pd)


class Model:
    """Owning handle of a pf_model (pf_create / pf_destroy)."""

    def __init__(self, desc, stream=None, bufs=None):
        self.desc = desc
        h = _vp()
        if bufs is None:
            check(lib().pf_create(ctypes.byref(desc), stream, ctypes.byref(h)))
        else:
            arr = (_vp * len(bufs))(*bufs)
            check(lib().pf_create_on(ctypes.byref(desc), stream, arr, len(bufs), ctypes.byref(h)))
        self.h = h
        self.nsites = desc.n[0] * desc.n[1] * desc.n[2]
        self.shape = (desc.n[2], desc.n[1], desc.n[0])

    def close(self):
        if self.h:
            lib().pf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, ic, seed, params):
        p = np.asarray(params, dtype=np.float64)
        check(lib().pf_init(self.h, ic, seed, _dp(p), p.size))

    def set_field(self, f, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        check(lib().pf_set_field(self.h, f, _dp(a), a.size))

    def get_field(self, f):
        out = np.empty(self.nsites, dtype=np.float64)
        check(lib().pf_get_field(self.h, f, _dp(out), out.size))
        return out.reshape(self.shape)

    def get_window(self, f, origin, wshape):
        """origin, wshape as (z, y, x); returns a (wz, wy, wx) array."""
        o = (_i64 * 3)(origin[2], origin[1], origin[0])
        w = (_i64 * 3)(wshape[2], wshape[1], wshape[0])
        out = np.empty(int(np.prod(wshape)), dtype=np.float64)
        check(lib().pf_get_window(self.h, f, o, w, _dp(out)))
        return out.reshape(wshape)

    def step(self, n):
        check(lib().pf_step(self.h, int(n)))

    def sync(self):
        check(lib().pf_sync(self.h))

    def reduce(self, which):
        hi, lo = _d(), _d()
        check(lib().pf_reduce(self.h, which, ctypes.byref(hi), ctypes.byref(lo)))
        return hi.value, lo.value

    def reduce_history(self, which, count):
        hi = np.empty(count)
        lo = np.empty(count)
        check(lib().pf_reduce_history(self.h, which, _dp(hi), _dp(lo), count))
        return hi, lo

    def steps_done(self):
        return lib().pf_steps_done(self.h)

    def set_steps_done(self, n):
        check(lib().pf_set_steps_done(self.h, int(n)))

    def field_device(self, f):
        """(device pointer, pitch in elements, bytes per element) of field f's current buffer."""
        p, pitch, eb = _vp(), _i64(), _i32()
        check(lib().pf_field_device(self.h, f, ctypes.byref(p), ctypes.byref(pitch), ctypes.byref(eb)))
        return p.value, pitch.value, eb.value

    def set_tile(self, chunk):
        check(lib().pf_set_tile(self.h, chunk))

    def tile(self):
        c, f = _i32(), _i32()
        check(lib().pf_get_tile(self.h, ctypes.byref(c), ctypes.byref(f)))
        return c.value, f.value

    def autotune(self, trials=3):
        check(lib().pf_autotune(self.h, trials))

    def timing(self, on):
        check(lib().pf_timing_enable(self.h, 1 if on else 0))

    def timing_read(self):
        """(kernel ms, launches, steps) since timing(True)."""
        ms, n, st = _d(), _i64(), _i64()
        check(lib().pf_timing_read(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(st)))
        return ms.value, n.value, st.value

    def set_time_block(self, tb):
        check(lib().pf_set_time_block(self.h, tb))

    def time_block(self):
        return lib().pf_get_time_block(self.h)

    def set_tile_rows(self, rows):
        check(lib().pf_set_tile_rows(self.h, rows))

    def tile_rows(self):
        return lib().pf_get_tile_rows(self.h)

    def set_passes(self, passes):
        check(lib().pf_set_passes(self.h, passes))

    def passes(self):
        return lib().pf_get_passes(self.h)

    def stream(self):
        s = _vp()
        check(lib().pf_stream(self.h, ctypes.byref(s)))
        return s.value


def step_noalloc(desc, stream, bufs, parity, nsteps, history=None):
    """pf_step_noalloc: nsteps steps on caller-owned device buffers (device
    pointers, pf_create_on layout) with no allocation; `history` is a device
    pointer of 6 * nsteps doubles or None."""
    arr = (_vp * len(bufs))(*bufs)
    check(lib().pf_step_noalloc(ctypes.byref(desc), stream, arr, len(bufs), int(parity), int(nsteps),
                                history))


def weights(order):
    w = np.empty(order // 2 + 1)
    check(lib().pf_weights(order, _dp(w)))
    return w


def weights1(order):
    w = np.empty(order // 2 + 1)
    check(lib().pf_weights1(order, _dp(w)))
    return w


def weights4(order):
    w = np.empty(order // 2 + 2)
    check(lib().pf_weights4(order, _dp(w)))
    return w


def stability(desc):
    v = _d()
    check(lib().pf_stability(ctypes.byref(desc), ctypes.byref(v)))
    return v.value


def footprint_bytes(desc):
    return lib().pf_footprint_bytes(ctypes.byref(desc))


def buffer_elems(desc):
    return lib().pf_buffer_elems(ctypes.byref(desc))
