"""Python handle of the serving engine (pf_server_*), argument marshalling
only: continuous batching of independent simulation requests runs in the
library's scheduler thread and HIP kernels."""
import ctypes

import numpy as np

from . import check, lib, pf_result

_vp, _u64, _i32, _i64, _d = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class Server:
    def __init__(self, hbm_budget=0, max_slots=256, steps_per_tick=64, device=0):
        h = _vp()
        check(lib().pf_server_create(device, hbm_budget, max_slots, steps_per_tick, ctypes.byref(h)))
        self.h = h

    def submit(self, desc, ic, seed, icp, nsteps):
        p = np.asarray(icp, dtype=np.float64)
        t = _u64()
        check(lib().pf_server_submit(self.h, ctypes.byref(desc), ic, seed,
                                     p.ctypes.data_as(ctypes.POINTER(_d)), p.size, int(nsteps),
                                     ctypes.byref(t)))
        return t.value

    def poll(self, maxn=512):
        arr = (pf_result * maxn)()
        n = _i32()
        check(lib().pf_server_poll(self.h, arr, maxn, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            r = arr[i]
            out.append(dict(ticket=r.ticket, status=r.status, t_submit=r.t_submit, t_admit=r.t_admit,
                            t_done=r.t_done, mass=(r.mass[0], r.mass[1]), energy=r.energy,
                            nonfinite=r.nonfinite, steps_done=r.steps_done))
        return out

    def fetch(self, ticket, field, shape):
        out = np.empty(int(np.prod(shape)), dtype=np.float64)
        check(lib().pf_server_fetch(self.h, ticket, field, out.ctypes.data_as(ctypes.POINTER(_d)), out.size))
        return out.reshape(shape)

    def release(self, ticket):
        check(lib().pf_server_release(self.h, ticket))

    def cancel(self, ticket):
        check(lib().pf_server_cancel(self.h, ticket))

    def drain(self, timeout=600.0):
        check(lib().pf_server_drain(self.h, timeout))

    def stats(self):
        v = [_i64() for _ in range(4)]
        check(lib().pf_server_stats(self.h, *[ctypes.byref(x) for x in v]))
        return dict(ticks=v[0].value, launches=v[1].value, captures=v[2].value, replays=v[3].value)

    def close(self):
        if self.h:
            lib().pf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
