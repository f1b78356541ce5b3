"""Serving driver: the batched server against a one-at-a-time loop.

Server wraps pf_server_* (argument marshalling only).  compare() replays the
mixed request workload (synth.serving_trace: model uniform over AC / CH / GS,
2D sides 64..2048 or 3D sides 32..256 log-uniform, 100..10000 steps, orders 2
and 4, parameters jittered by +-20 %, FP32 storage) through

  * the server (continuous batching, graph-replayed persistent launches), and
  * a plain loop that, for each request in arrival order, creates a model,
    initialises it, runs its steps one launch per step, reduces and destroys
    it,

and reports p50 / p99 latency (completion minus arrival) and aggregate
site-updates/s (all requests' sites x steps over the makespan) for both.
"""
import ctypes
import threading
import time

import numpy as np

import synth
from . import (PF_AC, PF_CH, PF_FP32, PF_FP64, PF_GS, PF_IC_GS_CUBES, PF_IC_UNIFORM, Model,
               check, lib, make_desc, pf_result, stability)

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


def request_spec(req):
    """(desc, ic, icp, sites) of a trace request; dt is clamped to 0.9 of the limit."""
    kind = req["kind"]
    n = list(reversed(req["shape"]))[:req["ndim"]]
    prec = PF_FP32 if req["fp32"] else PF_FP64
    d = make_desc(kind, n, dx=1.0, dt=req["dt"], order=req["order"], precision=prec,
                  params=req["params"])
    lim = stability(d)
    if d.dt > 0.9 * lim:
        d.dt = 0.9 * lim
    if kind == PF_GS:
        ic, icp = PF_IC_GS_CUBES, (20, req["cube_side"], 0.01)
    elif kind == PF_AC:
        ic, icp = PF_IC_UNIFORM, (-0.1, 0.1)
    else:
        ic, icp = PF_IC_UNIFORM, (-0.05, 0.05)
    return d, ic, icp, int(np.prod(req["shape"]))


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def _progress(log, every=30.0):
    """Calls log(msg) at most every `every` seconds."""
    last = [time.perf_counter()]

    def tick(msg):
        now = time.perf_counter()
        if log and now - last[0] >= every:
            last[0] = now
            log(msg)
    return tick


def run_batched(trace, max_slots=256, steps_per_tick=64, budget=0, log=None):
    srv = Server(hbm_budget=budget, max_slots=max_slots, steps_per_tick=steps_per_tick)
    progress = _progress(log)
    specs = [request_spec(r) for r in trace]
    work = sum(s[3] * r["steps"] for s, r in zip(specs, trace))
    t_arr = {}
    done = {}
    start = time.perf_counter()

    def submitter():
        for r, (d, ic, icp, _) in zip(trace, specs):
            wait = r["arrival"] - (time.perf_counter() - start)
            if wait > 0:
                time.sleep(wait)
            tk = srv.submit(d, ic, r["seed"], icp, r["steps"])
            t_arr[tk] = start + r["arrival"]

    th = threading.Thread(target=submitter)
    th.start()
    lat = []
    while len(done) < len(trace):
        for res in srv.poll():
            now = time.perf_counter()
            done[res["ticket"]] = res
            srv.release(res["ticket"])
            while res["ticket"] not in t_arr:
                time.sleep(0.0005)
            lat.append(now - t_arr[res["ticket"]])
        progress("  batched: %d of %d requests done" % (len(done), len(trace)))
        time.sleep(0.0005)
    th.join()
    makespan = time.perf_counter() - start
    st = srv.stats()
    srv.close()
    bad = sum(1 for r in done.values() if r["status"] != 0)
    return dict(p50_s=_pct(lat, 50), p99_s=_pct(lat, 99), makespan_s=makespan,
                su_per_s=work / makespan, failed=bad, **st)


def run_serial(trace, log=None):
    specs = [request_spec(r) for r in trace]
    work = sum(s[3] * r["steps"] for s, r in zip(specs, trace))
    lat = []
    progress = _progress(log)
    start = time.perf_counter()
    for r, (d, ic, icp, _) in zip(trace, specs):
        progress("  serial: %d of %d requests done" % (len(lat), len(trace)))
        wait = r["arrival"] - (time.perf_counter() - start)
        if wait > 0:
            time.sleep(wait)
        m = Model(d)
        m.init(ic, r["seed"], icp)
        m.step(r["steps"])
        m.reduce(0)
        m.close()
        lat.append(time.perf_counter() - (start + r["arrival"]))
    makespan = time.perf_counter() - start
    return dict(p50_s=_pct(lat, 50), p99_s=_pct(lat, 99), makespan_s=makespan, su_per_s=work / makespan)


def compare(nreq, seed=505, load=0.8, steps_per_tick=64, log=None):
    """Throughput: both loops on the whole trace submitted at t = 0 (capacity,
    aggregate site-updates/s over the makespan).  Latency: both loops on the
    same Poisson trace at `load` x the batched capacity (requests/s); p50 and
    p99 of completion minus arrival."""
    log = log or (lambda m: None)
    burst = synth.serving_trace(nreq, seed=seed, rate=None)
    cap_b = run_batched(burst, steps_per_tick=steps_per_tick, log=log)
    log("serving batched capacity: %.2f s" % cap_b["makespan_s"])
    cap_s = run_serial(burst, log=log)
    log("serving serial capacity: %.2f s" % cap_s["makespan_s"])
    rate = load * nreq / cap_b["makespan_s"]
    trace = synth.serving_trace(nreq, seed=seed, rate=rate)
    lat_b = run_batched(trace, steps_per_tick=steps_per_tick, log=log)
    log("serving batched at %.1f req/s: %.2f s" % (rate, lat_b["makespan_s"]))
    lat_s = run_serial(trace, log=log)
    log("serving serial at %.1f req/s: %.2f s" % (rate, lat_s["makespan_s"]))
    return dict(requests=nreq, site_updates=sum(request_spec(r)[3] * r["steps"] for r in burst),
                batched_su_per_s=cap_b["su_per_s"], serial_su_per_s=cap_s["su_per_s"],
                throughput_speedup=cap_b["su_per_s"] / cap_s["su_per_s"],
                load=load, rate_req_per_s=rate,
                batched_p50_s=lat_b["p50_s"], batched_p99_s=lat_b["p99_s"],
                serial_p50_s=lat_s["p50_s"], serial_p99_s=lat_s["p99_s"],
                batched_capacity=cap_b, serial_capacity=cap_s, batched_load=lat_b, serial_load=lat_s)
