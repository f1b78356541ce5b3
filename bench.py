"""Benchmark of the explicit FD phase-field step on one MI355X.

Workload (the headline one): 2D Cahn-Hilliard dc/dt = lap(c^3 - c - lap c) on
a 32768^2 periodic grid, dx = 1, dt = 0.01, 4th-order Laplacian applied
twice, c0 = U[-0.05, 0.05] (seed 202), synthetic data.  One step = one
forward-Euler update of every site with the mass / free-energy reductions of
the state fused into the same kernel (the whole hot path).  `value` is FP64
site-updates/s; the FP32-storage run is reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu] [--skip-fp32]
                    [--serving N]

Prints one JSON line.  The roofline object covers the dominant kernel (the
fused step): achieved = algorithmic bytes per launch (2 * fields * bytes per
value * sites: every field read once and written once) / mean kernel time,
timed with HIP events on the model's stream.
"""
import argparse
import ctypes
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print("[bench %.1fs] %s" % (time.perf_counter() - T0, msg), file=sys.stderr, flush=True)


T0 = time.perf_counter()


FAMILY_SOURCES = {"2d": ("pf_march2d.h", "pf_fused2d.h", "pf_fused2d_kind.h", "kernels_fused2d.hip"),
                  "3d": ("pf_march3d.h", "pf_fused3d.h", "pf_fused3d_kind.h", "kernels_fused3d.hip"),
                  "1d": ("kernels_fused1d.hip",),
                  "mh2d": ("kernels_mh2d.hip",),
                  "mh3d": ("pf_march3d.h", "kernels_mh3d.hip"),
                  "chd3d": ("pf_march3d.h", "kernels_chd3d.hip"),
                  "spectral": ("kernels_spectral.hip", "spectral.cpp")}


def source_hash(family="2d"):
    """Hash of the device code of one kernel family ("2d", "3d" or "mh3d"):
    its marching header and instantiation file plus the shared headers, with
    comments and whitespace removed (they do not change the kernels)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_10508_amd", "csrc")
    for f in ("pf_device.h", "pf_internal.h", "pf_dispatch.h") + FAMILY_SOURCES[family]:
        with open(os.path.join(csrc, f)) as fh:
            code = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(f.encode() + " ".join(code.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(tag, src_hash, layout=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and (given `layout`, a dict of
    time_block / tile_rows) on the same layout as the timed kernel (else
    None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % tag)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != src_hash:
        return None
    for key, field in (("time_block", "layout_tb"), ("tile_rows", "layout_rpw")):
        if layout and layout.get(key) is not None and field in vals and int(vals[field]) != int(layout[key]):
            return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def attach_traffic(r, tag, src_hash):
    """Add the HBM bytes per launch measured by the counters (committed
    summary profiles/traffic_<tag>.txt, taken on the current kernel sources)
    and the fraction of peak they make at the measured launch time."""
    t = measured_traffic(tag, src_hash, r)
    r["hbm_bytes_per_launch"] = t
    per = r.get("kernel_ms_per_launch")
    r["frac_hbm_measured"] = None if (t is None or not per) else round(t / (per * 1e-3) / 1e9 / PEAK_GBS, 4)
    return r


def copy_probe(P, torch, nbytes=2 ** 31, reps=10):
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    ms = ctypes.c_double()
    P.check(P.lib().pf_copy_probe(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                  nbytes, None, reps, ctypes.byref(ms)))
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms.value * 1e-3) / 1e9


def run_ch(P, n, prec, steps, warmup, seed=202, flags=0):
    d = P.make_desc(P.PF_CH, (n, n), dx=1.0, dt=0.01, order=4, precision=prec,
                    params=[1.0, 1.0], flags=P.PF_REDUCE_EACH_STEP | flags)
    m = P.Model(d)
    m.init(P.PF_IC_UNIFORM, seed, (-0.05, 0.05))
    m.autotune(2)
    m.step(warmup)
    m.sync()
    # per-launch events replace the graph, so a graph run is timed by wall only
    graph = (flags & P.PF_USE_GRAPH) != 0
    m.timing(not graph)
    t0 = time.perf_counter()
    m.step(steps)
    m.sync()
    t1 = time.perf_counter()
    kernel_ms, launches, ksteps = m.timing_read()
    hi, lo = m.reduce_history(P.PF_RED_MASS0, steps)
    mass = hi + lo
    drift = float(abs(mass - mass[0]).max())
    chunk, family = m.tile()
    tb = m.time_block()
    m.close()
    sites = float(n) * n
    wall = t1 - t0
    if graph:
        kernel_ms, launches, ksteps = wall * 1e3, 1, steps
    per_launch = kernel_ms / launches
    # algorithmic bytes of one launch: every field read and written once per
    # time step it advances (a two-step launch counts two steps)
    alg_bytes = 2 * 1 * (8 if prec == P.PF_FP64 else 4) * sites * (ksteps / launches)
    return dict(sites=sites, wall=wall, su_s=sites * steps / wall, ms_per_step=wall / steps * 1e3,
                kernel_ms=per_launch, alg_bytes=alg_bytes, steps_per_launch=ksteps / launches,
                achieved_gbs=alg_bytes / (per_launch * 1e-3) / 1e9, mass_drift=drift,
                chunk=chunk, family=family, time_block=tb)


def run_mc(P, n, prec, steps, warmup, seed=606):
    """Model C (Eq. model-c) 2D n^2, p = 4, dt = 0.01, c1 = c2 = 1, c3 = 0.5,
    phi0, rho0 = U[-0.1, 0.1], fused mass reductions of both fields every step."""
    d = P.make_desc(P.PF_MC, (n, n), dx=1.0, dt=0.01, order=4, precision=prec,
                    params=[1.0, 1.0, 0.5], flags=P.PF_REDUCE_EACH_STEP)
    m = P.Model(d)
    m.init(P.PF_IC_UNIFORM, seed, (-0.1, 0.1))
    m.autotune(2)
    m.step(warmup)
    m.sync()
    m.timing(True)
    t0 = time.perf_counter()
    m.step(steps)
    m.sync()
    wall = time.perf_counter() - t0
    kernel_ms, launches, ksteps = m.timing_read()
    hi, lo = m.reduce_history(P.PF_RED_MASS1, steps)
    drift = float(abs((hi + lo) - (hi[0] + lo[0])).max())
    chunk, tb = m.tile()[0], m.time_block()
    m.close()
    sites = float(n) * n
    per = kernel_ms / ksteps
    gbs = 2 * 2 * (8 if prec == P.PF_FP64 else 4) * sites / (per * 1e-3) / 1e9
    return {"value": sites * steps / wall, "ms_per_step": round(wall / steps * 1e3, 4),
            "kernel_ms": round(per, 4), "kernel_ms_per_launch": round(kernel_ms / launches, 4),
            "achieved_gbs": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4),
            "rho_mass_drift": drift, "chunk": chunk, "time_block": tb}


def run_ch_variant(P, n, prec, steps, warmup, direct, ndim, seed=202):
    """Cahn-Hilliard (Eq. model-b) p = 4, c1 = c2 = 1, c0 = U[-0.05, 0.05],
    fused mass / energy reductions every step: the 2D n^2 grid (dt = 0.01) or
    the 3D n^3 grid (dt = 0.005) with the direct biharmonic stencil
    (direct=True), or a 1D row of n sites with the composed operator."""
    flags = P.PF_REDUCE_EACH_STEP | (P.PF_BIHARMONIC_DIRECT if direct else 0)
    shape = {1: (n,), 2: (n, n), 3: (n, n, n)}[ndim]
    d = P.make_desc(P.PF_CH, shape, dx=1.0, dt=0.005 if ndim == 3 else 0.01, order=4, precision=prec,
                    params=[1.0, 1.0], flags=flags)
    m = P.Model(d)
    m.init(P.PF_IC_UNIFORM, seed, (-0.05, 0.05))
    m.autotune(2)
    m.step(warmup)
    m.sync()
    m.timing(True)
    t0 = time.perf_counter()
    m.step(steps)
    m.sync()
    wall = time.perf_counter() - t0
    kernel_ms, launches, ksteps = m.timing_read()
    hi, lo = m.reduce_history(P.PF_RED_MASS0, steps)
    drift = float(abs((hi + lo) - (hi[0] + lo[0])).max())
    chunk, tb = m.tile()[0], m.time_block()
    m.close()
    sites = float(n) ** ndim
    per = kernel_ms / ksteps
    gbs = 2 * (8 if prec == P.PF_FP64 else 4) * sites / (per * 1e-3) / 1e9
    return {"value": sites * steps / wall, "ms_per_step": round(wall / steps * 1e3, 4),
            "kernel_ms": round(per, 4), "kernel_ms_per_launch": round(kernel_ms / launches, 4),
            "achieved_gbs": round(gbs, 1),
            "frac_of_peak": round(gbs / PEAK_GBS, 4), "mass_drift": drift,
            "chunk": chunk, "time_block": tb}


def run_spectral(P, n, prec, steps, warmup, seed=202):
    """Semi-implicit Fourier spectral Cahn-Hilliard (Eq. model-b) on a 2D n^2
    grid, dx = 1, dt = 0.5 (far above the explicit limit), c1 = c2 = 1, c0 =
    U[-0.05, 0.05]: two hipFFT transforms (the updated spectrum is kept
    between steps) and two element-wise kernels per step.  `per_site_bytes`
    is the scheme's minimum HBM traffic per site and step with these
    transforms (each transform reads and writes its data once, the
    element-wise kernels likewise)."""
    d = P.make_desc(P.PF_CH, (n, n), dx=1.0, dt=0.5, order=2, precision=prec,
                    params=[1.0, 1.0], flags=P.PF_SPECTRAL)
    m = P.Model(d)
    m.init(P.PF_IC_UNIFORM, seed, (-0.05, 0.05))
    m.step(warmup)
    m.sync()
    m.timing(True)
    t0 = time.perf_counter()
    m.step(steps)
    m.sync()
    wall = time.perf_counter() - t0
    kernel_ms, launches, ksteps = m.timing_read()
    hi, lo = m.reduce(P.PF_RED_MASS0)
    m.close()
    Pb = 8 if prec == P.PF_FP64 else 4
    # nonlinear: read u, write g (2P); forward transform of g: read P, write
    # ~P (half spectrum of 2P-byte complex values); update: read 2 spectra,
    # write 2 (4P); inverse: read P, write P
    per_site = 2 * Pb + 2 * Pb + 4 * Pb + 2 * Pb
    sites = float(n) * n
    per = kernel_ms / ksteps
    gbs = per_site * sites / (per * 1e-3) / 1e9
    return {"value": sites * steps / wall, "ms_per_step": round(wall / steps * 1e3, 4),
            "kernel_ms": round(per, 4), "per_site_bytes": per_site,
            "achieved_gbs_of_min_traffic": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4),
            "mass": hi + lo}


def run_mh(P, n, prec, steps, warmup, seed=707, ndim=2):
    """Model H (Eq. model-h, transverse projector one) on a 2D n^2 grid (one
    y-marching pass over column strips), a 3D n^3 grid (one z-marching pass,
    the 3D march with four rows per wave at p = 4; mu in registers and LDS in
    both) or a 1D row of n
    sites (the fused strip kernel), autotuned, p = 4, dt = 0.005, c1 = c2 =
    1, c3 = 0.5, m and j = U[-0.1, 0.1]."""
    shape = {1: (n,), 2: (n, n), 3: (n, n, n)}[ndim]
    d = P.make_desc(P.PF_MH, shape, dx=1.0, dt=0.005, order=4, precision=prec,
                    params=[1.0, 1.0, 0.5])
    m = P.Model(d)
    m.init(P.PF_IC_UNIFORM, seed, (-0.1, 0.1))
    m.autotune(2)
    m.step(warmup)
    m.sync()
    m.timing(True)
    t0 = time.perf_counter()
    m.step(steps)
    m.sync()
    wall = time.perf_counter() - t0
    kernel_ms, launches, ksteps = m.timing_read()
    m.close()
    sites = float(n) ** ndim
    per = kernel_ms / ksteps
    gbs = 2 * (1 + ndim) * (8 if prec == P.PF_FP64 else 4) * sites / (per * 1e-3) / 1e9
    return {"value": sites * steps / wall, "ms_per_step": round(wall / steps * 1e3, 4),
            "kernel_ms": round(per, 4), "kernel_ms_per_launch": round(kernel_ms / launches, 4),
            "achieved_gbs": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4)}


def run_ch3d(P, n, order, prec, steps, warmup, seed=404):
    """Precision-study workload: 3D Cahn-Hilliard n^3, dt 0.005, c1 = c2 = 1,
    c0 = U[-0.05, 0.05] (seed 404), order 2 / 4 / 6, fused mass / energy
    reductions every step, autotuned."""
    d = P.make_desc(P.PF_CH, (n, n, n), dx=1.0, dt=0.005, order=order, precision=prec,
                    params=[1.0, 1.0], flags=P.PF_REDUCE_EACH_STEP)
    m = P.Model(d)
    m.init(P.PF_IC_UNIFORM, seed, (-0.05, 0.05))
    m.autotune(2)
    m.step(warmup)
    m.sync()
    m.timing(True)
    t0 = time.perf_counter()
    m.step(steps)
    m.sync()
    wall = time.perf_counter() - t0
    kernel_ms, launches, ksteps = m.timing_read()
    hi, lo = m.reduce_history(P.PF_RED_MASS0, steps)
    drift = float(abs((hi + lo) - (hi[0] + lo[0])).max())
    chunk, family = m.tile()
    tb, rows, passes = m.time_block(), m.tile_rows(), m.passes()
    m.close()
    sites = float(n) ** 3
    per = kernel_ms / ksteps
    gbs = 2 * (8 if prec == P.PF_FP64 else 4) * sites / (per * 1e-3) / 1e9
    return {"value": sites * steps / wall, "ms_per_step": round(wall / steps * 1e3, 4),
            "kernel_ms": round(per, 4), "kernel_ms_per_launch": round(kernel_ms / launches, 4),
            "achieved_gbs": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4),
            "mass_drift": drift, "chunk": chunk, "family": family, "time_block": tb,
            "tile_rows": rows, "passes": passes}


def run_ac128(P, steps=1000, seed=101):
    """The small workload: 2D Allen-Cahn 128^2, dx 1, dt 0.05, order 2, FP64,
    phi0 = U[-0.1, 0.1] (seed 101), 1000 steps: microseconds per step (wall)
    of the default path, which runs the 1000 steps of a call in one
    workgroup's LDS, eager and with PF_USE_GRAPH (the same launches), plus
    the kernel time of one launch per step with HIP events (timing mode takes
    that path)."""
    out = {}
    for name, flags in (("lds", 0), ("lds_graph_flag", P.PF_USE_GRAPH)):
        d = P.make_desc(P.PF_AC, (128, 128), dx=1.0, dt=0.05, order=2, precision=P.PF_FP64,
                        params=[1.0, 1.0], flags=flags)
        m = P.Model(d)
        m.init(P.PF_IC_UNIFORM, seed, (-0.1, 0.1))
        m.step(steps)  # warm-up (captures the graphs)
        m.sync()
        best = 1e30
        for _ in range(3):
            t0 = time.perf_counter()
            m.step(steps)
            m.sync()
            best = min(best, time.perf_counter() - t0)
        out[name + "_us_per_step"] = round(best / steps * 1e6, 3)
        if name == "lds":
            m.timing(True)
            m.step(steps)
            kms, _, ks = m.timing_read()
            out["per_launch_kernel_us_per_step"] = round(kms / ks * 1e3, 3)
        m.close()
    out["site_updates_per_s"] = 128 * 128 / (out["lds_us_per_step"] * 1e-6)
    return out


# ---------------------------------------------------------------------------
# Serving workload: the batched server against a one-at-a-time loop on the
# mixed request trace (synth.serving_trace: model uniform over AC / CH / GS,
# 2D sides 64..2048 or 3D sides 32..256 log-uniform, 100..10000 steps, orders
# 2 and 4, parameters jittered by +-20 %, FP32 storage, dt clamped to 0.9 of
# the stability limit).

def request_spec(req):
    """(desc, ic, icp, sites) of a trace request; dt is clamped to 0.9 of the limit."""
    import paper_2511_10508_amd as P
    kind = req["kind"]
    n = list(reversed(req["shape"]))[:req["ndim"]]
    prec = P.PF_FP32 if req["fp32"] else P.PF_FP64
    d = P.make_desc(kind, n, dx=1.0, dt=req["dt"], order=req["order"], precision=prec,
                    params=req["params"])
    lim = P.stability(d)
    if d.dt > 0.9 * lim:
        d.dt = 0.9 * lim
    if kind == P.PF_GS:
        ic, icp = P.PF_IC_GS_CUBES, (20, req["cube_side"], 0.01)
    elif kind == P.PF_AC:
        ic, icp = P.PF_IC_UNIFORM, (-0.1, 0.1)
    else:
        ic, icp = P.PF_IC_UNIFORM, (-0.05, 0.05)
    return d, ic, icp, int(np.prod(req["shape"]))


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else float("nan")


def _progress(every=30.0):
    """log(msg) at most every `every` seconds."""
    last = [time.perf_counter()]

    def tick(msg):
        now = time.perf_counter()
        if now - last[0] >= every:
            last[0] = now
            log(msg)
    return tick


def run_batched(trace, max_slots=256, steps_per_tick=64, budget=0):
    """The server: a submitter thread replays the arrivals, this thread polls
    and releases; latency = completion seen by the poller minus arrival."""
    import threading
    from paper_2511_10508_amd.serving import Server
    srv = Server(hbm_budget=budget, max_slots=max_slots, steps_per_tick=steps_per_tick)
    progress = _progress()
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


def run_serial(trace):
    """The one-at-a-time loop: for each request in arrival order, create,
    initialise, one launch per step, reduce, destroy.  Its capacity is the
    work over its busy time (the makespan less the time it waited for
    arrivals), so one run on the Poisson trace gives both."""
    import paper_2511_10508_amd as P
    specs = [request_spec(r) for r in trace]
    work = sum(s[3] * r["steps"] for s, r in zip(specs, trace))
    lat, svc = [], []
    idle = 0.0
    progress = _progress()
    start = time.perf_counter()
    for r, (d, ic, icp, _) in zip(trace, specs):
        progress("  serial: %d of %d requests done" % (len(lat), len(trace)))
        wait = r["arrival"] - (time.perf_counter() - start)
        if wait > 0:
            time.sleep(wait)
            idle += wait
        t_begin = time.perf_counter()
        m = P.Model(d)
        m.init(ic, r["seed"], icp)
        m.step(r["steps"])
        m.reduce(0)
        m.close()
        t_end = time.perf_counter()
        svc.append(t_end - t_begin)
        lat.append(t_end - (start + r["arrival"]))
    makespan = time.perf_counter() - start
    return dict(p50_s=_pct(lat, 50), p99_s=_pct(lat, 99), makespan_s=makespan, idle_s=idle,
                su_per_s=work / (makespan - idle), service_s=svc)


def fifo_replay(arrivals, service):
    """Latencies of a single FIFO server with the given per-request service
    times (the one-at-a-time loop, whose service time does not depend on the
    load) for other arrival times: completion_i = max(arrival_i,
    completion_{i-1}) + service_i."""
    done, lat = 0.0, []
    for a, s in zip(arrivals, service):
        done = max(a, done) + s
        lat.append(done - a)
    return lat


def serving_compare(nreq, seed=505, load=0.8, load2=0.5, steps_per_tick=64):
    """Throughput: the server's capacity with the whole trace submitted at
    t = 0 (work over makespan); the one-at-a-time loop's capacity is its work
    over busy time.  Latency: both on the same Poisson trace at `load` x the
    server's capacity (requests/s); p50 and p99 of completion minus arrival.
    A second load point (`load2`): the server measured again, the loop's
    latencies from a FIFO replay of its measured per-request service times.
    The traces hold the same requests at every rate."""
    import synth
    burst = synth.serving_trace(nreq, seed=seed, rate=None)
    cap_b = run_batched(burst, steps_per_tick=steps_per_tick)
    log("serving batched capacity: %.2f s" % cap_b["makespan_s"])
    rate = load * nreq / cap_b["makespan_s"]
    trace = synth.serving_trace(nreq, seed=seed, rate=rate)
    lat_b = run_batched(trace, steps_per_tick=steps_per_tick)
    log("serving batched at %.1f req/s: %.2f s" % (rate, lat_b["makespan_s"]))
    lat_s = run_serial(trace)
    log("serving serial at %.1f req/s: %.2f s (idle %.2f s)" % (rate, lat_s["makespan_s"],
                                                                lat_s["idle_s"]))
    rate2 = load2 * nreq / cap_b["makespan_s"]
    trace2 = synth.serving_trace(nreq, seed=seed, rate=rate2)
    lat_b2 = run_batched(trace2, steps_per_tick=steps_per_tick)
    log("serving batched at %.1f req/s: %.2f s" % (rate2, lat_b2["makespan_s"]))
    lat_s2 = fifo_replay([r["arrival"] for r in trace2], lat_s["service_s"])
    # the replay at the measured load, beside the measured loop: how well it models the loop
    lat_s1 = fifo_replay([r["arrival"] for r in trace], lat_s["service_s"])
    svc = lat_s.pop("service_s")
    return dict(requests=nreq, site_updates=sum(request_spec(r)[3] * r["steps"] for r in burst),
                batched_su_per_s=cap_b["su_per_s"], serial_su_per_s=lat_s["su_per_s"],
                throughput_speedup=cap_b["su_per_s"] / lat_s["su_per_s"],
                load=load, rate_req_per_s=rate,
                batched_p50_s=lat_b["p50_s"], batched_p99_s=lat_b["p99_s"],
                serial_p50_s=lat_s["p50_s"], serial_p99_s=lat_s["p99_s"],
                load2=load2, rate2_req_per_s=rate2,
                batched_p50_s_at_load2=lat_b2["p50_s"], batched_p99_s_at_load2=lat_b2["p99_s"],
                serial_p50_s_at_load2=_pct(lat_s2, 50), serial_p99_s_at_load2=_pct(lat_s2, 99),
                serial_p50_s_replayed=_pct(lat_s1, 50), serial_p99_s_replayed=_pct(lat_s1, 99),
                serial_service_total_s=sum(svc),
                batched_capacity=cap_b, batched_load=lat_b, batched_load2=lat_b2, serial_load=lat_s)


def cpu_baseline(n=4096, seconds=10.0, batch=10):
    """The oracle as it stands on the host cores: CH 2D p4 FP64 on an n^2
    sample of the workload, stepped in batches until `seconds` have passed."""
    import oracle
    import synth
    oracle.build()
    f = synth.initial_fields(2, (1, n, n), 202, synth.IC_UNIFORM, (-0.05, 0.05))
    f = oracle.run(2, f, 2, 1.0, 0.01, 4, [1.0, 1.0], 1)  # warm
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        f = oracle.run(2, f, 2, 1.0, 0.01, 4, [1.0, 1.0], batch)
        steps += batch
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", 0) or os.cpu_count() or 1)
    return dict(value=n * n * steps / dt, unit="site-updates/s", cores=cores, kind="oracle",
                sample="2D Cahn-Hilliard %d^2 p4 FP64, %d steps in %.1f s (OpenMP)" % (n, steps, dt))


def run_generic(P, kind, n, order, prec, dt, params, flags, ic, icp, steps=20, warmup=4, seed=808):
    """One autotuned model on synthetic input: kernel milliseconds per step
    (HIP events around every step launch) and the fraction of the 8 TB/s
    HBM peak that its algorithmic bytes (every field read and written once
    per step) make; the spectral step is priced at its 10 P per site."""
    d = P.make_desc(kind, n, dx=1.0, dt=dt, order=order, precision=prec, params=params, flags=flags)
    m = P.Model(d)
    m.init(ic, seed, icp)
    m.autotune(2)
    m.step(warmup)
    m.sync()
    m.timing(True)
    m.step(steps)
    kms, launches, ks = m.timing_read()
    chunk, family = m.tile()
    tb = m.time_block()
    m.close()
    per = kms / ks
    sites = 1.0
    for e in n:
        sites *= e
    Pb = 8 if prec == P.PF_FP64 else 4
    nf = {P.PF_GS: 2, P.PF_MC: 2, P.PF_MH: 1 + len(n)}.get(kind, 1)
    per_site = 10 * Pb if flags & P.PF_SPECTRAL else 2 * nf * Pb
    return {"kernel_ms": round(per, 4), "frac_of_peak": round(per_site * sites / (per * 1e-3) / 1e9 / PEAK_GBS, 4),
            "chunk": chunk, "family": family, "time_block": tb}


def run_extra(P):
    """Workloads beside the bench lines, for the kernel tables: 2D CH without
    per-step reductions, 2D AC and GS, 3D AC, Model C in 3D, the spectral
    step in 3D and 1D, Model H and the direct biharmonic at order 2."""
    R = P.PF_REDUCE_EACH_STEP
    U = P.PF_IC_UNIFORM
    cases = {
        "ch2d_32768_p4_noreduce": (P.PF_CH, (32768, 32768), 4, 0.01, [1.0, 1.0], 0, U, (-0.05, 0.05)),
        "ac2d_32768_p2": (P.PF_AC, (32768, 32768), 2, 0.05, [1.0, 1.0], R, U, (-0.1, 0.1)),
        "gs2d_16384_p2": (P.PF_GS, (16384, 16384), 2, 0.5, [0.2, 0.1, 0.04, 0.06], R, P.PF_IC_GS_CUBES, (20, 64, 0.01)),
        "ac3d_1024_p2": (P.PF_AC, (1024, 1024, 1024), 2, 0.05, [1.0, 1.0], 0, U, (-0.1, 0.1)),
        "mc3d_512_p2": (P.PF_MC, (512, 512, 512), 2, 0.01, [1.0, 1.0, 0.5], R, U, (-0.1, 0.1)),
        "spectral_ch3d_512": (P.PF_CH, (512, 512, 512), 2, 0.5, [1.0, 1.0], P.PF_SPECTRAL, U, (-0.05, 0.05)),
        "spectral_ch1d_67108864": (P.PF_CH, (1 << 26,), 2, 0.5, [1.0, 1.0], P.PF_SPECTRAL, U, (-0.05, 0.05)),
        "mh3d_512_p2": (P.PF_MH, (512, 512, 512), 2, 0.005, [1.0, 1.0, 0.5], 0, U, (-0.1, 0.1)),
        "mh2d_8192_p2": (P.PF_MH, (8192, 8192), 2, 0.005, [1.0, 1.0, 0.5], 0, U, (-0.1, 0.1)),
        "chd3d_512_p2": (P.PF_CH, (512, 512, 512), 2, 0.005, [1.0, 1.0], R | P.PF_BIHARMONIC_DIRECT, U,
                         (-0.05, 0.05)),
        "chd3d_512_p6": (P.PF_CH, (512, 512, 512), 6, 0.002, [1.0, 1.0], R | P.PF_BIHARMONIC_DIRECT, U,
                         (-0.05, 0.05)),
    }
    out = {}
    for key, (kind, n, order, dt, params, flags, ic, icp) in cases.items():
        for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
            out["%s_%s" % (key, tag)] = run_generic(P, kind, n, order, prec, dt, params, flags, ic, icp)
    return out


def run_gs3d(P, n, prec, steps, warmup, seed=303):
    """3D Gray-Scott n^3, p = 2, dt = 0.5, 20 cubes of side 16 plus 1 % noise."""
    d = P.make_desc(P.PF_GS, (n, n, n), dx=1.0, dt=0.5, order=2, precision=prec,
                    params=[0.2, 0.1, 0.04, 0.06])
    m = P.Model(d)
    m.init(P.PF_IC_GS_CUBES, seed, (20, 16, 0.01))
    m.autotune(2)
    m.step(warmup)
    m.sync()
    m.timing(True)
    t0 = time.perf_counter()
    m.step(steps)
    m.sync()
    wall = time.perf_counter() - t0
    kernel_ms, launches, ksteps = m.timing_read()
    chunk, tb, rows = m.tile()[0], m.time_block(), m.tile_rows()
    m.close()
    sites = float(n) ** 3
    per = kernel_ms / ksteps
    gbs = 2 * 2 * (8 if prec == P.PF_FP64 else 4) * sites / (per * 1e-3) / 1e9
    return {"value": sites * steps / wall, "ms_per_step": round(wall / steps * 1e3, 4),
            "kernel_ms": round(per, 4), "kernel_ms_per_launch": round(kernel_ms / launches, 4),
            "achieved_gbs": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_GBS, 4),
            "chunk": chunk, "time_block": tb, "tile_rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--serving", type=int, default=2000,
                    help="requests in the serving comparison (0 skips it)")
    ap.add_argument("--skip-3d", action="store_true")
    ap.add_argument("--skip-mc", action="store_true", help="skip the Model C lines")
    ap.add_argument("--skip-next", action="store_true",
                    help="skip the direct-biharmonic, 1D, spectral and Model H lines")
    ap.add_argument("--only", default="",
                    help="comma-separated sections to run besides the headline: gs3d, ch3d, "
                         "sizes, ac128, mc, next, serving, cpu (default: all), and the opt-in "
                         "extra (the kernel tables' other workloads)")
    args = ap.parse_args()
    only = set(x for x in args.only.split(",") if x)

    def want(section, skipped=False):
        return (section in only) if only else not skipped
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(requests would shard per GPU, a single model by slabs along its slowest "
              "axis). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_10508_amd as P
    P.lib()
    assert torch.cuda.is_available(), "no GPU visible"

    attain = copy_probe(P, torch)
    log("copy probe %.1f GB/s" % attain)
    src, src3 = source_hash("2d"), source_hash("3d")
    fp64 = run_ch(P, args.n, P.PF_FP64, args.steps, args.warmup)
    log("CH FP64: %.3f ms/step" % fp64["ms_per_step"])
    extra = {"copy_probe_gbs": round(attain, 1), "source_hash": src, "source_hash_3d": src3}
    if not args.skip_fp32:  # the headline's FP32 twin always runs unless skipped
        fp32 = run_ch(P, args.n, P.PF_FP32, args.steps, args.warmup)
        extra["fp32"] = {
            "value": fp32["su_s"], "ms_per_step": round(fp32["ms_per_step"], 4),
            "kernel_ms": round(fp32["kernel_ms"], 4), "achieved_gbs": round(fp32["achieved_gbs"], 1),
            "frac_of_peak": round(fp32["achieved_gbs"] / PEAK_GBS, 4),
            "mass_drift": fp32["mass_drift"], "chunk": fp32["chunk"],
            "time_block": fp32["time_block"], "kernel_ms_per_launch": round(fp32["kernel_ms"], 4)}
        attach_traffic(extra["fp32"], "ch2d_%d_fp32" % args.n, src)
        log("CH FP32: %.3f ms/step" % fp32["ms_per_step"])
    if want("gs3d", args.skip_3d):
        for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
            r = run_gs3d(P, 1024, prec, max(10, args.steps // 4), 5)
            extra["gs3d_1024_" + tag] = attach_traffic(r, "gs3d_1024_" + tag, src3)
            extra["gs3d_512_" + tag] = run_gs3d(P, 512, prec, max(20, args.steps // 2), 5)
        log("GS 3D done")
    if want("sizes"):
        # the 2D Cahn-Hilliard workload at its smaller sizes (4096^2 FP32 fits
        # the 256 MB last-level cache: not a roofline point)
        # (at 4096^2 the host's launch gaps show: the graph line replays the
        # step batch as one HIP graph)
        for n, gname, gflag in ((4096, "", 0), (4096, "_graph", P.PF_USE_GRAPH), (16384, "", 0)):
            for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
                r = run_ch(P, n, prec, max(20, args.steps), 10, flags=gflag)
                line = {"value": r["su_s"], "ms_per_step": round(r["ms_per_step"], 4),
                        "chunk": r["chunk"], "time_block": r["time_block"]}
                if not gflag:
                    line["kernel_ms_per_launch"] = round(r["kernel_ms"], 4)
                    line["frac_of_peak"] = round(r["achieved_gbs"] / PEAK_GBS, 4)
                extra["ch2d_%d_%s%s" % (n, tag, gname)] = line
        log("CH 2D sizes done")
    if want("ch3d", args.skip_3d):
        for order in (2, 4, 6):
            for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
                key = "ch3d_512_p%d_%s" % (order, tag)
                r = run_ch3d(P, 512, order, prec, max(20, args.steps // 2), 4)
                # a two-pass plan's traffic covers both of its kernels
                extra[key] = attach_traffic(r, key + ("_2pass" if r["passes"] == 2 else ""), src3)
        log("CH 3D 512^3 done")
    if "extra" in only:  # opt-in: the kernel tables' other workloads
        extra["extra"] = run_extra(P)
        log("extra workloads done")
    if want("ac128"):
        extra["ac2d_128_fp64_1000_steps"] = run_ac128(P)
        log("AC 128^2 done")
    if want("mc", args.skip_mc):
        for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
            key = "mc2d_%d_%s" % (args.n, tag)
            extra[key] = attach_traffic(run_mc(P, args.n, prec, max(10, args.steps // 4), 4), key, src)
        log("Model C done")
    if want("next", args.skip_next):
        for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
            key = "chd2d_%d_%s" % (args.n, tag)
            extra[key] = attach_traffic(run_ch_variant(
                P, args.n, prec, max(10, args.steps // 4), 4, direct=True, ndim=2), key, src)
            key = "ch1d_%d_%s" % (args.n * args.n // 4, tag)
            extra[key] = attach_traffic(run_ch_variant(
                P, args.n * args.n // 4, prec, max(10, args.steps // 4), 4, direct=False, ndim=1), key,
                source_hash("1d"))
            key = "chd3d_512_%s" % tag
            extra[key] = attach_traffic(run_ch_variant(P, 512, prec, max(10, args.steps // 4), 4,
                                                       direct=True, ndim=3), key, source_hash("chd3d"))
        log("direct biharmonic and 1D done")
        for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
            extra["spectral_ch2d_%d_%s" % (args.n // 2, tag)] = run_spectral(
                P, args.n // 2, prec, max(10, args.steps // 10), 3)
        log("spectral done")
        for prec, tag in ((P.PF_FP64, "fp64"), (P.PF_FP32, "fp32")):
            key = "mh2d_%d_%s" % (args.n // 4, tag)
            extra[key] = attach_traffic(run_mh(P, args.n // 4, prec, max(10, args.steps // 10), 2), key,
                                        source_hash("mh2d"))
            key = "mh1d_%d_%s" % (args.n * args.n // 16, tag)
            extra[key] = attach_traffic(run_mh(
                P, args.n * args.n // 16, prec, max(10, args.steps // 10), 2, ndim=1), key, source_hash("1d"))
            extra["mh3d_512_%s" % tag] = attach_traffic(
                run_mh(P, 512, prec, max(10, args.steps // 10), 2, ndim=3), "mh3d_512_" + tag,
                source_hash("mh3d"))
        log("Model H done")
    extra["fp64_mass_drift"] = fp64["mass_drift"]
    extra["fp64_chunk"] = fp64["chunk"]
    extra["fp64_time_block"] = fp64["time_block"]
    extra["fp64_kernel_ms_per_launch"] = round(fp64["kernel_ms"], 4)
    if args.serving and want("serving"):
        extra["serving"] = serving_compare(args.serving)
        log("serving done")

    traffic = measured_traffic("ch2d_%d_fp64" % args.n, src, {"time_block": fp64["time_block"]})
    out = {
        "metric": "site-updates/s & % HBM peak (FP64 vs FP32); serving p50/p99 vs serial",
        "value": fp64["su_s"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D Cahn-Hilliard %d^2 periodic, dx=1, dt=0.01, 4th-order "
                               "Laplacian applied twice, c0=U[-0.05,0.05] seed 202, fused "
                               "mass/energy reductions every step" % args.n,
                   "grid": [args.n, args.n], "order": 4, "fields": 1, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(fp64["achieved_gbs"], 1),
                     "peak": PEAK_GBS, "unit": "GB/s",
                     "frac": round(fp64["achieved_gbs"] / PEAK_GBS, 4),
                     "traffic": traffic,
                     # HBM bytes the counters measured per launch over the launch time
                     "traffic_frac": None if traffic is None else
                     round(traffic / (fp64["kernel_ms"] * 1e-3) / 1e9 / PEAK_GBS, 4)},
        "extra": extra,
    }
    if want("cpu", args.skip_cpu):
        out["cpu_baseline"] = cpu_baseline()
        log("cpu baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
