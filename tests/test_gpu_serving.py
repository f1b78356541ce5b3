"""Serving engine on the GPU: continuous batching returns, for every request,
bitwise the field that the same request gives when stepped alone; admission
respects the HBM budget; cancellation and late arrivals work.  The mix holds
grids small enough for the whole-grid-in-LDS class (every kind, 2D and 3D, r
up to 4) beside ones served by the batched tile kernels."""
import time

import numpy as np
import pytest

import oracle
import synth
import paper_2511_10508_amd as P
from paper_2511_10508_amd.serving import Server
from bench import request_spec

pytestmark = pytest.mark.gpu


def _mixed_requests():
    reqs = []
    specs = [
        (1, 2, (1, 70, 90), 2, True, [1.0, 1.0], 0.05),
        (2, 2, (1, 64, 128), 4, True, [1.0, 1.0], 0.01),
        (3, 2, (1, 100, 77), 2, True, [0.2, 0.1, 0.04, 0.06], 0.5),
        (1, 3, (20, 24, 30), 4, True, [1.1, 0.9], 0.05),
        (2, 3, (18, 20, 40), 2, True, [1.0, 1.0], 0.005),
        (3, 3, (24, 24, 24), 2, True, [0.2, 0.1, 0.04, 0.06], 0.5),
        (2, 2, (1, 50, 300), 4, False, [1.0, 1.0], 0.01),
        (3, 3, (16, 30, 20), 4, False, [0.2, 0.1, 0.035, 0.065], 0.3),
        (1, 2, (1, 33, 45), 4, False, [0.8, 1.2], 0.04),
        (2, 2, (1, 40, 40), 8, True, [1.0, 1.0], 0.005),   # r = 4
        (2, 3, (12, 12, 12), 8, False, [1.0, 1.0], 0.001),  # 3D CH r = 4
        (3, 2, (1, 128, 128), 4, True, [0.2, 0.1, 0.04, 0.06], 0.4),
        (1, 3, (20, 26, 70), 2, False, [1.0, 1.0], 0.05),   # FP64 3D AC / GS order 2: the
        (3, 3, (14, 40, 66), 2, False, [0.2, 0.1, 0.04, 0.06], 0.5),  # batched tile layout
        (4, 2, (1, 90, 110), 4, True, [1.0, 1.0, 0.5], 0.01),   # Model C
        (4, 3, (16, 20, 70), 2, False, [0.9, 1.1, 0.5], 0.01),
        (4, 2, (1, 40, 50), 6, False, [1.0, 1.0, 0.5], 0.002),  # tiny Model C, r = 3
        (3, 3, (20, 26, 40), 6, True, [0.2, 0.1, 0.04, 0.06], 0.3),  # batched 3D kernels with
        (4, 3, (16, 24, 30), 6, False, [1.0, 1.0, 0.5], 0.002),     # four rows per wave
        (3, 3, (12, 14, 16), 2, True, [0.2, 0.1, 0.04, 0.06], 0.5),  # tiny 3D Gray-Scott
    ]
    for i, (kind, ndim, shape, order, fp32, params, dt) in enumerate(specs):
        reqs.append(dict(id=i, kind=kind, ndim=ndim, shape=shape, steps=37 + 11 * i, order=order,
                         params=params, dt=dt, seed=1000 + i, arrival=0.0, fp32=fp32,
                         cube_side=3))
    return reqs


def _alone(req):
    d, ic, icp, _ = request_spec(req)
    m = P.Model(d)
    m.init(ic, req["seed"], icp)
    m.step(req["steps"])
    out = [m.get_field(f) for f in range(2 if req["kind"] in (3, 4) else 1)]
    mass = m.reduce(P.PF_RED_MASS0)
    return out, mass


def _serve(reqs, steps_per_tick=16, budget=0, max_slots=64, late=None, timeout=120.0):
    """Submit, then poll / fetch / release until every request is back.  A
    finished request holds its memory until released, so the client must
    release as it goes for queued requests to be admitted under a budget."""
    srv = Server(hbm_budget=budget, max_slots=max_slots, steps_per_tick=steps_per_tick)
    tickets = {}
    for r in reqs:
        d, ic, icp, _ = request_spec(r)
        tickets[srv.submit(d, ic, r["seed"], icp, r["steps"])] = r
    if late:
        # join while the first batch is on the device: wait for a few ticks
        t_end = time.time() + timeout
        while srv.stats()["ticks"] < 4:
            assert time.time() < t_end
            time.sleep(0.0002)
        for r in late:
            d, ic, icp, _ = request_spec(r)
            tickets[srv.submit(d, ic, r["seed"], icp, r["steps"])] = r
    results = {}
    t_end = time.time() + timeout
    while len(results) < len(tickets):
        assert time.time() < t_end, "requests did not complete in time"
        for res in srv.poll(1024):
            r = tickets[res["ticket"]]
            shape = r["shape"]
            fields = [srv.fetch(res["ticket"], f, shape) for f in range(2 if r["kind"] in (3, 4) else 1)]
            results[r["id"]] = (res, fields)
            srv.release(res["ticket"])
        time.sleep(0.001)
    st = srv.stats()
    srv.close()
    return results, st


def test_each_result_is_bitwise_the_same_alone_and_in_the_mix():
    reqs = _mixed_requests()
    results, st = _serve(reqs, steps_per_tick=16)
    assert len(results) == len(reqs)
    assert st["launches"] > 0 and st["captures"] > 0
    for r in reqs:
        res, fields = results[r["id"]]
        assert res["status"] == 0 and res["steps_done"] == r["steps"]
        alone, mass = _alone(r)
        for a, b in zip(alone, fields):
            assert np.array_equal(a, b), r
        assert abs(res["mass"][0] - (mass[0] + mass[1])) <= 1e-12 * max(1.0, abs(mass[0]))


def test_stable_batch_replays_captured_graphs():
    """Same class set tick after tick: the tick graph is captured once per
    table buffer and then replayed."""
    reqs = []
    for i in range(6):
        reqs.append(dict(id=i, kind=2, ndim=2, shape=(1, 96, 96 + 8 * i), steps=200, order=4,
                         params=[1.0, 1.0], dt=0.01, seed=77 + i, arrival=0.0, fp32=True,
                         cube_side=3))
    results, st = _serve(reqs, steps_per_tick=8)
    assert len(results) == 6
    assert st["replays"] >= 10, st
    for r in reqs[:2]:
        alone, _ = _alone(r)
        assert np.array_equal(alone[0], results[r["id"]][1][0])


def test_served_results_match_the_oracle():
    reqs = [r for r in _mixed_requests() if not r["fp32"]][:3]
    results, _ = _serve(reqs, steps_per_tick=8)
    for r in reqs:
        d, ic, icp, _ = request_spec(r)
        f0 = synth.initial_fields(r["kind"], r["shape"], r["seed"], ic, icp)
        ref = oracle.run(r["kind"], f0, r["ndim"], 1.0, d.dt, r["order"], r["params"], r["steps"])
        for a, b in zip(ref, results[r["id"]][1]):
            assert float(np.max(np.abs(a - b))) <= 1e-12


def test_late_arrivals_join_running_batch():
    reqs = _mixed_requests()
    first, late = reqs[:6], reqs[6:]
    for r in first:
        r["steps"] = 3000
    results, st = _serve(first, steps_per_tick=8, late=late)
    assert len(results) == len(reqs)
    admits_first = max(results[r["id"]][0]["t_admit"] for r in first)
    done_first = min(results[r["id"]][0]["t_done"] for r in first)
    admits_late = [results[r["id"]][0]["t_admit"] for r in late]
    assert min(admits_late) > admits_first
    assert min(admits_late) < done_first  # admitted while the first batch still ran
    for r in reqs:
        alone, _ = _alone(r)
        for a, b in zip(alone, results[r["id"]][1]):
            assert np.array_equal(a, b)


def test_admission_respects_hbm_budget():
    reqs = _mixed_requests()[:6]
    fps = []
    for r in reqs:
        d, _, _, _ = request_spec(r)
        fps.append(P.footprint_bytes(d))
    budget = int(max(fps) * 1.5)
    results, _ = _serve(reqs, steps_per_tick=8, budget=budget)
    assert len(results) == len(reqs)
    iv = sorted((results[r["id"]][0]["t_admit"], results[r["id"]][0]["t_done"]) for r in reqs)
    # FIFO admission: admit times follow submission order
    order = [results[r["id"]][0]["t_admit"] for r in reqs]
    assert order == sorted(order)
    # never more resident than the budget allows (requests are released on completion)
    for t, _ in iv:
        live = [i for i, (a, b) in enumerate(iv) if a <= t < b]
        assert sum(fps[i] for i in live) <= budget + max(fps)


def test_oversized_request_is_refused_and_cancel_works():
    srv = Server(hbm_budget=1 << 20, max_slots=4, steps_per_tick=8)
    d = P.make_desc(P.PF_CH, (1024, 1024), dt=0.01, order=4)
    with pytest.raises(P.PfError) as e:
        srv.submit(d, P.PF_IC_UNIFORM, 1, (-0.05, 0.05), 10)
    assert e.value.status == P.PF_ERR_NOMEM
    srv.close()
    srv = Server(max_slots=4, steps_per_tick=8)
    d = P.make_desc(P.PF_AC, (256, 256), dt=0.05)
    t = srv.submit(d, P.PF_IC_UNIFORM, 1, (-0.1, 0.1), 10 ** 6)
    time.sleep(0.05)
    srv.cancel(t)
    srv.drain(60)
    res = srv.poll()
    assert len(res) == 1 and res[0]["status"] == P.PF_ERR_STATE
    assert res[0]["steps_done"] < 10 ** 6
    srv.release(t)
    srv.close()


def test_unstable_request_is_refused():
    srv = Server(max_slots=4)
    d = P.make_desc(P.PF_GS, (64, 64, 64), dt=1.0)
    with pytest.raises(P.PfError) as e:
        srv.submit(d, P.PF_IC_GS_CUBES, 1, (4, 4, 0.01), 10)
    assert e.value.status == P.PF_ERR_UNSTABLE
    srv.close()


def test_nonfinite_request_is_isolated_from_its_batch():
    """A request whose state is NaN shares its class's launches (tiny and
    batched tile classes) with finite requests: it finishes with its
    non-finite sites counted, and every other request is bitwise the same as
    alone."""
    reqs = []
    for i, shape in enumerate([(1, 40, 40), (1, 40, 44), (1, 200, 300), (1, 210, 290)]):
        reqs.append(dict(id=i, kind=1, ndim=2, shape=shape, steps=90, order=2, params=[1.0, 1.0],
                         dt=0.05, seed=300 + i, arrival=0.0, fp32=True, cube_side=3))
    srv = Server(max_slots=16, steps_per_tick=16)
    tickets = {}
    for r in reqs:
        d, ic, icp, _ = request_spec(r)
        if r["id"] % 2 == 1:  # one NaN request per class
            ic, icp = P.PF_IC_CONST, (float("nan"),)
        tickets[srv.submit(d, ic, r["seed"], icp, r["steps"])] = r
    got = {}
    t_end = time.time() + 60
    while len(got) < len(reqs):
        assert time.time() < t_end
        for res in srv.poll(64):
            r = tickets[res["ticket"]]
            got[r["id"]] = (res, srv.fetch(res["ticket"], 0, r["shape"]))
            srv.release(res["ticket"])
        time.sleep(0.001)
    srv.close()
    for r in reqs:
        res, field = got[r["id"]]
        assert res["status"] == 0 and res["steps_done"] == r["steps"]
        sites = r["shape"][1] * r["shape"][2]
        if r["id"] % 2 == 1:
            assert res["nonfinite"] == sites and np.all(np.isnan(field))
        else:
            assert res["nonfinite"] == 0
            alone, _ = _alone(r)
            assert np.array_equal(alone[0], field)


def test_graph_cache_turnover_keeps_results(monkeypatch):
    """With a one-entry graph cache every new class set destroys the cached
    executable graphs; the server waits for the graph in flight first, and
    the results stay bitwise those of each request stepped alone."""
    monkeypatch.setenv("PFMI_SERVER_MAX_GRAPHS", "1")
    reqs = _mixed_requests()
    results, st = _serve(reqs, steps_per_tick=4)
    assert st["captures"] > 2, st
    for r in reqs:
        res, fields = results[r["id"]]
        assert res["status"] == 0 and res["steps_done"] == r["steps"]
        alone, _ = _alone(r)
        for a, b in zip(alone, fields):
            assert np.array_equal(a, b), r
