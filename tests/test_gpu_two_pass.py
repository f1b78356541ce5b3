"""Two-pass 3D Cahn-Hilliard (mu through a field-sized buffer): bitwise the
fields of the fused single pass, reductions equal to their compensated
accuracy, parity with the FP64 oracle, graph replay, the autotuner's choice
and the refusals of pf_set_passes."""
import numpy as np
import pytest

import oracle
import paper_2511_10508_amd as P
from test_gpu_parity import BASE, TOL, dt_for, fields_for, oracle_run

pytestmark = pytest.mark.gpu


def _run(f0, n, order, prec, dt, steps, passes, flags=P.PF_REDUCE_EACH_STEP, chunk=8):
    d = P.make_desc(P.PF_CH, n, dt=dt, order=order, precision=prec, params=BASE[P.PF_CH][0],
                    flags=flags)
    m = P.Model(d)
    m.set_tile(chunk)
    m.set_passes(passes)
    assert m.passes() == passes
    m.set_field(0, f0[0])
    m.step(steps)
    return m


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_two_passes_equal_one_pass_and_the_oracle(order, prec):
    """Ragged strips, y tiles and z chunks, 101 steps with per-step reductions."""
    shape, ndim, steps = (29, 45, 150), 3, 101
    params = BASE[P.PF_CH][0]
    dt = dt_for(P.PF_CH, ndim, order, params)
    f0 = fields_for(P.PF_CH, shape, 71)
    n = (shape[2], shape[1], shape[0])
    outs, hist = [], []
    for passes in (1, 2):
        m = _run(f0, n, order, prec, dt, steps, passes)
        outs.append(m.get_field(0))
        hist.append([sum(m.reduce_history(q, steps)) for q in (P.PF_RED_MASS0, P.PF_RED_ENERGY)])
    assert np.array_equal(outs[0], outs[1])
    for a, b in zip(hist[0], hist[1]):
        assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, float(np.max(np.abs(a))))
    ref = oracle_run(P.PF_CH, shape, ndim, order, params, dt, steps, 71)[1]
    assert float(np.max(np.abs(outs[1] - ref[0]))) <= TOL[prec]


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
def test_two_pass_history_matches_oracle_reductions(prec):
    """Entry k of the history reduces the state at the start of step k (mass and
    free energy, FP64 sums of the stored values)."""
    shape, ndim, order, steps = (12, 30, 40), 3, 4, 5
    params = BASE[P.PF_CH][0]
    dt = dt_for(P.PF_CH, ndim, order, params)
    f0 = fields_for(P.PF_CH, shape, 17)
    n = (shape[2], shape[1], shape[0])
    m = _run(f0, n, order, prec, dt, steps, 2, chunk=16)
    h0, l0 = m.reduce_history(P.PF_RED_MASS0, steps)
    h1, l1 = m.reduce_history(P.PF_RED_ENERGY, steps)
    state = f0[0].copy()
    if prec == P.PF_FP32:
        state = state.astype(np.float32).astype(np.float64)
    tol = 2e-12 if prec == P.PF_FP64 else 1e-4
    N = state.size
    for k in range(steps):
        mass, energy, _ = oracle.reduce(P.PF_CH, [state], ndim, 1.0, order, params)
        assert abs(h0[k] + l0[k] - mass[0]) <= tol * N * 1e-2 + 1e-13
        assert abs(h1[k] + l1[k] - energy) <= tol * N * 1e-1 + 1e-12
        state = oracle.run(P.PF_CH, [state], ndim, 1.0, dt, order, params, 1)[0]


def test_two_pass_graph_replay_equals_eager():
    shape, order = (20, 37, 70), 4
    params = BASE[P.PF_CH][0]
    dt = dt_for(P.PF_CH, 3, order, params)
    f0 = fields_for(P.PF_CH, shape, 5)
    n = (shape[2], shape[1], shape[0])
    a = _run(f0, n, order, P.PF_FP64, dt, 70, 2, flags=P.PF_REDUCE_EACH_STEP)
    b = _run(f0, n, order, P.PF_FP64, dt, 70, 2, flags=P.PF_REDUCE_EACH_STEP | P.PF_USE_GRAPH)
    assert np.array_equal(a.get_field(0), b.get_field(0))
    for q in (P.PF_RED_MASS0, P.PF_RED_ENERGY):
        assert np.array_equal(sum(a.reduce_history(q, 70)), sum(b.reduce_history(q, 70)))


def test_autotuner_considers_two_passes_and_keeps_the_fields():
    shape, order = (24, 40, 64), 6
    params = BASE[P.PF_CH][0]
    dt = dt_for(P.PF_CH, 3, order, params)
    f0 = fields_for(P.PF_CH, shape, 9)
    n = (shape[2], shape[1], shape[0])
    ref = _run(f0, n, order, P.PF_FP32, dt, 12, 1).get_field(0)
    d = P.make_desc(P.PF_CH, n, dt=dt, order=order, precision=P.PF_FP32, params=params,
                    flags=P.PF_REDUCE_EACH_STEP)
    m = P.Model(d)
    m.set_field(0, f0[0])
    m.autotune(2)
    assert m.passes() in (1, 2)
    m.step(12)
    assert np.array_equal(m.get_field(0), ref)


def test_set_passes_refusals():
    ch3 = P.Model(P.make_desc(P.PF_CH, (40, 30, 20), dt=0.001, order=2))
    assert ch3.passes() == 1
    ch3.set_passes(2)
    with pytest.raises(P.PfError) as e:
        ch3.set_time_block(2)
    assert e.value.status == P.PF_ERR_UNSUPPORTED
    ch3.set_passes(1)
    assert ch3.passes() == 1
    with pytest.raises(P.PfError) as e:
        ch3.set_passes(3)
    assert e.value.status == P.PF_ERR_ARG
    ch6 = P.Model(P.make_desc(P.PF_CH, (40, 30, 20), dt=1e-4, order=6, precision=P.PF_FP32,
                              flags=P.PF_REDUCE_EACH_STEP))
    assert ch6.passes() == 1 and ch6.tile_rows() == 4  # the 48-row tiles of 12 waves
    ch6.set_passes(2)
    assert ch6.passes() == 2 and ch6.tile_rows() == 2
    ch6.set_passes(1)
    assert ch6.passes() == 1 and ch6.tile_rows() == 4
    assert P.Model(P.make_desc(P.PF_CH, (40, 30, 20), dt=1e-4, order=6, precision=P.PF_FP32)).passes() == 1
    for d in (P.make_desc(P.PF_CH, (40, 30), dt=0.001, order=4),
              P.make_desc(P.PF_AC, (40, 30, 20), dt=0.01, order=2),
              P.make_desc(P.PF_CH, (40, 30, 20), dt=1e-5, order=8),
              P.make_desc(P.PF_CH, (40, 30, 20), dt=1e-4, order=4, flags=P.PF_BIHARMONIC_DIRECT)):
        m = P.Model(d)
        with pytest.raises(P.PfError) as e:
            m.set_passes(2)
        assert e.value.status == P.PF_ERR_UNSUPPORTED
