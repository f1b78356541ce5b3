"""GPU parity: libpfmi's HIP kernels against the CPU FP64 oracle.

Every case starts both sides from the same seeded synthetic fields (synth),
runs the GPU through the C ABI and compares element by element:
max |GPU - oracle| <= 1e-12 for FP64 storage and <= 1e-4 for FP32 storage
after 100 steps.  Grids span several strips, tiles and chunks with ragged
tails; bitwise checks cover the per-site invariances (kernel family, tile
shape, graph replay).
"""
import math

import numpy as np
import pytest

import oracle
import synth
import paper_2511_10508_amd as P

pytestmark = pytest.mark.gpu

TOL = {P.PF_FP64: 1e-12, P.PF_FP32: 1e-4}
BASE = {P.PF_AC: ([1.0, 1.0], 0.05), P.PF_CH: ([1.0, 1.0], 0.01),
        P.PF_GS: ([0.2, 0.1, 0.04, 0.06], 0.5), P.PF_MC: ([1.0, 1.0, 0.5], 0.01)}


def dt_for(kind, ndim, order, params, dx=1.0):
    return min(BASE[kind][1], 0.8 * oracle.dt_max(kind, ndim, dx, order, params))


def fields_for(kind, shape, seed):
    if kind == P.PF_AC:
        return synth.initial_fields(1, shape, seed, synth.IC_UNIFORM, (-0.1, 0.1))
    if kind == P.PF_CH:
        return synth.initial_fields(2, shape, seed, synth.IC_UNIFORM, (-0.05, 0.05))
    if kind == P.PF_MC:
        return synth.initial_fields(4, shape, seed, synth.IC_UNIFORM, (-0.1, 0.1))
    return synth.initial_fields(3, shape, seed, synth.IC_GS_CUBES, (6, 4, 0.01))


def gpu_run(kind, fields, ndim, order, prec, params, dt, nsteps, flags=0, chunk=None):
    shape = fields[0].shape
    n = (shape[2], shape[1]) if ndim == 2 else (shape[2], shape[1], shape[0])
    d = P.make_desc(kind, n, dt=dt, order=order, precision=prec, params=params, flags=flags)
    m = P.Model(d)
    if chunk:
        m.set_tile(chunk)
    for f, a in enumerate(fields):
        m.set_field(f, a)
    m.step(nsteps)
    out = [m.get_field(f) for f in range(len(fields))]
    return out, m


_oracle_cache = {}


def oracle_run(kind, shape, ndim, order, params, dt, nsteps, seed):
    key = (kind, shape, ndim, order, tuple(params), dt, nsteps, seed)
    if key not in _oracle_cache:
        f0 = fields_for(kind, shape, seed)
        _oracle_cache[key] = (f0, oracle.run(kind, f0, ndim, 1.0, dt, order, params, nsteps))
    return _oracle_cache[key]


CASES = []
for kind in (P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC):
    for ndim, shape, chunk in ((2, (1, 75, 301), 32), (3, (21, 37, 150), 8)):
        for order in (2, 4, 6):
            CASES.append((kind, ndim, shape, chunk, order))
CASES.append((P.PF_CH, 2, (1, 70, 260), 24, 8))
CASES.append((P.PF_AC, 2, (1, 40, 90), 16, 12))
CASES.append((P.PF_GS, 3, (12, 13, 40), 5, 8))


def _id(c):
    return "k%d-%dd-%s-p%d" % (c[0], c[1], "x".join(map(str, c[2])), c[4])


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
def test_parity_100_steps(case, prec):
    kind, ndim, shape, chunk, order = case
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0, ref = oracle_run(kind, shape, ndim, order, params, dt, 100, 17)
    got, m = gpu_run(kind, f0, ndim, order, prec, params, dt, 100, chunk=chunk)
    for g, r in zip(got, ref):
        err = float(np.max(np.abs(g - r)))
        assert err <= TOL[prec], (err, m.tile())
    assert m.steps_done() == 100


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", [P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC])
@pytest.mark.parametrize("ndim,shape", [(2, (1, 67, 277)), (3, (19, 35, 140))])
def test_fused_equals_generic_bitwise(kind, ndim, shape, prec):
    order = 4
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 5)
    a, ma = gpu_run(kind, f0, ndim, order, prec, params, dt, 30, chunk=16)
    b, mb = gpu_run(kind, f0, ndim, order, prec, params, dt, 30, flags=P.PF_FORCE_GENERIC)
    assert ma.tile()[1] == 0 and mb.tile()[1] == 1
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("kind", [P.PF_CH, P.PF_GS])
@pytest.mark.parametrize("ndim,shape,chunks", [(2, (1, 90, 300), (7, 32, 512)), (3, (30, 33, 130), (3, 11, 64))])
def test_tile_shape_invariance_bitwise(kind, ndim, shape, chunks):
    order = 4
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 8)
    outs = [gpu_run(kind, f0, ndim, order, P.PF_FP64, params, dt, 20, chunk=c)[0] for c in chunks]
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("kind", [P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC])
def test_graph_replay_equals_eager_bitwise(kind):
    shape, ndim, order = (1, 64, 96), 2, 4
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 9)
    a, _ = gpu_run(kind, f0, ndim, order, P.PF_FP64, params, dt, 70)
    b, _ = gpu_run(kind, f0, ndim, order, P.PF_FP64, params, dt, 70, flags=P.PF_USE_GRAPH)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_config_allen_cahn_128_1000_steps():
    """2D Allen-Cahn 128^2, dx 1, dt 0.05, p = 2, phi0 ~ U[-0.1, 0.1], 1000 steps, FP64."""
    shape = (1, 128, 128)
    f0 = synth.initial_fields(1, shape, 101, synth.IC_UNIFORM, (-0.1, 0.1))
    ref = oracle.run(1, f0, 2, 1.0, 0.05, 2, [1.0, 1.0], 1000)
    for flags in (0, P.PF_USE_GRAPH):
        got, _ = gpu_run(P.PF_AC, f0, 2, 2, P.PF_FP64, [1.0, 1.0], 0.05, 1000, flags=flags)
        assert float(np.max(np.abs(got[0] - ref[0]))) <= 1e-12


# the first six fit the whole-grid kernel (2D, ny a multiple of 16, every
# 16-row segment of every column a thread of one 1024-thread workgroup), the
# last two take the per-launch path
LDS_CASES = [((1, 128, 128), 2, P.PF_FP64, 37), ((1, 128, 128), 2, P.PF_FP32, 4100),
             ((1, 32, 70), 4, P.PF_FP32, 64), ((1, 16, 1000), 2, P.PF_FP64, 21),
             ((1, 64, 64), 4, P.PF_FP64, 13), ((1, 48, 20), 2, P.PF_FP32, 31),
             ((1, 5, 7), 4, P.PF_FP64, 13), ((9, 10, 11), 2, P.PF_FP64, 30),
             # p = 2 on 64 or 128 columns and p = 4 on 128 columns, of 64 or
             # 128 rows: the row kernel (one wave per band of rows,
             # x-neighbours by lane rotation)
             ((1, 64, 128), 2, P.PF_FP64, 29), ((1, 128, 64), 2, P.PF_FP32, 33),
             ((1, 64, 64), 2, P.PF_FP32, 8), ((1, 128, 64), 2, P.PF_FP64, 1),
             ((1, 64, 128), 4, P.PF_FP64, 17), ((1, 128, 128), 4, P.PF_FP32, 9)]


@pytest.mark.parametrize("shape,order,prec,steps", LDS_CASES,
                         ids=["%s-p%d-%s-%d" % ("x".join(map(str, c[0])), c[1], "fp64" if c[2] == P.PF_FP64
                                                else "fp32", c[3]) for c in LDS_CASES])
def test_allen_cahn_whole_grid_in_lds_bitwise(shape, order, prec, steps):
    """Small 2D Allen-Cahn grids run all the steps of a call in one
    workgroup's LDS (up to 4096 per launch): fields bitwise those of the per-site
    kernels, for odd and even step counts, calls split in two, graphs, and
    per-step reductions (which take the one-launch-per-step path)."""
    ndim = 3 if shape[0] > 1 else 2
    params = BASE[P.PF_AC][0]
    dt = dt_for(P.PF_AC, ndim, order, params)
    f0 = fields_for(P.PF_AC, shape, 44)
    ref, _ = gpu_run(P.PF_AC, f0, ndim, order, prec, params, dt, steps, flags=P.PF_FORCE_GENERIC)
    for flags in (0, P.PF_USE_GRAPH, P.PF_REDUCE_EACH_STEP):
        got, m = gpu_run(P.PF_AC, f0, ndim, order, prec, params, dt, steps, flags=flags)
        assert m.tile()[1] == 0 and m.steps_done() == steps
        assert np.array_equal(got[0], ref[0]), flags
    n = {2: (shape[2], shape[1]), 3: (shape[2], shape[1], shape[0])}[ndim]
    m = P.Model(P.make_desc(P.PF_AC, n, dt=dt, order=order, precision=prec, params=params))
    m.set_field(0, f0[0])
    m.step(steps // 3)
    m.step(steps - steps // 3)
    assert np.array_equal(m.get_field(0), ref[0])


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind,ndim,shape,ic,icp", [
    (P.PF_AC, 2, (1, 33, 70), P.PF_IC_UNIFORM, (-0.1, 0.1)),
    (P.PF_CH, 3, (9, 10, 11), P.PF_IC_UNIFORM, (-0.05, 0.05)),
    (P.PF_GS, 3, (20, 18, 17), P.PF_IC_GS_CUBES, (5, 4, 0.01)),
    (P.PF_GS, 2, (1, 40, 50), P.PF_IC_CONST, (1.0, 0.0)),
    (P.PF_MC, 2, (1, 40, 50), P.PF_IC_UNIFORM, (-0.1, 0.1)),
])
def test_device_init_matches_generator(kind, ndim, shape, ic, icp, prec):
    n = (shape[2], shape[1]) if ndim == 2 else (shape[2], shape[1], shape[0])
    d = P.make_desc(kind, n, dt=0.001, precision=prec)
    m = P.Model(d)
    m.init(ic, 4242, icp)
    ref = synth.initial_fields(kind, shape, 4242, ic, icp)
    for f, r in enumerate(ref):
        g = m.get_field(f)
        if prec == P.PF_FP32:
            r = r.astype(np.float32).astype(np.float64)
        assert np.array_equal(g, r)


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("ndim,shape", [(2, (1, 50, 60)), (3, (10, 12, 14))])
@pytest.mark.parametrize("order", [2, 6])
def test_gray_scott_fixed_point_bitwise(ndim, shape, order, prec):
    n = (shape[2], shape[1]) if ndim == 2 else (shape[2], shape[1], shape[0])
    d = P.make_desc(P.PF_GS, n, dt=0.3, order=order, precision=prec)
    m = P.Model(d)
    m.init(P.PF_IC_CONST, 0, (1.0, 0.0))
    m.step(50)
    assert np.all(m.get_field(0) == 1.0) and np.all(m.get_field(1) == 0.0)


def _oracle_reductions(kind, fields, ndim, order, params):
    mass, energy, bad = oracle.reduce(kind, fields, ndim, 1.0, order, params)
    return mass, energy


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind,ndim,shape", [
    (P.PF_AC, 2, (1, 70, 200)), (P.PF_CH, 2, (1, 64, 250)), (P.PF_CH, 3, (16, 20, 70)),
    (P.PF_GS, 3, (16, 20, 70)), (P.PF_AC, 3, (12, 30, 40)), (P.PF_MC, 2, (1, 66, 210)),
    (P.PF_MC, 3, (14, 22, 70)),
])
def test_reductions_match_exact_sums_of_the_state(kind, ndim, shape, prec):
    """pf_reduce of the GPU state vs the oracle's exact sums of the same downloaded state."""
    order = 4
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 12)
    got, m = gpu_run(kind, f0, ndim, order, prec, params, dt, 10)
    mass, energy = _oracle_reductions(kind, got, ndim, order, params)
    N = got[0].size
    hi, lo = m.reduce(P.PF_RED_MASS0)
    scale = float(np.sum(np.abs(got[0])))
    assert abs((hi + lo) - mass[0]) <= 1e-15 * scale + 1e-300
    if kind in (P.PF_GS, P.PF_MC):
        hi, lo = m.reduce(P.PF_RED_MASS1)
        assert abs((hi + lo) - mass[1]) <= 1e-15 * float(np.sum(np.abs(got[1])))
        with pytest.raises(P.PfError):
            m.reduce(P.PF_RED_ENERGY)
    else:
        hi, lo = m.reduce(P.PF_RED_ENERGY)
        e = oracle.energy_density(got[0], ndim, 1.0, order, params)
        assert abs((hi + lo) - energy) <= 1e-13 * float(np.sum(np.abs(e)))
    assert m.reduce(P.PF_RED_NONFINITE)[0] == 0.0
    assert N == got[0].size


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind,ndim,shape,generic", [
    (P.PF_CH, 2, (1, 64, 250), False), (P.PF_AC, 3, (12, 30, 40), False),
    (P.PF_GS, 3, (12, 30, 40), False), (P.PF_CH, 3, (12, 30, 40), False),
    (P.PF_CH, 2, (1, 30, 40), True), (P.PF_MC, 2, (1, 64, 250), False),
    (P.PF_MC, 3, (12, 30, 40), False), (P.PF_MC, 2, (1, 30, 40), True),
])
def test_fused_history_matches_oracle(kind, ndim, shape, generic, prec):
    """PF_REDUCE_EACH_STEP: entry k reduces the state at the start of step k."""
    order = 4
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 13)
    flags = P.PF_REDUCE_EACH_STEP | (P.PF_FORCE_GENERIC if generic else 0)
    nsteps = 6
    got, m = gpu_run(kind, f0, ndim, order, prec, params, dt, nsteps, flags=flags, chunk=16)
    h0, l0 = m.reduce_history(P.PF_RED_MASS0, nsteps)
    which1 = P.PF_RED_MASS1 if kind in (P.PF_GS, P.PF_MC) else P.PF_RED_ENERGY
    h1, l1 = m.reduce_history(which1, nsteps)
    state = [a.copy() for a in f0]
    if prec == P.PF_FP32:
        state = [a.astype(np.float32).astype(np.float64) for a in state]
    tol = 2e-12 if prec == P.PF_FP64 else 1e-4
    for k in range(nsteps):
        mass, energy = _oracle_reductions(kind, state, ndim, order, params)
        N = state[0].size
        assert abs(h0[k] + l0[k] - mass[0]) <= tol * N * 1e-2 + 1e-13
        ref1 = mass[1] if kind in (P.PF_GS, P.PF_MC) else energy
        assert abs(h1[k] + l1[k] - ref1) <= tol * N * 1e-1 + 1e-12
        state = oracle.run(kind, state, ndim, 1.0, dt, order, params, 1)


def test_cahn_hilliard_mass_drift_on_gpu():
    shape = (1, 128, 192)
    f0 = fields_for(P.PF_CH, shape, 21)
    m0 = oracle.exact_sum(f0[0])
    got, m = gpu_run(P.PF_CH, f0, 2, 4, P.PF_FP64, [1.0, 1.0], 0.01, 200,
                     flags=P.PF_REDUCE_EACH_STEP)
    h, l = m.reduce_history(P.PF_RED_MASS0, 200)
    assert np.max(np.abs((h + l) - m0)) <= 200 * shape[1] * shape[2] * 2.2e-16 * 0.1


@pytest.mark.parametrize("kind", [P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC])
@pytest.mark.parametrize("n", [(5, 3), (2, 1), (64, 1), (3, 4, 2)])
def test_tiny_and_degenerate_grids(kind, n):
    """Extents smaller than the stencil (true periodic wrap), 1D as ny = 1, 1-site axes."""
    order = 8 if len(n) == 2 else 4
    ndim = len(n)
    shape = (n[2] if ndim == 3 else 1, n[1], n[0])
    params = BASE[kind][0]
    dt = 0.5 * dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 3)
    ref = oracle.run(kind, f0, ndim, 1.0, dt, order, params, 40)
    for flags in (0, P.PF_FORCE_GENERIC):
        got, _ = gpu_run(kind, f0, ndim, order, P.PF_FP64, params, dt, 40, flags=flags)
        for g, r in zip(got, ref):
            assert float(np.max(np.abs(g - r))) <= 1e-12


def test_one_dimensional_line_matches_1d_oracle():
    shape = (1, 1, 200)
    f0 = fields_for(P.PF_CH, shape, 4)
    ref = oracle.run(2, f0, 1, 1.0, 0.01, 4, [1.0, 1.0], 100)
    got, _ = gpu_run(P.PF_CH, f0, 2, 4, P.PF_FP64, [1.0, 1.0], 0.01, 100)
    assert float(np.max(np.abs(got[0] - ref[0]))) <= 1e-12


def test_nonfinite_values_are_counted():
    d = P.make_desc(P.PF_AC, (40, 30), dt=0.05)
    m = P.Model(d)
    a = np.zeros((1, 30, 40))
    a[0, 3, 4] = np.nan
    a[0, 10, 11] = np.inf
    m.set_field(0, a)
    assert m.reduce(P.PF_RED_NONFINITE)[0] == 2.0


def test_get_window_matches_full_field():
    d = P.make_desc(P.PF_GS, (30, 20, 10), dt=0.3)
    m = P.Model(d)
    m.init(P.PF_IC_GS_CUBES, 9, (4, 3, 0.01))
    full = m.get_field(1)
    w = m.get_window(1, (8, 15, 25), (5, 9, 11))
    zz, yy, xx = np.meshgrid((np.arange(5) + 8) % 10, (np.arange(9) + 15) % 20,
                             (np.arange(11) + 25) % 30, indexing="ij")
    assert np.array_equal(w, full[zz, yy, xx])


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", [P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC])
@pytest.mark.parametrize("order", [2, 4])
def test_two_step_blocking_is_bitwise_two_single_steps(kind, order, prec):
    """Temporal blocking (two steps per sweep) against one step per sweep over
    101 steps (the last runs alone) with ragged tiles, and against the oracle."""
    shape, ndim = (1, 83, 301), 2
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 31)
    n = (shape[2], shape[1])
    outs = []
    for tb in (1, 2):
        d = P.make_desc(kind, n, dt=dt, order=order, precision=prec, params=params)
        m = P.Model(d)
        m.set_tile(24)
        m.set_time_block(tb)
        assert m.time_block() == tb
        for f, a in enumerate(f0):
            m.set_field(f, a)
        m.step(101)
        assert m.steps_done() == 101
        outs.append([m.get_field(f) for f in range(len(f0))])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    ref = oracle_run(kind, shape, ndim, order, params, dt, 101, 31)[1]
    for g, r in zip(outs[1], ref):
        assert float(np.max(np.abs(g - r))) <= TOL[prec]


@pytest.mark.parametrize("kind", [P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC])
def test_two_step_history_and_graphs(kind):
    """Fused per-step reductions and graph replay with two-step sweeps."""
    shape, ndim, order = (1, 64, 200), 2, 4
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 41)
    n = (shape[2], shape[1])
    hist = []
    fields = []
    for tb, flags in ((1, 0), (2, 0), (2, P.PF_USE_GRAPH)):
        d = P.make_desc(kind, n, dt=dt, order=order, params=params,
                        flags=P.PF_REDUCE_EACH_STEP | flags)
        m = P.Model(d)
        m.set_tile(16)
        m.set_time_block(tb)
        for f, a in enumerate(f0):
            m.set_field(f, a)
        m.step(70)
        which = P.PF_RED_MASS1 if kind in (P.PF_GS, P.PF_MC) else P.PF_RED_ENERGY
        hist.append([sum(m.reduce_history(P.PF_RED_MASS0, 70)), sum(m.reduce_history(which, 70))])
        fields.append([m.get_field(f) for f in range(len(f0))])
    for other in (1, 2):
        for x, y in zip(fields[0], fields[other]):
            assert np.array_equal(x, y)
        for q in range(2):
            a, b = hist[0][q], hist[other][q]
            assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, float(np.max(np.abs(a))))


def test_time_block_refused_where_unavailable():
    d = P.make_desc(P.PF_GS, (40, 30, 20), dt=0.3, order=4)
    m = P.Model(d)
    with pytest.raises(P.PfError) as e:
        m.set_time_block(2)
    assert e.value.status == P.PF_ERR_UNSUPPORTED
    d = P.make_desc(P.PF_AC, (40, 30), dt=0.01, order=8)
    m = P.Model(d)
    with pytest.raises(P.PfError):
        m.set_time_block(2)


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", [P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC])
def test_two_step_blocking_3d(kind, prec):
    """3D two-step sweeps (order 2) against single steps, bitwise, with ragged
    strips, y tiles and z chunks, 101 steps and fused reductions, and against
    the oracle."""
    shape, ndim, order = (29, 37, 150), 3, 2
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 51)
    n = (shape[2], shape[1], shape[0])
    outs, hist = [], []
    for tb in (1, 2):
        d = P.make_desc(kind, n, dt=dt, order=order, precision=prec, params=params,
                        flags=P.PF_REDUCE_EACH_STEP)
        m = P.Model(d)
        m.set_tile(8)
        m.set_time_block(tb)
        for f, a in enumerate(f0):
            m.set_field(f, a)
        m.step(101)
        outs.append([m.get_field(f) for f in range(len(f0))])
        hist.append(sum(m.reduce_history(P.PF_RED_MASS0, 101)))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    assert np.max(np.abs(hist[0] - hist[1])) <= 1e-13 * max(1.0, float(np.max(np.abs(hist[0]))))
    ref = oracle_run(kind, shape, ndim, order, params, dt, 101, 51)[1]
    for g, r in zip(outs[1], ref):
        assert float(np.max(np.abs(g - r))) <= TOL[prec]


@pytest.mark.parametrize("tb", [1, 2])
@pytest.mark.parametrize("kind,order", [(P.PF_AC, 2), (P.PF_AC, 4), (P.PF_GS, 2)])
def test_3d_tile_rows_bitwise(kind, order, tb):
    """FP64 3D Allen-Cahn / Gray-Scott: one and two tile rows per wave give
    bitwise equal fields (ragged strips, y tiles and z chunks, an odd step
    count, fused reductions) that match the oracle."""
    if tb == 2 and order != 2:
        pytest.skip("two-step 3D kernels are built for order 2")
    shape, ndim, steps = (23, 45, 150), 3, 17
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 61)
    n = (shape[2], shape[1], shape[0])
    outs, hist = [], []
    for rows in (1, 2):
        d = P.make_desc(kind, n, dt=dt, order=order, params=params, flags=P.PF_REDUCE_EACH_STEP)
        m = P.Model(d)
        m.set_tile(8)
        m.set_time_block(tb)
        m.set_tile_rows(rows)
        assert m.tile_rows() == rows
        for f, a in enumerate(f0):
            m.set_field(f, a)
        m.step(steps)
        outs.append([m.get_field(f) for f in range(len(f0))])
        hist.append(sum(m.reduce_history(P.PF_RED_MASS0, steps)))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    assert np.max(np.abs(hist[0] - hist[1])) <= 1e-13 * max(1.0, float(np.max(np.abs(hist[0]))))
    ref = oracle_run(kind, shape, ndim, order, params, dt, steps, 61)[1]
    for g, r in zip(outs[0], ref):
        assert float(np.max(np.abs(g - r))) <= TOL[P.PF_FP64]


FOUR_ROWS = [(P.PF_CH, 2, 1), (P.PF_CH, 2, 2), (P.PF_CH, 4, 1), (P.PF_CH, 6, 1), (P.PF_MC, 2, 1),
             (P.PF_MC, 2, 2), (P.PF_MC, 6, 1), (P.PF_GS, 4, 1), (P.PF_GS, 6, 1), (P.PF_GS, 8, 1),
             (P.PF_AC, 8, 1)]


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind,order,tb", FOUR_ROWS, ids=["k%d-p%d-tb%d" % c for c in FOUR_ROWS])
def test_3d_four_rows_per_wave_bitwise(kind, order, tb, prec):
    """3D kernels with four 16-lane rows per wave (8-wave workgroups; 12
    waves and 48-row tiles for CH order 6): bitwise the fields of two rows
    per wave (ragged strips, y tiles and z chunks, an odd step count),
    reductions equal to their compensated accuracy (the 8- and 12-wave items
    clear their unused partial slots), and the oracle."""
    shape, ndim, steps = (23, 45, 150), 3, 17
    params = BASE[kind][0]
    dt = dt_for(kind, ndim, order, params)
    f0 = fields_for(kind, shape, 62)
    n = (shape[2], shape[1], shape[0])
    second = P.PF_RED_MASS1 if kind in (P.PF_GS, P.PF_MC) else P.PF_RED_ENERGY
    outs, hist = [], []
    for rows in (2, 4):
        d = P.make_desc(kind, n, dt=dt, order=order, precision=prec, params=params,
                        flags=P.PF_REDUCE_EACH_STEP)
        m = P.Model(d)
        m.set_passes(1)
        m.set_tile(8)
        m.set_time_block(tb)
        m.set_tile_rows(rows)
        assert m.tile_rows() == rows
        for f, a in enumerate(f0):
            m.set_field(f, a)
        m.step(steps)
        outs.append([m.get_field(f) for f in range(len(f0))])
        hist.append([sum(m.reduce_history(q, steps)) for q in (P.PF_RED_MASS0, second)])
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    for a, b in zip(hist[0], hist[1]):
        assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, float(np.max(np.abs(a))))
    ref = oracle_run(kind, shape, ndim, order, params, dt, steps, 62)[1]
    for g, r in zip(outs[1], ref):
        assert float(np.max(np.abs(g - r))) <= TOL[prec]


def test_tile_rows_defaults_and_refusals():
    gs = P.Model(P.make_desc(P.PF_GS, (40, 30, 20), dt=0.3, order=2))
    assert gs.tile_rows() == 1            # FP64 Gray-Scott default
    gs.set_tile_rows(2)
    assert gs.tile_rows() == 2
    gs.set_tile_rows(0)
    assert gs.tile_rows() == 1
    with pytest.raises(P.PfError) as e:
        gs.set_tile_rows(3)
    assert e.value.status == P.PF_ERR_ARG
    with pytest.raises(P.PfError) as e:
        gs.set_tile_rows(4)               # four rows per wave: not Gray-Scott at r = 1
    assert e.value.status == P.PF_ERR_UNSUPPORTED
    gs6 = P.Model(P.make_desc(P.PF_GS, (40, 30, 20), dt=0.1, order=6))
    assert gs6.tile_rows() == 4           # the default where two rows per wave would spill
    ch = P.Model(P.make_desc(P.PF_CH, (40, 30, 20), dt=0.001, order=2))
    assert ch.tile_rows() == 2
    with pytest.raises(P.PfError) as e:
        ch.set_tile_rows(1)
    assert e.value.status == P.PF_ERR_UNSUPPORTED
    ch.set_tile_rows(4)
    assert ch.tile_rows() == 4
    ac32 = P.Model(P.make_desc(P.PF_AC, (40, 30, 20), dt=0.01, order=2, precision=P.PF_FP32))
    assert ac32.tile_rows() == 2
    with pytest.raises(P.PfError):
        ac32.set_tile_rows(1)
    flat = P.Model(P.make_desc(P.PF_AC, (40, 30), dt=0.01, order=2))
    assert flat.tile_rows() == 0
    with pytest.raises(P.PfError) as e:
        flat.set_tile_rows(2)
    assert e.value.status == P.PF_ERR_UNSUPPORTED


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", [P.PF_AC, P.PF_CH, P.PF_GS, P.PF_MC])
@pytest.mark.parametrize("ndim,shape", [(2, (1, 70, 300)), (3, (20, 37, 150))])
def test_fused_reductions_count_nonfinite_values(kind, ndim, shape, prec):
    """The fused per-step reductions count NaN and infinities exactly (in both
    fields of Gray-Scott), including at strip edges and periodic seams, and do
    not count a finite value whose energy density overflows."""
    f0 = fields_for(kind, shape, 71)
    rng = np.random.default_rng(5)
    sites = [(0, 0, 0), (shape[0] - 1, shape[1] - 1, shape[2] - 1), (0, 5, 63), (0, 6, 64)]
    sites += [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(8)]
    bad = 0
    for i, (z, y, x) in enumerate(sites):
        f = f0[i % len(f0)]
        if np.isfinite(f[z, y, x]):
            f[z, y, x] = (np.nan, np.inf, -np.inf)[i % 3]
            bad += 1
    if kind != P.PF_GS and prec == P.PF_FP64 and np.isfinite(f0[0][0, 1, 1]):
        f0[0][0, 1, 1] = 1e100          # x^4 overflows: energy is infinite, x is not
    n = (shape[2], shape[1]) if ndim == 2 else (shape[2], shape[1], shape[0])
    params = BASE[kind][0]
    d = P.make_desc(kind, n, dt=dt_for(kind, ndim, 2, params), order=2, precision=prec,
                    params=params, flags=P.PF_REDUCE_EACH_STEP)
    m = P.Model(d)
    for i, a in enumerate(f0):
        m.set_field(i, a)
    m.step(1)
    hi, _ = m.reduce_history(P.PF_RED_NONFINITE, 1)
    assert hi[0] == bad


@pytest.mark.parametrize("ndim,shape", [(2, (1, 128, 192)), (3, (40, 44, 70))])
def test_model_c_rho_mass_conserved_on_gpu(ndim, shape):
    """Eq. model-c conserves rho: the fused per-step mass of rho stays at its
    initial exact sum to FP64 rounding (the phi mass is not conserved)."""
    f0 = fields_for(P.PF_MC, shape, 25)
    r0 = oracle.exact_sum(f0[1])
    got, m = gpu_run(P.PF_MC, f0, ndim, 4, P.PF_FP64, [1.0, 1.0, 0.5], 0.01, 200,
                     flags=P.PF_REDUCE_EACH_STEP)
    h, l = m.reduce_history(P.PF_RED_MASS1, 200)
    assert np.max(np.abs((h + l) - r0)) <= 200 * got[1].size * 2.2e-16 * 0.1
