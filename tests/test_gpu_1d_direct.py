"""GPU parity of the native 1D kernels and of Cahn-Hilliard with the direct
biharmonic stencil, against the CPU FP64 oracle.

1D grids (ndim = 1) run their own strip-marching kernels; the direct
biharmonic (PF_BIHARMONIC_DIRECT) has fused 1D, 2D and 3D (r <= 2) kernels
and runs the per-site generic kernel beyond them.  Tolerances as in the other parity tests:
max |GPU - oracle| <= 1e-12 (FP64 storage) and <= 1e-4 (FP32 storage) after
100 steps; kernel family, strip layout, two-step blocking and graph replay
are checked bitwise.
"""
import numpy as np
import pytest

import oracle
import synth
import paper_2511_10508_amd as P
import paper_2511_10508_amd.serving as S

pytestmark = pytest.mark.gpu

TOL = {P.PF_FP64: 1e-12, P.PF_FP32: 1e-4}
CHD = "chd"  # Cahn-Hilliard with the direct biharmonic (a descriptor flag on PF_CH)
BASE = {P.PF_AC: ([1.0, 1.0], 0.05), P.PF_CH: ([1.0, 1.0], 0.01), CHD: ([1.0, 1.0], 0.01),
        P.PF_GS: ([0.2, 0.1, 0.04, 0.06], 0.5), P.PF_MC: ([1.0, 1.0, 0.5], 0.01)}
KINDS = [P.PF_AC, P.PF_CH, CHD, P.PF_GS, P.PF_MC]


def _lib_kind(kind):
    return P.PF_CH if kind == CHD else kind


def _bih(kind):
    return "direct" if kind == CHD else "composed"


def _flags(kind):
    return P.PF_BIHARMONIC_DIRECT if kind == CHD else 0


def dt_for(kind, ndim, order, params):
    lim = oracle.dt_max(_lib_kind(kind), ndim, 1.0, order, params, biharmonic=_bih(kind))
    return min(BASE[kind][1], 0.8 * lim)


def fields_for(kind, shape, seed):
    k = _lib_kind(kind)
    if k == P.PF_GS:
        return synth.initial_fields(3, shape, seed, synth.IC_GS_CUBES, (3, 4, 0.01))
    lo_hi = (-0.05, 0.05) if k == P.PF_CH else (-0.1, 0.1)
    return synth.initial_fields(k, shape, seed, synth.IC_UNIFORM, lo_hi)


def gpu_run(kind, fields, ndim, order, prec, params, dt, nsteps, flags=0, chunk=None, tb=None):
    shape = fields[0].shape
    n = {1: (shape[2],), 2: (shape[2], shape[1]), 3: (shape[2], shape[1], shape[0])}[ndim]
    d = P.make_desc(_lib_kind(kind), n, dt=dt, order=order, precision=prec, params=params,
                    flags=flags | _flags(kind))
    m = P.Model(d)
    if chunk:
        m.set_tile(chunk)
    if tb:
        m.set_time_block(tb)
    for f, a in enumerate(fields):
        m.set_field(f, a)
    m.step(nsteps)
    return [m.get_field(f) for f in range(len(fields))], m


def oracle_run(kind, f0, ndim, order, params, dt, nsteps):
    return oracle.run(_lib_kind(kind), f0, ndim, 1.0, dt, order, params, nsteps,
                      biharmonic=_bih(kind))


def _id(k):
    return {P.PF_AC: "ac", P.PF_CH: "ch", CHD: "chd", P.PF_GS: "gs", P.PF_MC: "mc"}[k]


# ------------------------------------------------------------------ 1D --

CASES_1D = [(k, nx, order, chunk) for k in KINDS for (nx, order, chunk) in
            ((1001, 2, 3), (3000, 4, 5), (777, 6, 2))]
CASES_1D += [(P.PF_CH, 2049, 8, 4), (CHD, 1500, 8, 3), (P.PF_AC, 900, 10, None),
             (CHD, 640, 12, None)]


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES_1D, ids=["%s-%d-p%d" % (_id(c[0]), c[1], c[2]) for c in CASES_1D])
def test_1d_parity_100_steps(case, prec):
    kind, nx, order, chunk = case
    params = BASE[kind][0]
    dt = dt_for(kind, 1, order, params)
    f0 = fields_for(kind, (1, 1, nx), 31)
    ref = oracle_run(kind, f0, 1, order, params, dt, 100)
    got, m = gpu_run(kind, f0, 1, order, prec, params, dt, 100, chunk=chunk)
    assert m.tile()[1] == (0 if order <= 8 else 1)
    for g, r in zip(got, ref):
        err = float(np.max(np.abs(g - r)))
        assert err <= TOL[prec], (err, m.tile())


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", KINDS, ids=_id)
def test_1d_fused_equals_generic_bitwise(kind, prec):
    order = 4
    params = BASE[kind][0]
    dt = dt_for(kind, 1, order, params)
    f0 = fields_for(kind, (1, 1, 2500), 5)
    a, ma = gpu_run(kind, f0, 1, order, prec, params, dt, 30, chunk=3)
    b, mb = gpu_run(kind, f0, 1, order, prec, params, dt, 30, flags=P.PF_FORCE_GENERIC)
    assert ma.tile()[1] == 0 and mb.tile()[1] == 1
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", KINDS, ids=_id)
@pytest.mark.parametrize("order", [2, 6])
def test_1d_two_step_and_strip_layout_bitwise(kind, order, prec):
    """Two steps per sweep equal two single steps; strips per wave do not
    change the result; an odd step count ends with one single step."""
    params = BASE[kind][0]
    dt = dt_for(kind, 1, order, params)
    f0 = fields_for(kind, (1, 1, 3333), 6)
    a, _ = gpu_run(kind, f0, 1, order, prec, params, dt, 21, chunk=4, tb=1)
    b, mb = gpu_run(kind, f0, 1, order, prec, params, dt, 21, chunk=4, tb=2)
    c, _ = gpu_run(kind, f0, 1, order, prec, params, dt, 21, chunk=1, tb=2)
    assert mb.time_block() == 2
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)


@pytest.mark.parametrize("kind", KINDS, ids=_id)
@pytest.mark.parametrize("nx", [1, 2, 3, 7, 130, 257])
def test_1d_tiny_and_wrapping_grids(kind, nx):
    """Rows shorter than the stencil or than one strip (true periodic wrap)."""
    order = 8
    params = BASE[kind][0]
    dt = 0.5 * dt_for(kind, 1, order, params)
    f0 = fields_for(kind, (1, 1, nx), 3)
    ref = oracle_run(kind, f0, 1, order, params, dt, 40)
    for flags, tb in ((0, 1), (0, 2), (P.PF_FORCE_GENERIC, None)):
        got, _ = gpu_run(kind, f0, 1, order, P.PF_FP64, params, dt, 40, flags=flags, tb=tb)
        for g, r in zip(got, ref):
            assert float(np.max(np.abs(g - r))) <= 1e-12


def _reductions(kind, state, ndim, order, params):
    mass, energy, _ = oracle.reduce(_lib_kind(kind), state, ndim, 1.0, order, params)
    return mass, energy


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("kind", KINDS, ids=_id)
@pytest.mark.parametrize("tb", [1, 2])
def test_1d_fused_history_matches_oracle(kind, tb, prec):
    """PF_REDUCE_EACH_STEP on 1D grids: entry k reduces the state at the
    start of step k (mass, and energy or the second field's mass)."""
    order = 4
    params = BASE[kind][0]
    dt = dt_for(kind, 1, order, params)
    f0 = fields_for(kind, (1, 1, 4099), 13)
    nsteps = 6
    got, m = gpu_run(kind, f0, 1, order, prec, params, dt, nsteps, flags=P.PF_REDUCE_EACH_STEP,
                     chunk=3, tb=tb)
    two = _lib_kind(kind) in (P.PF_GS, P.PF_MC)
    h0, l0 = m.reduce_history(P.PF_RED_MASS0, nsteps)
    h1, l1 = m.reduce_history(P.PF_RED_MASS1 if two else P.PF_RED_ENERGY, nsteps)
    state = [a.copy() for a in f0]
    if prec == P.PF_FP32:
        state = [a.astype(np.float32).astype(np.float64) for a in state]
    tol = 2e-12 if prec == P.PF_FP64 else 1e-4
    N = state[0].size
    for k in range(nsteps):
        mass, energy = _reductions(kind, state, 1, order, params)
        assert abs(h0[k] + l0[k] - mass[0]) <= tol * N * 1e-2 + 1e-13
        ref1 = mass[1] if two else energy
        assert abs(h1[k] + l1[k] - ref1) <= tol * N * 1e-1 + 1e-12
        state = oracle_run(kind, state, 1, order, params, dt, 1)


def test_1d_graph_replay_equals_eager_bitwise():
    for kind in KINDS:
        params = BASE[kind][0]
        dt = dt_for(kind, 1, 4, params)
        f0 = fields_for(kind, (1, 1, 5000), 9)
        a, _ = gpu_run(kind, f0, 1, 4, P.PF_FP64, params, dt, 33, tb=2)
        b, _ = gpu_run(kind, f0, 1, 4, P.PF_FP64, params, dt, 33, flags=P.PF_USE_GRAPH, tb=2)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


# --------------------------------------------------- direct biharmonic --

CASES_D = [(2, (1, 75, 301), 32, o) for o in (2, 4, 6, 8)]
CASES_D += [(2, (1, 40, 90), 16, 10), (3, (13, 17, 40), 8, 2), (3, (11, 14, 33), 8, 4),
            (3, (21, 37, 150), 8, 2), (3, (19, 35, 140), 6, 4), (3, (9, 12, 30), 4, 6)]


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES_D, ids=["%dd-%s-p%d" % (c[0], "x".join(map(str, c[1])), c[3])
                                                for c in CASES_D])
def test_direct_biharmonic_parity_100_steps(case, prec):
    ndim, shape, chunk, order = case
    params = BASE[CHD][0]
    dt = dt_for(CHD, ndim, order, params)
    f0 = fields_for(CHD, shape, 17)
    ref = oracle_run(CHD, f0, ndim, order, params, dt, 100)
    got, m = gpu_run(CHD, f0, ndim, order, prec, params, dt, 100, chunk=chunk)
    fused = (ndim == 2 and order <= 8) or (ndim == 3 and order <= 6)
    assert m.tile()[1] == (0 if fused else 1)
    err = float(np.max(np.abs(got[0] - ref[0])))
    assert err <= TOL[prec], err


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("ndim,shape,order", [(2, (1, 67, 277), 2), (2, (1, 67, 277), 4),
                                              (2, (1, 67, 277), 6), (3, (19, 35, 140), 2),
                                              (3, (19, 35, 140), 4), (3, (23, 30, 41), 6),
                                              (3, (5, 40, 37), 2), (3, (6, 7, 9), 4)])
def test_direct_biharmonic_fused_equals_generic_bitwise(ndim, shape, order, prec):
    """The fused kernels (2D march; 3D march with z chunks, partial,
    wrapping and thin grids) give bitwise the per-site kernel's fields."""
    params = BASE[CHD][0]
    dt = dt_for(CHD, ndim, order, params)
    f0 = fields_for(CHD, shape, 5)
    a, ma = gpu_run(CHD, f0, ndim, order, prec, params, dt, 30, chunk=16 if ndim == 2 else 7)
    b, mb = gpu_run(CHD, f0, ndim, order, prec, params, dt, 30, flags=P.PF_FORCE_GENERIC)
    assert ma.tile()[1] == 0 and mb.tile()[1] == 1
    assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("order,shape", [(2, (21, 45, 150)), (4, (23, 45, 150)), (6, (19, 53, 140))])
def test_direct_biharmonic_3d_layouts_bitwise(order, shape, prec):
    """3D direct biharmonic in both tile layouts (column tiles; the 3D march
    with four rows per wave, ragged strips, y tiles and z chunks):
    fields bitwise those of the per-site kernel, fused reductions of every
    step equal to their compensated accuracy."""
    params = BASE[CHD][0]
    dt = dt_for(CHD, 3, order, params)
    f0 = fields_for(CHD, shape, 29)
    n = (shape[2], shape[1], shape[0])
    steps = 13
    ref, mg = gpu_run(CHD, f0, 3, order, prec, params, dt, steps,
                      flags=P.PF_FORCE_GENERIC | P.PF_REDUCE_EACH_STEP)
    hist_ref = [sum(mg.reduce_history(q, steps)) for q in (P.PF_RED_MASS0, P.PF_RED_ENERGY)]
    for rows in (2, 4):
        d = P.make_desc(P.PF_CH, n, dt=dt, order=order, precision=prec, params=params,
                        flags=P.PF_BIHARMONIC_DIRECT | P.PF_REDUCE_EACH_STEP)
        m = P.Model(d)
        m.set_tile(8)
        m.set_tile_rows(rows)
        assert m.tile_rows() == rows and m.tile()[1] == 0
        m.set_field(0, f0[0])
        m.step(steps)
        assert np.array_equal(m.get_field(0), ref[0]), rows
        for a, b in zip(hist_ref, [sum(m.reduce_history(q, steps)) for q in (P.PF_RED_MASS0, P.PF_RED_ENERGY)]):
            assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, float(np.max(np.abs(a)))), rows


def test_direct_biharmonic_strip_chunk_invariance_and_graphs_bitwise():
    params = BASE[CHD][0]
    dt = dt_for(CHD, 2, 4, params)
    f0 = fields_for(CHD, (1, 90, 300), 8)
    outs = [gpu_run(CHD, f0, 2, 4, P.PF_FP64, params, dt, 20, chunk=c)[0][0] for c in (7, 32, 512)]
    outs.append(gpu_run(CHD, f0, 2, 4, P.PF_FP64, params, dt, 20, flags=P.PF_USE_GRAPH)[0][0])
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_direct_biharmonic_order2_is_the_composed_scheme():
    """At accuracy 2 both forms are one stencil: the GPU results agree to
    rounding, and at order 4 they differ by the truncation term."""
    f0 = fields_for(P.PF_CH, (1, 64, 96), 4)
    a, _ = gpu_run(CHD, f0, 2, 2, P.PF_FP64, [1.0, 1.0], 0.01, 50)
    b, _ = gpu_run(P.PF_CH, f0, 2, 2, P.PF_FP64, [1.0, 1.0], 0.01, 50)
    assert float(np.max(np.abs(a[0] - b[0]))) <= 1e-13
    c, _ = gpu_run(CHD, f0, 2, 4, P.PF_FP64, [1.0, 1.0], 0.01, 50)
    d, _ = gpu_run(P.PF_CH, f0, 2, 4, P.PF_FP64, [1.0, 1.0], 0.01, 50)
    assert float(np.max(np.abs(c[0] - d[0]))) > 1e-8


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("ndim,shape,generic,order", [(2, (1, 64, 250), False, 4), (2, (1, 30, 40), True, 4),
                                                      (3, (12, 20, 30), True, 4), (3, (14, 40, 70), False, 4),
                                                      (3, (20, 37, 45), False, 2), (3, (18, 21, 40), False, 6)])
def test_direct_biharmonic_history_and_mass(ndim, shape, generic, order, prec):
    """Fused reductions of the direct scheme: mass and energy of the state at
    the start of every step, and mass conservation over the run."""
    params = BASE[CHD][0]
    dt = dt_for(CHD, ndim, order, params)
    f0 = fields_for(CHD, shape, 13)
    nsteps = 6
    flags = P.PF_REDUCE_EACH_STEP | (P.PF_FORCE_GENERIC if generic else 0)
    got, m = gpu_run(CHD, f0, ndim, order, prec, params, dt, nsteps, flags=flags, chunk=16)
    h0, l0 = m.reduce_history(P.PF_RED_MASS0, nsteps)
    h1, l1 = m.reduce_history(P.PF_RED_ENERGY, nsteps)
    state = [a.copy() for a in f0]
    if prec == P.PF_FP32:
        state = [a.astype(np.float32).astype(np.float64) for a in state]
    tol = 2e-12 if prec == P.PF_FP64 else 1e-4
    N = state[0].size
    for k in range(nsteps):
        mass, energy = _reductions(CHD, state, ndim, order, params)
        assert abs(h0[k] + l0[k] - mass[0]) <= tol * N * 1e-2 + 1e-13
        assert abs(h1[k] + l1[k] - energy) <= tol * N * 1e-1 + 1e-12
        state = oracle_run(CHD, state, ndim, order, params, dt, 1)
    m0 = oracle.exact_sum(f0[0])
    drift = float(np.max(np.abs((h0 + l0) - m0)))
    assert drift <= (1e-13 if prec == P.PF_FP64 else 1e-3) * max(1.0, N * 1e-3)


def test_direct_biharmonic_has_no_two_step_kernel_and_no_server():
    d = P.make_desc(P.PF_CH, (40, 30), dt=0.005, order=4, flags=P.PF_BIHARMONIC_DIRECT)
    m = P.Model(d)
    with pytest.raises(P.PfError) as e:
        m.set_time_block(2)
    assert e.value.status == P.PF_ERR_UNSUPPORTED
    srv = S.Server(hbm_budget=1 << 28)
    try:
        for desc in (d, P.make_desc(P.PF_AC, (256,), dt=0.05)):
            with pytest.raises(P.PfError) as e:
                srv.submit(desc, P.PF_IC_UNIFORM, 1, (-0.05, 0.05), 10)
            assert e.value.status == P.PF_ERR_UNSUPPORTED
    finally:
        srv.close()


@pytest.mark.parametrize("n", [(5, 3), (2, 1), (9, 2), (3, 4, 2), (7, 6, 5), (33, 2, 3)])
def test_direct_biharmonic_tiny_and_wrapping_grids(n):
    """Extents smaller than the radius-(r+1) fourth-derivative stencil (true
    periodic wrap), through the fused kernels and the per-site ones."""
    ndim = len(n)
    shape = (n[2] if ndim == 3 else 1, n[1], n[0])
    order = 4
    params = BASE[CHD][0]
    dt = 0.5 * dt_for(CHD, ndim, order, params)
    f0 = fields_for(CHD, shape, 3)
    ref = oracle_run(CHD, f0, ndim, order, params, dt, 40)
    for flags in (0, P.PF_FORCE_GENERIC):
        got, _ = gpu_run(CHD, f0, ndim, order, P.PF_FP64, params, dt, 40, flags=flags)
        assert float(np.max(np.abs(got[0] - ref[0]))) <= 1e-12, flags
