"""The C-ABI boundary with PyTorch memory and streams, and checkpoint / resume.

pf_create_on steps device buffers the caller owns -- torch tensors here, of
pf_buffer_elems elements each, their row padding filled with NaN so that a
read outside the grid would show -- on the caller's stream (a
torch.cuda.Stream's hipStream_t).  The state must live in those tensors and
be bitwise the state of a model whose buffers and stream the library owns,
and match the oracle after 100 steps.  Checkpoint / resume: n1 steps,
pf_get_field of every field, a new model, pf_set_field + pf_set_steps_done,
n2 steps: bitwise the fields of n1 + n2 steps in one model.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2511_10508_amd as P

pytestmark = pytest.mark.gpu

TOL = {P.PF_FP64: 1e-12, P.PF_FP32: 1e-4}

# kind, n (x, y[, z]), order, params, dt, ic, ic params, oracle ic code
CASES = [
    (P.PF_CH, (301, 75), 4, [1.0, 1.0], 0.01, P.PF_IC_UNIFORM, (-0.05, 0.05), synth.IC_UNIFORM),
    (P.PF_AC, (150, 37, 21), 2, [1.0, 1.0], 0.05, P.PF_IC_UNIFORM, (-0.1, 0.1), synth.IC_UNIFORM),
    (P.PF_GS, (150, 37, 21), 2, [0.2, 0.1, 0.04, 0.06], 0.5, P.PF_IC_GS_CUBES, (6, 4, 0.01),
     synth.IC_GS_CUBES),
    (P.PF_MC, (260, 70), 2, [1.0, 1.0, 0.5], 0.01, P.PF_IC_UNIFORM, (-0.1, 0.1), synth.IC_UNIFORM),
]


def _id(c):
    return "k%d-%s-p%d" % (c[0], "x".join(map(str, c[1])), c[2])


def _shape(n):
    return (n[2] if len(n) == 3 else 1, n[1], n[0])


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
def test_torch_buffers_and_stream(case, prec):
    kind, n, order, params, dt, ic, icp, oic = case
    seed, steps = 61, 100
    d = P.make_desc(kind, n, dt=dt, order=order, precision=prec, params=params,
                    flags=P.PF_REDUCE_EACH_STEP)
    nf = d.nfields
    elems = P.buffer_elems(d)
    dtype = torch.float64 if prec == P.PF_FP64 else torch.float32
    bufs = [torch.full((elems,), float("nan"), dtype=dtype, device="cuda") for _ in range(2 * nf)]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    m = P.Model(d, stream=ctypes.c_void_p(stream.cuda_stream), bufs=[b.data_ptr() for b in bufs])
    assert m.stream() == stream.cuda_stream
    m.init(ic, seed, icp)
    m.autotune(2)
    m.step(steps)
    stream.synchronize()
    shape = _shape(n)
    got = [m.get_field(f) for f in range(nf)]
    hist = m.reduce_history(P.PF_RED_MASS0, steps)
    chunk, tb = m.tile()[0], m.time_block()
    rows = m.tile_rows()
    # the state is in the torch tensors, at the pitch the library reports
    for f in range(nf):
        ptr, pitch, eb = m.field_device(f)
        assert eb == (8 if prec == P.PF_FP64 else 4)
        t = bufs[[b.data_ptr() for b in bufs].index(ptr)]
        view = t[:pitch * shape[1] * shape[0]].view(shape[0], shape[1], pitch)
        assert np.array_equal(view[:, :, :n[0]].double().cpu().numpy(), got[f])
        # the row padding was neither read into the state nor written
        assert bool(torch.isnan(view[:, :, n[0]:]).all()) if pitch > n[0] else True
    m.close()
    # a model whose buffers and stream the library owns, same tile: bitwise
    o = P.Model(d)
    o.set_tile(chunk)
    if tb == 2:
        o.set_time_block(2)
    if rows:
        o.set_tile_rows(rows)
    o.init(ic, seed, icp)
    o.step(steps)
    for f in range(nf):
        assert np.array_equal(o.get_field(f), got[f])
    ohist = o.reduce_history(P.PF_RED_MASS0, steps)
    assert np.array_equal(ohist[0], hist[0]) and np.array_equal(ohist[1], hist[1])
    o.close()
    # and the oracle
    f0 = synth.initial_fields(kind, shape, seed, oic, icp)
    ref = oracle.run(kind, f0, len(n), 1.0, dt, order, params, steps)
    for f in range(nf):
        assert float(np.max(np.abs(got[f] - ref[f]))) <= TOL[prec]


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
def test_checkpoint_resume_bitwise(case, prec):
    kind, n, order, params, dt, ic, icp, oic = case
    seed, n1, n2 = 71, 37, 63
    d = P.make_desc(kind, n, dt=dt, order=order, precision=prec, params=params)
    nf = d.nfields

    def fresh():
        m = P.Model(d)
        m.set_tile(8)
        try:
            m.set_time_block(2)  # odd n1: the resumed run splits a two-step pair
        except P.PfError:
            pass
        return m

    a = fresh()
    a.init(ic, seed, icp)
    a.step(n1 + n2)
    straight = [a.get_field(f) for f in range(nf)]
    a.close()
    b = fresh()
    b.init(ic, seed, icp)
    b.step(n1)
    ckpt = [b.get_field(f) for f in range(nf)]
    done = b.steps_done()
    b.close()
    assert done == n1
    c = fresh()
    for f in range(nf):
        c.set_field(f, ckpt[f])
    c.set_steps_done(done)
    c.step(n2)
    assert c.steps_done() == n1 + n2
    for f in range(nf):
        assert np.array_equal(c.get_field(f), straight[f])
    c.close()
