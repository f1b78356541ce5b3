"""pf_step_noalloc (the allocation-free step) through the C ABI against the
model path it is a variant of: a pf_create_on model with the default tile,
one step per launch and the default 3D tile layout, stepped by pf_step and
read back (fields and the per-step reduction history), bitwise.

The no-alloc call runs on copies of the model's initial buffers (torch
tensors with NaN in the row padding and in the second buffer of every field,
so a read of either would show), on a torch stream, with its history in a
torch tensor.  Two calls in a row, the second on a smaller grid, check that
the static scratch left by the first call does not leak into the second.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2511_10508_amd as P

pytestmark = pytest.mark.gpu

RED = P.PF_REDUCE_EACH_STEP

# kind, n (x[, y[, z]]), order, params, dt, ic, ic params, precision, flags, steps
CASES = [
    (P.PF_CH, (301, 75), 4, [1.0, 1.0], 0.01, P.PF_IC_UNIFORM, (-0.05, 0.05), P.PF_FP64, RED, 100),
    (P.PF_CH, (301, 75), 4, [1.0, 1.0], 0.01, P.PF_IC_UNIFORM, (-0.05, 0.05), P.PF_FP32, RED, 100),
    (P.PF_GS, (150, 37, 21), 2, [0.2, 0.1, 0.04, 0.06], 0.5, P.PF_IC_GS_CUBES, (6, 4, 0.01),
     P.PF_FP32, RED, 101),
    (P.PF_AC, (150, 37, 21), 4, [1.0, 1.0], 0.05, P.PF_IC_UNIFORM, (-0.1, 0.1), P.PF_FP64, RED, 40),
    (P.PF_AC, (5000,), 4, [1.0, 1.0], 0.05, P.PF_IC_UNIFORM, (-0.1, 0.1), P.PF_FP64, 0, 64),
    (P.PF_MC, (260, 70), 2, [1.0, 1.0, 0.5], 0.01, P.PF_IC_UNIFORM, (-0.1, 0.1), P.PF_FP32, RED, 50),
    (P.PF_CH, (200, 90), 4, [1.0, 1.0], 0.01, P.PF_IC_UNIFORM, (-0.05, 0.05), P.PF_FP64,
     RED | P.PF_BIHARMONIC_DIRECT, 40),
]


def _id(c):
    return "k%d-%s-p%d-%s-f%d-s%d" % (c[0], "x".join(map(str, c[1])), c[2],
                                      "fp64" if c[7] == P.PF_FP64 else "fp32", c[8], c[9])


def _reference(case, seed):
    """Model path: (desc, initial buffers (clones), fields, history or None)."""
    kind, n, order, params, dt, ic, icp, prec, flags, steps = case
    d = P.make_desc(kind, n, dt=dt, order=order, precision=prec, params=params, flags=flags)
    nf = d.nfields
    elems = P.buffer_elems(d)
    dtype = torch.float64 if prec == P.PF_FP64 else torch.float32
    bufs = [torch.full((elems,), float("nan"), dtype=dtype, device="cuda") for _ in range(2 * nf)]
    torch.cuda.synchronize()
    m = P.Model(d, bufs=[b.data_ptr() for b in bufs])
    m.set_time_block(1)
    if len(n) == 3:
        m.set_tile_rows(0)
    m.set_tile(0)
    m.init(ic, seed, icp)
    m.sync()
    init = [b.clone() for b in bufs]
    torch.cuda.synchronize()
    m.step(steps)
    fields = [m.get_field(f) for f in range(nf)]
    hist = None
    if flags & RED:
        second = P.PF_RED_MASS1 if kind in (P.PF_GS, P.PF_MC) else P.PF_RED_ENERGY
        hist = [m.reduce_history(q, steps) for q in (P.PF_RED_MASS0, second, P.PF_RED_NONFINITE)]
    m.close()
    return d, init, fields, hist


def _check(case, d, bufs, hist_t, fields, hist, parity):
    kind, n, order, params, dt, ic, icp, prec, flags, steps = case
    nf = d.nfields
    shape = tuple(reversed(list(n) + [1] * (3 - len(n))))  # (z, y, x)
    pitch = P.buffer_elems(d) // (shape[0] * shape[1])
    out = parity ^ (steps & 1)
    for f in range(nf):
        t = bufs[2 * f + out][:pitch * shape[0] * shape[1]].view(shape[0], shape[1], pitch)
        got = t[:, :, :n[0]].double().cpu().numpy()
        assert np.array_equal(got, fields[f]), (f, float(np.nanmax(np.abs(got - fields[f]))))
    if hist is not None:
        h = hist_t.view(steps, 3, 2).cpu().numpy()  # dx = 1: the model's values unscaled
        for q in range(3):
            assert np.array_equal(h[:, q, 0], hist[q][0]), q
            if q < 2:
                assert np.array_equal(h[:, q, 1], hist[q][1]), q


def _noalloc(d, bufs, parity, steps, history, stream):
    P.step_noalloc(d, ctypes.c_void_p(stream.cuda_stream), [b.data_ptr() for b in bufs], parity,
                   steps, None if history is None else history.data_ptr())


@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
def test_noalloc_equals_model_path(case):
    d, init, fields, hist = _reference(case, 81)
    steps = case[9]
    hist_t = torch.full((6 * steps,), float("nan"), dtype=torch.float64, device="cuda") \
        if hist is not None else None
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    _noalloc(d, init, 0, steps, hist_t, stream)
    stream.synchronize()
    _check(case, d, init, hist_t, fields, hist, 0)


def test_noalloc_two_calls_second_smaller_and_odd_parity():
    """A large call, then a smaller one starting from buffer 1: each equals
    its model-path reference (the static scratch keeps the first call's
    partials; the second must not read them)."""
    big = (P.PF_CH, (1500, 900), 4, [1.0, 1.0], 0.01, P.PF_IC_UNIFORM, (-0.05, 0.05), P.PF_FP64,
           RED, 30)
    small = (P.PF_CH, (301, 75), 4, [1.0, 1.0], 0.01, P.PF_IC_UNIFORM, (-0.05, 0.05), P.PF_FP64,
             RED, 31)
    rb = _reference(big, 91)
    rs = _reference(small, 92)
    # the small call starts from buffer 1 of every field
    d_s, init_s = rs[0], rs[1]
    for f in range(d_s.nfields):
        init_s[2 * f + 1].copy_(init_s[2 * f])
        init_s[2 * f].fill_(float("nan"))
    hb = torch.full((6 * 30,), float("nan"), dtype=torch.float64, device="cuda")
    hs = torch.full((6 * 31,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    _noalloc(rb[0], rb[1], 0, 30, hb, stream)
    _noalloc(d_s, init_s, 1, 31, hs, stream)
    stream.synchronize()
    _check(big, rb[0], rb[1], hb, rb[2], rb[3], 0)
    _check(small, d_s, init_s, hs, rs[2], rs[3], 1)


def test_noalloc_refuses_what_it_cannot_run():
    """Refusals come before anything is enqueued: over the static scratch, a
    per-site-only descriptor, bad arguments."""
    stream = torch.cuda.Stream()
    dummy = [torch.zeros(16, dtype=torch.float32, device="cuda") for _ in range(4)]
    ptrs = [b.data_ptr() for b in dummy]
    hist = torch.zeros(16, dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(stream.cuda_stream)
    big = P.make_desc(P.PF_GS, (128, 4096, 6144), dt=0.5, order=2, precision=P.PF_FP32, flags=RED)
    with pytest.raises(P.PfError) as e:
        P.step_noalloc(big, s, ptrs, 0, 1, hist.data_ptr())
    assert e.value.status == P.PF_ERR_ARG and "16 MiB" in str(e.value)
    generic = P.make_desc(P.PF_CH, (20, 20, 20), dt=1e-4, order=10)
    with pytest.raises(P.PfError) as e:
        P.step_noalloc(generic, s, ptrs[:2], 0, 1, None)
    assert e.value.status == P.PF_ERR_UNSUPPORTED
    small = P.make_desc(P.PF_CH, (20, 20), dt=0.01, order=4, flags=RED)
    with pytest.raises(P.PfError):
        P.step_noalloc(small, s, ptrs[:2], 2, 1, hist.data_ptr())   # parity
    with pytest.raises(P.PfError):
        P.step_noalloc(small, s, ptrs[:1], 0, 1, hist.data_ptr())   # nbufs
    with pytest.raises(P.PfError):
        P.step_noalloc(small, s, ptrs[:2], 0, 1, None)              # history
    stream.synchronize()
    assert bool((dummy[0] == 0).all())
