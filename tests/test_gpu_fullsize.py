"""Full-size parity on sampled outputs, in the launch configuration bench.py
times (autotuned chunk and time block, fused reductions every step).

After n steps a site depends only on the initial data within n*H of it (H = r
for AC/GS, 2r for CH), so the oracle runs on a periodic window of the seeded
initial field of side W + 2 n H (generated directly by synth, whose
counter-based values are the ones pf_init writes) and its central W x W (x W)
block must match the GPU's window of the full grid.  Windows include the
periodic seams.  The headline grids run 100 steps (2D CH 32768^2: windows of
24^2 from 824^2 light cones; 3D GS 1024^3: 14^3 from 214^3).
"""
import numpy as np
import pytest

import oracle
import synth
import paper_2511_10508_amd as P

pytestmark = pytest.mark.gpu

TOL = {P.PF_FP64: 1e-12, P.PF_FP32: 1e-4}


def _check_windows(m, kind, ndim, n, order, params, dt, steps, seed, ic, icp, halo, windows, W, prec):
    nf = 2 if kind in (P.PF_GS, P.PF_MC) else 1
    shape = (n[2] if ndim == 3 else 1, n[1], n[0])
    margin = steps * halo
    for origin in windows:
        o = tuple(origin)
        win = tuple(W if (ndim == 3 or a > 0) else 1 for a in range(3))
        big = tuple(w + 2 * margin if (ndim == 3 or a > 0) else 1 for a, w in enumerate(win))
        org_big = tuple((o[a] - margin) if (ndim == 3 or a > 0) else 0 for a in range(3))
        f0 = synth.initial_fields(kind, shape, seed, ic, icp, origin=org_big, wshape=big)
        ref = oracle.run(kind, f0, ndim, 1.0, dt, order, params, steps)
        for f in range(nf):
            got = m.get_window(f, o, win)
            sl = tuple(slice(margin, margin + win[a]) if (ndim == 3 or a > 0) else slice(0, 1)
                       for a in range(3))
            err = float(np.max(np.abs(got - ref[f][sl])))
            assert err <= TOL[prec], (origin, f, err)


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
def test_cahn_hilliard_32768_sampled(prec):
    """2D CH 32768^2, dx 1, dt 0.01, order 4 twice, c0 = U[-0.05, 0.05] seed 202."""
    n, order, params, dt, steps, seed = (32768, 32768, 1), 4, [1.0, 1.0], 0.01, 100, 202
    d = P.make_desc(P.PF_CH, n[:2], dt=dt, order=order, precision=prec, params=params,
                    flags=P.PF_REDUCE_EACH_STEP)
    m = P.Model(d)
    m.init(P.PF_IC_UNIFORM, seed, (-0.05, 0.05))
    m.autotune(2)
    print("tile", m.tile(), "time block", m.time_block(), flush=True)
    m.step(steps)
    m.sync()
    hi, lo = m.reduce_history(P.PF_RED_MASS0, steps)
    drift = np.max(np.abs((hi + lo) - (hi[0] + lo[0])))
    if prec == P.PF_FP64:  # conservation up to FP64 rounding of the updates
        assert drift <= steps * 32768 ** 2 * 2.3e-16 * 0.1
    else:  # FP32 storage rounds every update: a random walk of ~sqrt(N) eps32 |c| per step
        assert drift <= 10 * steps * 32768 * 6e-8 * 0.05
    windows = [(0, 0, 0), (0, 32768 - 11, 32768 - 13), (0, 12345, 30001), (0, 1, 20000)]
    _check_windows(m, P.PF_CH, 2, n, order, params, dt, steps, seed, synth.IC_UNIFORM,
                   (-0.05, 0.05), 2 * 2, windows, 24, prec)
    m.close()


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
def test_gray_scott_1024_cubed_sampled(prec):
    """3D GS 1024^3, dt 0.5, order 2, 20 cubes of side 16 + 1 % noise, seed 303."""
    n, order, params, dt, steps, seed = (1024, 1024, 1024), 2, [0.2, 0.1, 0.04, 0.06], 0.5, 100, 303
    d = P.make_desc(P.PF_GS, n, dt=dt, order=order, precision=prec, params=params)
    m = P.Model(d)
    m.init(P.PF_IC_GS_CUBES, seed, (20, 16, 0.01))
    m.autotune(2)
    print("tile", m.tile(), "time block", m.time_block(), flush=True)
    m.step(steps)
    m.sync()
    corners = synth.cube_corners(seed, (1024, 1024, 1024), 20)
    cz, cy, cx = corners[0]
    windows = [(0, 0, 0), (1024 - 7, 1024 - 9, 1024 - 5), (cz, cy, cx)]
    _check_windows(m, P.PF_GS, 3, n, order, params, dt, steps, seed, synth.IC_GS_CUBES,
                   (20, 16, 0.01), 1, windows, 14, prec)
    m.close()


@pytest.mark.parametrize("order", [2, 4, 6])
def test_cahn_hilliard_512_cubed_sampled(order):
    """3D CH 512^3 (precision-study grid), dt 0.005, orders 2 / 4 / 6, FP64 and FP32."""
    n, params, dt, steps, seed = (512, 512, 512), [1.0, 1.0], 0.005, 6, 404
    for prec in (P.PF_FP64, P.PF_FP32):
        d = P.make_desc(P.PF_CH, n, dt=dt, order=order, precision=prec, params=params,
                        flags=P.PF_REDUCE_EACH_STEP)
        m = P.Model(d)
        m.init(P.PF_IC_UNIFORM, seed, (-0.05, 0.05))
        m.step(steps)
        m.sync()
        windows = [(0, 0, 0), (511, 300, 7)]
        _check_windows(m, P.PF_CH, 3, n, order, params, dt, steps, seed, synth.IC_UNIFORM,
                       (-0.05, 0.05), order, windows, 8, prec)
        m.close()
