"""GPU parity of the semi-implicit Fourier spectral step (PF_SPECTRAL:
hipFFT transforms on the pitched fields plus the library's element-wise
kernels) against the oracle's numpy scheme (oracle/spectral.py).

The transforms round differently from numpy's, so the bar is a tolerance:
max |GPU - oracle| <= 1e-12 for FP64 storage and <= 1e-4 for FP32 storage
after 100 steps, on grids with odd, even, prime and non-power-of-two extents.
Cahn-Hilliard amplifies its unstable band (0 < K2 < c1) by up to
g = max (1 + dt c1 K2) / (1 + dt K2^2) per step, and any rounding difference
with it until the nonlinear term saturates: at dt = 0.25 (the cases below)
g = 1.06 and g^100 = 300, at dt = 1 g^100 = 1.5e8, where two correct
implementations drift apart by more than 1e-12.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import spectral
import synth
import paper_2511_10508_amd as P

pytestmark = pytest.mark.gpu

TOL = {P.PF_FP64: 1e-12, P.PF_FP32: 1e-4}


def _fields(kind, shape, seed):
    lo_hi = (-0.05, 0.05) if kind == P.PF_CH else (-0.1, 0.1)
    return synth.initial_fields(kind, shape, seed, synth.IC_UNIFORM, lo_hi)


def gpu_run(kind, f0, ndim, prec, params, dx, dt, nsteps, flags=0):
    shape = f0.shape
    n = {1: (shape[2],), 2: (shape[2], shape[1]), 3: (shape[2], shape[1], shape[0])}[ndim]
    d = P.make_desc(kind, n, dx=dx, dt=dt, order=2, precision=prec, params=params,
                    flags=P.PF_SPECTRAL | flags)
    m = P.Model(d)
    m.set_field(0, f0)
    m.step(nsteps)
    return m.get_field(0), m


CASES = [
    (P.PF_CH, 1, (1, 1, 1000), 1.0, 0.25), (P.PF_AC, 1, (1, 1, 777), 1.0, 0.2),
    (P.PF_CH, 2, (1, 96, 130), 1.0, 0.25), (P.PF_AC, 2, (1, 75, 64), 0.9, 0.2),
    (P.PF_CH, 2, (1, 257, 300), 1.0, 0.25), (P.PF_CH, 3, (20, 24, 33), 1.0, 0.25),
    (P.PF_AC, 3, (16, 15, 40), 1.0, 0.2),
]


@pytest.mark.parametrize("prec", [P.PF_FP64, P.PF_FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=["k%d-%dd-%s" % (c[0], c[1], "x".join(map(str, c[2])))
                                              for c in CASES])
def test_spectral_parity_100_steps(case, prec):
    kind, ndim, shape, dx, dt = case
    params = [1.0, 1.0]
    f0 = _fields(kind, shape, 41)[0]
    ref = spectral.run(kind, f0, ndim, dx, dt, params, 100)
    got, m = gpu_run(kind, f0, ndim, prec, params, dx, dt, 100)
    assert m.tile()[1] == 2
    err = float(np.max(np.abs(got - ref)))
    assert err <= TOL[prec], err


@pytest.mark.parametrize("ndim,shape", [(1, (1, 1, 4096)), (2, (1, 128, 96)), (3, (24, 20, 18))])
def test_spectral_mass_history_and_no_energy(ndim, shape):
    """Fused per-step mass reductions of the spectral state: Cahn-Hilliard
    keeps its mass to rounding; the free energy is not offered."""
    f0 = _fields(P.PF_CH, shape, 42)[0]
    got, m = gpu_run(P.PF_CH, f0, ndim, P.PF_FP64, [1.0, 1.0], 1.0, 0.5, 40,
                     flags=P.PF_REDUCE_EACH_STEP)
    h, l = m.reduce_history(P.PF_RED_MASS0, 40)
    m0 = oracle.exact_sum(f0)
    assert float(np.max(np.abs((h + l) - m0))) <= 40 * f0.size * 2.2e-16 * 0.1 + 1e-15
    with pytest.raises(P.PfError) as e:
        m.reduce(P.PF_RED_ENERGY)
    assert e.value.status == P.PF_ERR_UNSUPPORTED


def test_spectral_time_step_far_beyond_the_explicit_limit():
    """dt = 1.5 is 60 times the finite-difference limit of this grid (p = 2)
    and within the scheme's own (2 / c1^2): the run matches the oracle for 20
    steps (g^20 = 1.6e2 of rounding growth) and stays bounded over 400; dt
    above the limit is refused."""
    d = P.make_desc(P.PF_CH, (64, 64), dt=1.5, flags=P.PF_SPECTRAL)
    assert P.stability(d) == 2.0
    f0 = _fields(P.PF_CH, (1, 64, 64), 43)[0]
    ref = spectral.run(P.PF_CH, f0, 2, 1.0, 1.5, [1.0, 1.0], 20)
    got, _ = gpu_run(P.PF_CH, f0, 2, P.PF_FP64, [1.0, 1.0], 1.0, 1.5, 20)
    assert float(np.max(np.abs(got - ref))) <= 1e-12
    got, _ = gpu_run(P.PF_CH, f0, 2, P.PF_FP64, [1.0, 1.0], 1.0, 1.5, 400)
    assert np.all(np.isfinite(got)) and float(np.max(np.abs(got))) < 1.5
    assert abs(float(np.sum(got)) - float(np.sum(f0))) <= 1e-10
    d.dt = 2.1
    with pytest.raises(P.PfError) as e:
        P.Model(d)
    assert e.value.status == P.PF_ERR_UNSTABLE


def test_spectral_descriptor_refusals():
    import paper_2511_10508_amd.serving as S
    for kind, flags in ((P.PF_GS, 0), (P.PF_MC, 0), (P.PF_CH, P.PF_BIHARMONIC_DIRECT),
                        (P.PF_AC, P.PF_USE_GRAPH)):
        d = P.make_desc(kind, (32, 32), dt=0.01, flags=P.PF_SPECTRAL | flags)
        with pytest.raises(P.PfError) as e:
            P.Model(d)
        assert e.value.status == P.PF_ERR_ARG
    srv = S.Server(hbm_budget=1 << 28)
    try:
        with pytest.raises(P.PfError) as e:
            srv.submit(P.make_desc(P.PF_CH, (32, 32), dt=0.01, flags=P.PF_SPECTRAL),
                       P.PF_IC_UNIFORM, 1, (-0.05, 0.05), 10)
        assert e.value.status == P.PF_ERR_UNSUPPORTED
    finally:
        srv.close()


@pytest.mark.parametrize("ndim,shape", [(1, (1, 1, 2)), (1, (1, 1, 3)), (1, (1, 1, 5)), (2, (1, 2, 3)),
                                        (2, (1, 7, 4)), (3, (2, 2, 3)), (3, (3, 5, 2))])
def test_spectral_tiny_grids(ndim, shape):
    """Grids of a few sites per axis, odd and even (the half spectrum of an
    odd row has no Nyquist column)."""
    f0 = _fields(P.PF_CH, shape, 44)[0]
    ref = spectral.run(P.PF_CH, f0, ndim, 1.0, 0.25, [1.0, 1.0], 30)
    got, _ = gpu_run(P.PF_CH, f0, ndim, P.PF_FP64, [1.0, 1.0], 1.0, 0.25, 30)
    assert float(np.max(np.abs(got - ref))) <= 1e-12
