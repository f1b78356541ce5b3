"""Pins of the oracle's semi-implicit Fourier spectral step (oracle/spectral.py).

Each pin comes from outside the code under test: closed-form amplification
factors of single Fourier modes, an explicit O(N^2) discrete Fourier
transform on tiny grids, exact invariants (mass, fixed points), unconditional
decay of the implicit linear part, and agreement with the (separately pinned)
finite-difference oracle in the limit the two schemes share.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import spectral

AC, CH = 1, 2


def _mode(shape, ndim, m, phase=0.3):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    arg = 2 * math.pi * m[2] * x / nx + phase
    if ndim >= 2:
        arg = arg + 2 * math.pi * m[1] * y / ny
    if ndim == 3:
        arg = arg + 2 * math.pi * m[0] * z / nz
    return np.cos(arg)


def _k2(shape, ndim, m, dx):
    nz, ny, nx = shape
    ns = (nx, ny, nz)[:ndim]
    ms = (m[2], m[1], m[0])[:ndim]
    return sum((2 * math.pi * mi / (ni * dx)) ** 2 for mi, ni in zip(ms, ns))


@pytest.mark.parametrize("shape,ndim,m", [
    ((1, 1, 32), 1, (0, 0, 3)), ((1, 1, 32), 1, (0, 0, 16)),
    ((1, 24, 20), 2, (0, 5, 2)), ((1, 24, 20), 2, (0, 12, 10)),
    ((8, 10, 12), 3, (2, 3, 1)), ((8, 10, 12), 3, (4, 5, 6)),
])
@pytest.mark.parametrize("kind,params", [(AC, [0.7, 0.0]), (CH, [0.7, 0.0]), (CH, [0.0, 0.0])])
def test_single_mode_amplification(shape, ndim, m, kind, params):
    """c2 = 0 makes both models linear: one step multiplies a mode by
    (1 + dt c1) / (1 + dt K2) (Model A) or (1 + dt c1 K2) / (1 + dt K2^2)
    (Model B), K2 = |k|^2 of the mode (Nyquist modes included)."""
    dx, dt, n = 0.8, 0.05, 7
    u0 = _mode(shape, ndim, m, phase=0.0 if 16 in m or 12 in m else 0.3)
    K2 = _k2(shape, ndim, m, dx)
    c1 = params[0]
    g = (1 + dt * c1) / (1 + dt * K2) if kind == AC else (1 + dt * c1 * K2) / (1 + dt * K2 * K2)
    out = spectral.run(kind, u0, ndim, dx, dt, params, n)
    assert np.max(np.abs(out - g ** n * u0)) <= 1e-13


def _dft_step(kind, u, ndim, dx, dt, params):
    """The scheme with an explicit complex DFT matrix per axis (no FFT)."""
    axes = list(range(3 - ndim, 3))
    uh = u.astype(complex)
    nh = spectral.nonlinear(kind, u, params).astype(complex)
    K2 = np.zeros(u.shape)
    for a in axes:
        n = u.shape[a]
        j = np.arange(n)
        F = np.exp(-2j * math.pi * np.outer(j, j) / n)
        uh = np.moveaxis(np.tensordot(F, np.moveaxis(uh, a, 0), axes=1), 0, a)
        nh = np.moveaxis(np.tensordot(F, np.moveaxis(nh, a, 0), axes=1), 0, a)
        mm = np.where(j <= n // 2, j, j - n)  # signed frequency
        shp = [1, 1, 1]
        shp[a] = n
        K2 = K2 + ((2 * math.pi * mm / (n * dx)) ** 2).reshape(shp)
    if kind == AC:
        uh = (uh + dt * nh) / (1 + dt * K2)
    else:
        uh = (uh - dt * K2 * nh) / (1 + dt * K2 * K2)
    for a in axes:
        n = u.shape[a]
        j = np.arange(n)
        Fi = np.exp(2j * math.pi * np.outer(j, j) / n) / n
        uh = np.moveaxis(np.tensordot(Fi, np.moveaxis(uh, a, 0), axes=1), 0, a)
    return uh.real


@pytest.mark.parametrize("shape,ndim", [((1, 1, 9), 1), ((1, 1, 8), 1), ((1, 5, 6), 2),
                                        ((1, 4, 4), 2), ((3, 4, 5), 3)])
@pytest.mark.parametrize("kind", [AC, CH])
def test_explicit_dft_brute_force(shape, ndim, kind):
    rng = np.random.default_rng(3)
    u = rng.uniform(-0.8, 0.8, size=shape)
    params, dx, dt = [1.1, 0.9], 0.7, 0.03
    a = spectral.step(kind, u, ndim, dx, dt, params)
    b = _dft_step(kind, u, ndim, dx, dt, params)
    assert np.max(np.abs(a - b)) <= 1e-13


@pytest.mark.parametrize("shape,ndim", [((1, 1, 64), 1), ((1, 48, 40), 2), ((10, 12, 14), 3)])
def test_cahn_hilliard_mass_conserved(shape, ndim):
    rng = np.random.default_rng(4)
    c = rng.uniform(-0.05, 0.05, size=shape)
    m0 = oracle.exact_sum(c)
    out = spectral.run(CH, c, ndim, 1.0, 0.5, [1.0, 1.0], 50)
    assert abs(oracle.exact_sum(out) - m0) <= 50 * c.size * 2.2e-16 * 0.05


def test_allen_cahn_uniform_fixed_points():
    for v in (1.0, -1.0, 0.0):
        u = np.full((1, 16, 16), v)
        out = spectral.run(AC, u, 2, 1.0, 0.7, [1.0, 1.0], 10)
        assert np.array_equal(out, u)


@pytest.mark.parametrize("kind,params", [(AC, [1.0, 1.0]), (AC, [0.6, 1.5]), (CH, [1.0, 1.0]),
                                         (CH, [0.7, 1.2])])
def test_dt_max_separates_growth_from_decay(kind, params):
    """About a separated uniform state u = sqrt(c1/c2), a small perturbation
    (the uniform shift for Model A, the mode with K2 = c1 for Model B, the
    most amplified one) decays just below dt_max and grows just above it."""
    c1, c2 = params
    u_star = math.sqrt(c1 / c2)
    n = 16
    if kind == AC:
        dx, pert = 1.0, np.full((1, 1, n), 1e-6)
    else:
        dx = 2 * math.pi * 2 / (n * math.sqrt(c1))  # mode m = 2 has K2 = c1
        pert = 1e-6 * _mode((1, 1, n), 1, (0, 0, 2), phase=0.0)
    lim = spectral.dt_max(kind, params)
    grow = spectral.run(kind, u_star + pert, 1, dx, 1.03 * lim, params, 300)
    decay = spectral.run(kind, u_star + pert, 1, dx, 0.97 * lim, params, 300)
    assert np.max(np.abs(grow - u_star)) > 1e-5
    assert np.max(np.abs(decay - u_star)) < 1e-6


def test_linear_part_is_unconditionally_stable():
    """dt far beyond any explicit limit: with c1 = c2 = 0 every non-constant
    mode of either model decays, and nothing grows."""
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-1, 1, size=(1, 32, 32))
    for kind in (AC, CH):
        u = u0
        norms = [np.linalg.norm(u - u0.mean())]
        for _ in range(20):
            u = spectral.step(kind, u, 2, 1.0, 100.0, [0.0, 0.0])
            norms.append(np.linalg.norm(u - u0.mean()))
        assert all(b < a for a, b in zip(norms, norms[1:]))
        assert abs(u.mean() - u0.mean()) <= 1e-15 or kind == AC


@pytest.mark.parametrize("kind,dt", [(AC, 1e-3), (CH, 1e-4)])
def test_agrees_with_finite_differences_on_resolved_fields(kind, dt):
    """On a field with a few low modes and a small time step the spectral and
    the (order-16) finite-difference schemes solve the same equation: they
    agree to the time-discretisation and truncation error."""
    shape = (1, 64, 64)
    u0 = 0.3 * _mode(shape, 2, (0, 2, 1)) + 0.2 * _mode(shape, 2, (0, 1, 3), phase=1.1)
    params = [1.0, 1.0]
    n = 20
    a = spectral.run(kind, u0, 2, 1.0, dt, params, n)
    b = oracle.run(kind, [u0], 2, 1.0, dt, 16, params, n)[0]
    change = np.max(np.abs(b - u0))
    assert change > 1e-5
    assert np.max(np.abs(a - b)) <= 1e-3 * change
