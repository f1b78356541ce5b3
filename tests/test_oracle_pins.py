"""Pins of the CPU FP64 oracle against what the paper and mathematics fix.

Every part of the oracle is checked against something other than itself:
closed forms, exact discrete eigenvalues, invariants, special cases, the
paper's printed table, exact-rational brute force and convergence rates.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import AC, CH, GS, MC
from oracle.exact import run_exact
from oracle.weights import (first_derivative_weights_exact, fourth_derivative_weights_exact,
                            second_derivative_weights_exact)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- weights --

def _closed_form(order):
    """w_j = 2 (-1)^(j+1) (r!)^2 / (j^2 (r-j)! (r+j)!), w_0 = -2 sum w_j."""
    r = order // 2
    w = [Fraction(0)] * (r + 1)
    for j in range(1, r + 1):
        w[j] = Fraction(2 * (-1) ** (j + 1) * math.factorial(r) ** 2,
                        j * j * math.factorial(r - j) * math.factorial(r + j))
    w[0] = -2 * sum(w[1:])
    return w


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_weights_polynomial_exactness(order):
    w = second_derivative_weights_exact(order)
    r = order // 2
    full = {j: w[abs(j)] for j in range(-r, r + 1)}
    for k in range(0, 2 * r + 2):
        moment = sum(wj * Fraction(j) ** k for j, wj in full.items())
        assert moment == (2 if k == 2 else 0), (order, k)
    # accuracy is exactly p, not more: the next even moment is non-zero
    k = 2 * r + 2
    assert sum(wj * Fraction(j) ** k for j, wj in full.items()) != 0


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_weights_closed_form(order):
    assert second_derivative_weights_exact(order) == _closed_form(order)


def test_weights_golden_table():
    with open(os.path.join(GOLDEN, "centered_d2_weights.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 4
    for line in rows:
        p, vals = line.split(":")
        expect = [Fraction(v) for v in vals.split()]
        assert second_derivative_weights_exact(int(p)) == expect


def test_weights_fp64_correctly_rounded():
    for order in (2, 4, 6, 8, 12, 16):
        exact = second_derivative_weights_exact(order)
        for e, f in zip(exact, oracle.second_derivative_weights(order)):
            err = abs(Fraction(f) - e)
            assert err <= Fraction(math.ulp(f)) / 2


# ------------------------------------------------------- Fourier eigenpins --

def _eig(order, thetas, dx):
    w = [float(v) for v in _closed_form(order)]
    lam = 0.0
    for th in thetas:
        lam += (w[0] + 2 * sum(w[j] * math.cos(j * th) for j in range(1, len(w)))) / dx ** 2
    return lam


@pytest.mark.parametrize("order", [2, 4, 6, 8])
@pytest.mark.parametrize("shape,ndim,modes", [
    ((1, 18, 24), 2, (0, 2, 5)),
    ((1, 18, 24), 2, (0, 7, 0)),
    ((1, 18, 24), 2, (0, 0, 11)),
    ((8, 10, 12), 3, (3, 1, 4)),
    ((8, 10, 12), 3, (4, 0, 0)),
])
def test_laplacian_fourier_eigenvalue(order, shape, ndim, modes):
    nz, ny, nx = shape
    dx = 0.7
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    thetas = [2 * math.pi * modes[2] / nx, 2 * math.pi * modes[1] / ny]
    if ndim == 3:
        thetas.append(2 * math.pi * modes[0] / nz)
    phase = thetas[0] * x + thetas[1] * y + (thetas[2] * z if ndim == 3 else 0)
    for u in (np.cos(phase + 0.3), np.sin(phase)):
        lu = oracle.laplacian(u, ndim, dx, order)
        lam = _eig(order, thetas, dx)
        scale = sum(abs(float(v)) for v in _closed_form(order)) * 2 * ndim / dx ** 2
        assert np.max(np.abs(lu - lam * u)) <= 4e-16 * scale * 8


def test_laplacian_dimension_reduction():
    """A 2D grid with ny = 1 gives exactly the 1D result; constants are exact zeros."""
    rng = np.random.default_rng(1)
    u = rng.uniform(-1, 1, size=(1, 1, 37))
    for order in (2, 4, 6):
        a = oracle.laplacian(u, 1, 0.5, order)
        b = oracle.laplacian(u, 2, 0.5, order)
        c = oracle.laplacian(np.broadcast_to(u, (5, 1, 37)), 3, 0.5, order)
        assert np.array_equal(a, b)
        assert np.array_equal(np.broadcast_to(a, (5, 1, 37)), c)
        k = oracle.laplacian(np.full((3, 4, 5), 0.123456789), 3, 0.3, order)
        assert np.all(k == 0.0)


def test_laplacian_stencil_wider_than_grid():
    """Periodic wrap with a true modulo: a radius-4 stencil on a 3-site axis."""
    u = np.array([[[1.0, 2.0, 4.0]]])
    w = second_derivative_weights_exact(8)
    expect = []
    for i in range(3):
        acc = Fraction(0)
        for j in range(1, 5):
            acc += w[j] * (Fraction(u[0, 0, (i + j) % 3]) + Fraction(u[0, 0, (i - j) % 3]) - 2 * Fraction(u[0, 0, i]))
        expect.append(float(acc))
    got = oracle.laplacian(u, 1, 1.0, 8)[0, 0]
    assert np.allclose(got, expect, rtol=0, atol=1e-14)


# -------------------------------------------------- single-mode decay pins --

def _mode(shape, ndim, modes):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    th = [2 * math.pi * modes[2] / nx, 2 * math.pi * modes[1] / ny, 2 * math.pi * modes[0] / nz]
    phase = th[0] * x + th[1] * y + (th[2] * z if ndim == 3 else 0)
    return np.cos(phase), th[:ndim]


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("shape,ndim,modes", [((1, 1, 22), 1, (0, 0, 3)), ((1, 16, 20), 2, (0, 3, 2)),
                                               ((6, 8, 10), 3, (1, 2, 3))])
def test_single_mode_decay_all_models(order, shape, ndim, modes):
    dx, n = 1.0, 25
    m, th = _mode(shape, ndim, modes)
    lam = _eig(order, th, dx)
    A0 = 0.01
    cases = [
        (AC, [0.0, 0.0], 0.02, 1 + 0.02 * lam),
        (AC, [0.7, 0.0], 0.02, 1 + 0.02 * (lam + 0.7)),
        (CH, [0.0, 0.0], 0.002, 1 - 0.002 * lam * lam),
        (CH, [0.7, 0.0], 0.002, 1 + 0.002 * (-0.7 * lam - lam * lam)),
    ]
    for kind, params, dt, g in cases:
        out = oracle.run(kind, [A0 * m], ndim, dx, dt, order, params, n)[0]
        assert np.max(np.abs(out - A0 * g ** n * m)) <= 1e-15 * n * 4, (kind, params)
    # Gray-Scott with v = 0: u = 1 + A mode decays with 1 + dt (Du lam - F)
    Du, Dv, F, k, dt = 0.2, 0.1, 0.04, 0.06, 0.3
    u0, v0 = 1.0 + A0 * m, np.zeros(shape)
    u, v = oracle.run(GS, [u0, v0], ndim, dx, dt, order, [Du, Dv, F, k], n)
    g = 1 + dt * (Du * lam - F)
    assert np.max(np.abs(u - (1 + A0 * g ** n * m))) <= 1e-15 * n * 4
    assert np.all(v == 0.0)


# -------------------------------------------------------------- invariants --

@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("shape,ndim", [((1, 24, 30), 2), ((8, 9, 10), 3)])
def test_cahn_hilliard_mass_conservation(order, shape, ndim):
    rng = np.random.default_rng(7)
    c = rng.uniform(-0.05, 0.05, size=shape)
    nsteps = 40
    m0 = oracle.exact_sum(c)
    drift = []
    for _ in range(4):
        c = oracle.run(CH, [c], ndim, 1.0, 0.005, order, [1.0, 1.0], nsteps // 4)[0]
        drift.append(abs(oracle.exact_sum(c) - m0))
    N = c.size
    bound = nsteps * N * 2.2e-16 * 0.1
    assert max(drift) <= bound


@pytest.mark.parametrize("order", [2, 4, 6, 8])
@pytest.mark.parametrize("shape,ndim", [((1, 12, 14), 2), ((5, 6, 7), 3)])
def test_gray_scott_trivial_fixed_point_bitwise(order, shape, ndim):
    u, v = np.ones(shape), np.zeros(shape)
    u2, v2 = oracle.run(GS, [u, v], ndim, 1.0, 0.5, order, [0.2, 0.1, 0.04, 0.06], 20)
    assert np.array_equal(u2, u) and np.array_equal(v2, v)


def _gs_fixed_points(F, k):
    """Homogeneous fixed points with v != 0: u v = F + k, (F+k) v^2 - F v + F (F+k) = 0."""
    a, b, c = F + k, -F, F * (F + k)
    disc = b * b - 4 * a * c
    if disc < 0:
        return []
    vs = [(-b + s * math.sqrt(max(disc, 0.0))) / (2 * a) for s in (1, -1)]
    return [((F + k) / v, v) for v in vs]


@pytest.mark.parametrize("F,k", [(0.04, 0.06), (0.03, 0.05), (0.02, 0.05)])
def test_gray_scott_nontrivial_fixed_point(F, k):
    """Every reaction term takes part; a wrong sign or a dropped term moves the state."""
    shape = (3, 4, 5)
    for u_s, v_s in _gs_fixed_points(F, k):
        u, v = np.full(shape, u_s), np.full(shape, v_s)
        u2, v2 = oracle.run(GS, [u, v], 3, 1.0, 0.1, 2, [0.2, 0.1, F, k], 10)
        assert np.max(np.abs(u2 - u_s)) < 1e-13
        assert np.max(np.abs(v2 - v_s)) < 1e-13
        # a perturbed state does move (the pin is not vacuous)
        u3, v3 = oracle.run(GS, [u * 1.01, v], 3, 1.0, 0.1, 2, [0.2, 0.1, F, k], 1)
        assert np.max(np.abs(u3 - u * 1.01)) > 1e-6


def test_gray_scott_homogeneous_reaction_euler():
    """Spatially constant state: L = 0 exactly, so one step is the ODE's Euler step.

    Checked against the rate functions written as a polynomial in (u, v) with
    the constants of the reaction network A: u + 2v -> 3v (rate uv^2), feed
    F(1-u), removal (F+k) v, evaluated in exact rationals.
    """
    Du, Dv, F, k, dt = 0.2, 0.1, 0.04, 0.06, 0.25
    u_s, v_s = 0.37, 0.61
    u, v = oracle.run(GS, [np.full((1, 3, 3), u_s), np.full((1, 3, 3), v_s)], 2, 1.0, dt, 4,
                      [Du, Dv, F, k], 1)
    U, V, Fq, Kq, T = (Fraction(x) for x in (u_s, v_s, F, k, dt))
    react = U * V * V
    assert abs(u[0, 0, 0] - float(U + T * (Fq * (1 - U) - react))) < 1e-16
    assert abs(v[0, 0, 0] - float(V + T * (react - (Fq + Kq) * V))) < 1e-16


# ------------------------------------------------------ tanh profile pins --

def _kinks(n, h, L):
    x = np.arange(n) * h
    s = 1 / math.sqrt(2)
    return np.tanh((x - L / 4) * s) * np.tanh((3 * L / 4 - x) * s)


@pytest.mark.parametrize("kind,order", [(AC, 2), (AC, 4), (CH, 2), (CH, 4)])
def test_tanh_profile_convergence_rate(kind, order):
    """phi* = tanh(x / sqrt 2) is stationary for c1 = c2 = 1; the scheme keeps it to O(h^p)."""
    L = 40.0
    errs = []
    for n in (80, 160):
        h = L / n
        phi = _kinks(n, h, L)[None, None, :]
        if kind == AC:
            dt, T = 0.1 * h * h, 2.0
        else:
            dt, T = 0.02 * h ** 4, 0.25
        nsteps = int(round(T / dt))
        out = oracle.run(kind, [phi], 1, h, dt, order, [1.0, 1.0], nsteps)[0]
        errs.append(np.max(np.abs(out - phi)))
    rate = math.log2(errs[0] / errs[1])
    assert order - 0.6 < rate < order + 0.6, (errs, rate)


def test_tanh_profile_sign_pins():
    """A wrong sign on c1 or c2 destroys the kink: the profile stays put only with the paper's signs."""
    L, n = 40.0, 160
    h = L / n
    phi = _kinks(n, h, L)[None, None, :]
    good = oracle.run(AC, [phi], 1, h, 0.1 * h * h, 4, [1.0, 1.0], 200)[0]
    bad = oracle.run(AC, [phi], 1, h, 0.1 * h * h, 4, [-1.0, -1.0], 200)[0]
    assert np.max(np.abs(good - phi)) < 1e-4
    assert np.max(np.abs(bad - phi)) > 1e-2


# ---------------------------------------------------- exact-rational brute --

@pytest.mark.parametrize("kind,shape,ndim,order,params,dt", [
    (AC, (1, 4, 4), 2, 2, [1.0, 1.0], 0.05),
    (AC, (1, 4, 4), 2, 4, [0.9, 1.3], 0.05),
    (CH, (1, 4, 4), 2, 4, [1.0, 1.0], 0.01),
    (CH, (3, 3, 3), 3, 2, [1.1, 0.8], 0.01),
    (GS, (3, 3, 3), 3, 2, [0.2, 0.1, 0.04, 0.06], 0.5),
    (GS, (1, 4, 4), 2, 6, [0.2, 0.1, 0.04, 0.06], 0.3),
    (AC, (1, 1, 9), 1, 4, [1.0, 1.0], 0.05),
    (CH, (1, 1, 11), 1, 6, [1.0, 1.0], 0.01),
    (GS, (1, 1, 7), 1, 2, [0.2, 0.1, 0.04, 0.06], 0.5),
])
def test_exact_rational_brute_force(kind, shape, ndim, order, params, dt):
    rng = np.random.default_rng(11)
    nf = 2 if kind == GS else 1
    fields = [rng.uniform(0.0, 1.0, size=shape) for _ in range(nf)]
    nsteps = 4
    got = oracle.run(kind, fields, ndim, 1.0, dt, order, params, nsteps)
    ex = run_exact(kind, fields, ndim, 1.0, dt, order, params, nsteps)
    for g, e in zip(got, ex):
        e = np.array([[[float(v) for v in row] for row in pl] for pl in e])
        assert np.max(np.abs(g - e)) < 5e-15


# ----------------------------------------------------------- energy pins --

def test_energy_constant_field_closed_form():
    a, c1, c2, dx = 0.3, 1.2, 0.7, 0.5
    x = np.full((4, 5, 6), a)
    m, e, bad = oracle.reduce(AC, [x], 3, dx, 4, [c1, c2])
    N = x.size
    assert bad == 0
    assert math.isclose(m[0], N * a * dx ** 3, rel_tol=1e-15)
    assert math.isclose(e, N * dx ** 3 * (-c1 * a * a / 2 + c2 * a ** 4 / 4), rel_tol=1e-14)


def test_energy_p2_summation_by_parts():
    """For p = 2 the gradient term -1/2 sum x L x equals 1/2 sum |forward difference|^2."""
    rng = np.random.default_rng(3)
    dx = 0.8
    for shape, ndim in (((1, 9, 11), 2), ((5, 6, 7), 3)):
        x = rng.uniform(-1, 1, size=shape)
        _, e, _ = oracle.reduce(AC, [x], ndim, dx, 2, [0.0, 0.0])
        g = 0.0
        for ax in range(ndim):
            d = (np.roll(x, -1, axis=2 - ax) - x) / dx
            g += 0.5 * float(np.sum(d * d))
        assert math.isclose(e, g * dx ** ndim, rel_tol=1e-12)


@pytest.mark.parametrize("order", [2, 4])
def test_allen_cahn_is_gradient_flow_of_energy(order):
    """AC rhs_i = -(1/dx^d) dF/dx_i, by central differences of the oracle energy."""
    rng = np.random.default_rng(5)
    shape, ndim, dx, params = (1, 5, 6), 2, 0.9, [1.1, 0.8]
    x = rng.uniform(-0.8, 0.8, size=shape)
    r = oracle.rhs(AC, [x], ndim, dx, order, params)[0]
    eps = 1e-5
    for (zi, yi, xi) in [(0, 0, 0), (0, 2, 3), (0, 4, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[zi, yi, xi] += eps
        xm[zi, yi, xi] -= eps
        Fp = oracle.reduce(AC, [xp], ndim, dx, order, params)[1]
        Fm = oracle.reduce(AC, [xm], ndim, dx, order, params)[1]
        grad = (Fp - Fm) / (2 * eps) / dx ** ndim
        assert abs(grad + r[zi, yi, xi]) < 1e-7


@pytest.mark.parametrize("order", [2, 4, 6])
def test_cahn_hilliard_is_laplacian_of_chemical_potential(order):
    """CH rhs = L(dF/dc / dx^d) = L(-AC rhs): conserved dynamics of the same functional."""
    rng = np.random.default_rng(9)
    shape, ndim, dx, params = (4, 5, 6), 3, 1.0, [1.0, 1.0]
    c = rng.uniform(-0.5, 0.5, size=shape)
    ac = oracle.rhs(AC, [c], ndim, dx, order, params)[0]
    ch = oracle.rhs(CH, [c], ndim, dx, order, params)[0]
    expect = oracle.laplacian(-ac, ndim, dx, order)
    assert np.max(np.abs(ch - expect)) < 1e-13


def test_cahn_hilliard_energy_decreases():
    rng = np.random.default_rng(2)
    c = rng.uniform(-0.5, 0.5, size=(1, 32, 32))
    E = []
    for _ in range(6):
        E.append(oracle.reduce(CH, [c], 2, 1.0, 4, [1.0, 1.0])[1])
        c = oracle.run(CH, [c], 2, 1.0, 0.01, 4, [1.0, 1.0], 20)[0]
    assert all(b < a for a, b in zip(E, E[1:]))


# ------------------------------------------------------------- exact sums --

def test_exact_sum_matches_fsum():
    rng = np.random.default_rng(4)
    cases = [
        rng.uniform(-1, 1, 10000),
        np.array([1e100, 1.0, -1e100, 1e-100, 3.0]),
        np.array([1.0, 1e-16, 1e-16, -1.0]),
        np.concatenate([rng.uniform(-1, 1, 1000) * 10.0 ** rng.integers(-30, 30, 1000)]),
        np.array([0.1] * 10),
        np.array([2.0 ** 53, 1.0, 1e-300]),
        np.array([]),
    ]
    for x in cases:
        assert oracle.exact_sum(x) == math.fsum(x)


def test_reduce_counts_nonfinite():
    x = np.zeros((1, 4, 4))
    x[0, 1, 2] = np.nan
    x[0, 3, 3] = np.inf
    assert oracle.reduce(AC, [x], 2, 1.0, 2, [1.0, 1.0])[2] == 2


# ---------------------------------------------------------- stability pins --

@pytest.mark.parametrize("kind,params,order,ndim", [
    (AC, [0.0, 0.0], 2, 2), (AC, [0.0, 0.0], 4, 3),
    (CH, [0.0, 0.0], 2, 2), (CH, [0.0, 0.0], 6, 3),
])
def test_dt_max_separates_growth_from_decay(kind, params, order, ndim):
    """The Nyquist (checkerboard) mode grows just above dt_max and decays just below it."""
    shape = (1, 8, 8) if ndim == 2 else (4, 4, 4)
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    cb = ((-1.0) ** (x + y + (z if ndim == 3 else 0))) * 1e-3
    lim = oracle.dt_max(kind, ndim, 1.0, order, params)
    up = oracle.run(kind, [cb], ndim, 1.0, lim * 1.02, order, params, 200)[0]
    dn = oracle.run(kind, [cb], ndim, 1.0, lim * 0.98, order, params, 200)[0]
    assert np.max(np.abs(up)) > 1e-3 and np.max(np.abs(dn)) < 1e-3


def test_dt_max_config_values():
    """Reading of the explicit-stability limit at the workloads' settings."""
    assert math.isclose(oracle.dt_max(AC, 2, 1.0, 2, [1.0, 1.0]), 0.2, rel_tol=1e-12)
    assert oracle.dt_max(CH, 2, 1.0, 4, [1.0, 1.0]) > 0.01
    assert oracle.dt_max(CH, 3, 1.0, 6, [1.0, 1.0]) > 0.005
    # 3D Gray-Scott with the 7-point stencil: dt = 1 is beyond the limit
    assert oracle.dt_max(GS, 3, 1.0, 2, [0.2, 0.1, 0.04, 0.06]) < 1.0


# The c1 terms of the limit are pinned about the separated homogeneous states
# phi0^2 = c1/c2, where the linearised step is tightest: the checkerboard
# perturbation of the oracle's own step grows just above dt_max and decays
# just below it.  Model C (c3 = 0, rho = 0) and Model H (c3 = 0) reduce there
# to Allen-Cahn and Cahn-Hilliard plus diffusion; large dx makes Model H's
# diffusion branch (|lam*| > lam*^2 + 2 c1 |lam*|) the binding one.

def _nyquist_ratio(kind, base, f, ndim, dx, order, params, dt, steps=300, amp=1e-9):
    """Field f of the homogeneous state `base` perturbed by amp times the
    checkerboard; max deviation of field f after `steps` oracle steps, over amp."""
    shape = (1, 8, 8) if ndim == 2 else (4, 4, 4)
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    cb = (-1.0) ** (x + y + (z if ndim == 3 else 0))
    init = [np.full(shape, float(b)) + (amp * cb if g == f else 0.0) for g, b in enumerate(base)]
    out = oracle.run(kind, init, ndim, dx, dt, order, params, steps)
    return float(np.max(np.abs(out[f] - base[f]))) / amp


MH = 5


@pytest.mark.parametrize("kind,base,f,ndim,dx,order,params", [
    (AC, [math.sqrt(1.5 / 0.6)], 0, 2, 1.0, 2, [1.5, 0.6]),
    (AC, [math.sqrt(2.0 / 0.5)], 0, 3, 0.8, 4, [2.0, 0.5]),
    (CH, [2.0], 0, 2, 1.0, 4, [2.0, 0.5]),
    (CH, [math.sqrt(3.0)], 0, 3, 1.2, 2, [3.0, 1.0]),
    (MC, [2.0, 0.0], 0, 2, 1.0, 4, [1.2, 0.3, 0.0]),
    (MH, [1.0, 0.0, 0.0], 0, 2, 1.0, 4, [1.5, 1.5, 0.0]),
    (MH, [0.0, 0.0, 0.0], 1, 2, 4.0, 4, [0.05, 1.0, 0.0]),
    (MH, [0.0, 0.0, 0.0, 0.0], 3, 3, 4.0, 2, [0.01, 1.0, 0.0]),
])
def test_dt_max_c1_terms_separate_growth_from_decay(kind, base, f, ndim, dx, order, params):
    lim = oracle.dt_max(kind, ndim, dx, order, params)
    assert _nyquist_ratio(kind, base, f, ndim, dx, order, params, 1.02 * lim) > 10.0
    assert _nyquist_ratio(kind, base, f, ndim, dx, order, params, 0.98 * lim) < 0.1


@pytest.mark.parametrize("ndim,order,dx,Du,Dv", [
    (2, 2, 1.0, 0.2, 0.1), (3, 2, 1.0, 0.2, 0.1), (3, 2, 1.0, 0.4, 0.1),
    (2, 4, 0.7, 0.1, 0.3), (3, 2, 1.3, 0.05, 0.4),
])
def test_gs_dt_max_bounds_the_nyquist_spectrum(ndim, order, dx, Du, Dv):
    """Gray-Scott: the Jacobian of the oracle's right-hand side at the
    checkerboard mode (central differences about homogeneous states), over u,
    v in [0, 1]: dt_max keeps dt |eig| <= 2 everywhere, and its rate 2/dt_max
    exceeds the largest |eig| by at most the reaction slack 1 + F + k."""
    F, k = 0.04, 0.06
    params = [Du, Dv, F, k]
    lim = oracle.dt_max(GS, ndim, dx, order, params)
    shape = (1, 8, 8) if ndim == 2 else (4, 4, 4)
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    cb = (-1.0) ** (x + y + (z if ndim == 3 else 0))
    eps = 1e-6
    worst = 0.0
    for u0 in np.linspace(0.0, 1.0, 11):
        for v0 in np.linspace(0.0, 1.0, 11):
            J = np.zeros((2, 2))
            for f in range(2):
                d = [eps * cb if g == f else 0.0 for g in range(2)]
                rp = oracle.rhs(GS, [np.full(shape, u0) + d[0], np.full(shape, v0) + d[1]], ndim, dx,
                                order, params)
                rm = oracle.rhs(GS, [np.full(shape, u0) - d[0], np.full(shape, v0) - d[1]], ndim, dx,
                                order, params)
                for g in range(2):
                    J[g, f] = np.mean((rp[g] - rm[g]) * cb) / (2 * eps)
            worst = max(worst, float(np.max(np.abs(np.linalg.eigvals(J)))))
    assert lim * worst <= 2.0 * (1 + 1e-9)
    assert 2.0 / lim <= worst + 1.0 + F + k + 1e-9


def test_gray_scott_3d_dt1_is_unstable():
    """The Nyquist u-mode amplification at dt = 1 is 1 - dt (12 Du + F) = -1.44."""
    shape = (8, 8, 8)
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    cb = (-1.0) ** (x + y + z)
    u0, v0 = 1.0 + 1e-6 * cb, np.zeros(shape)
    u, v = oracle.run(GS, [u0, v0], 3, 1.0, 1.0, 2, [0.2, 0.1, 0.04, 0.06], 10)
    amp = np.max(np.abs(u - 1.0)) / 1e-6
    assert math.isclose(amp, 1.44 ** 10, rel_tol=1e-6)


# ------------------------------------------------------- Model C pins --
# Eq. model-c: phi_t = L phi + c1 phi - c2 phi^3 - 2 phi rho,
#              rho_t = L (rho + c3 phi^2).

@pytest.mark.parametrize("shape,ndim,order", [((1, 4, 4), 2, 2), ((1, 4, 4), 2, 4), ((3, 3, 3), 3, 2),
                                              ((1, 1, 10), 1, 6)])
def test_model_c_exact_rational_brute_force(shape, ndim, order):
    rng = np.random.default_rng(13)
    fields = [rng.uniform(-0.5, 0.5, size=shape) for _ in range(2)]
    params, dt, nsteps = [1.1, 0.9, 0.5], 0.01, 4
    got = oracle.run(MC, fields, ndim, 1.0, dt, order, params, nsteps)
    ex = run_exact(MC, fields, ndim, 1.0, dt, order, params, nsteps)
    for g, e in zip(got, ex):
        e = np.array([[[float(v) for v in row] for row in pl] for pl in e])
        assert np.max(np.abs(g - e)) < 5e-15
    # rho is conserved exactly by the scheme (a sum of Laplacians vanishes)
    r0 = sum(Fraction(float(v)) for v in fields[1].ravel())
    r4 = sum(v for pl in ex[1] for row in pl for v in row)
    assert r4 == r0


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("shape,ndim", [((1, 24, 30), 2), ((8, 9, 10), 3)])
def test_model_c_rho_mass_conservation(order, shape, ndim):
    rng = np.random.default_rng(17)
    phi, rho = rng.uniform(-0.1, 0.1, shape), rng.uniform(-0.1, 0.1, shape)
    n = 20
    out = oracle.run(MC, [phi, rho], ndim, 1.0, 0.01, order, [1.0, 1.0, 0.5], n)
    drift = abs(oracle.exact_sum(out[1]) - oracle.exact_sum(rho))
    assert drift <= n * rho.size * 2.3e-16 * 0.2


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_model_c_fixed_point_bitwise(order):
    """phi = 0 with any constant rho is a fixed point, exactly."""
    shape = (4, 5, 6)
    phi, rho = np.zeros(shape), np.full(shape, 0.37)
    out = oracle.run(MC, [phi, rho], 3, 1.0, 0.01, order, [1.0, 1.0, 0.5], 10)
    assert np.array_equal(out[0], phi) and np.array_equal(out[1], rho)


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("shape,ndim,modes", [((1, 16, 20), 2, (0, 3, 2)), ((6, 8, 10), 3, (1, 2, 3))])
def test_model_c_linear_modes(order, shape, ndim, modes):
    """c2 = c3 = 0 and rho = rho0: phi = A mode grows by 1 + dt (lam + c1 - 2 rho0),
    rho stays rho0 (the coupling sign and factor 2 are pinned).  c3 = 0 and
    rho = rho0 + B mode: rho diffuses by 1 + dt lam whatever phi is."""
    dx, n, dt = 1.0, 25, 0.01
    m, th = _mode(shape, ndim, modes)
    lam = _eig(order, th, dx)
    A0, c1, rho0 = 0.01, 0.7, 0.3
    phi, rho = oracle.run(MC, [A0 * m, np.full(shape, rho0)], ndim, dx, dt, order, [c1, 0.0, 0.0], n)
    g = 1 + dt * (lam + c1 - 2 * rho0)
    assert np.max(np.abs(phi - A0 * g ** n * m)) <= 1e-15 * n * 4
    assert np.all(rho == rho0)
    rng = np.random.default_rng(19)
    phi0 = rng.uniform(-0.2, 0.2, shape)
    _, rho = oracle.run(MC, [phi0, rho0 + A0 * m], ndim, dx, dt, order, [1.0, 1.0, 0.0], n)
    assert np.max(np.abs(rho - (rho0 + A0 * (1 + dt * lam) ** n * m))) <= 1e-15 * n * 4


@pytest.mark.parametrize("order", [2, 4])
def test_model_c_coupling_one_step(order):
    """phi = A cos(theta.x), rho = 0, c1 = c2 = 0: after one step
    rho = dt c3 L(phi^2) = dt c3 (A^2 / 2) lam(2 theta) cos(2 theta.x) and
    phi = (1 + dt lam(theta)) phi (pins c3, the square and the outer L)."""
    shape, ndim, dx, dt, c3, A = (1, 16, 24), 2, 1.0, 0.01, 0.5, 0.2
    m, th = _mode(shape, ndim, (0, 3, 2))
    m2, th2 = _mode(shape, ndim, (0, 6, 4))
    phi, rho = oracle.run(MC, [A * m, np.zeros(shape)], ndim, dx, dt, order, [0.0, 0.0, c3], 1)
    assert np.max(np.abs(phi - (1 + dt * _eig(order, th, dx)) * A * m)) <= 1e-16
    assert np.max(np.abs(rho - dt * c3 * A * A / 2 * _eig(order, th2, dx) * m2)) <= 1e-17


def test_model_c_reduces_to_model_a():
    """c3 = 0 and rho = 0: rho stays 0 and phi follows Eq. model-a bitwise."""
    rng = np.random.default_rng(23)
    shape = (1, 20, 22)
    phi0 = rng.uniform(-0.1, 0.1, shape)
    phi, rho = oracle.run(MC, [phi0, np.zeros(shape)], 2, 1.0, 0.05, 4, [1.0, 1.0, 0.0], 30)
    ref = oracle.run(AC, [phi0], 2, 1.0, 0.05, 4, [1.0, 1.0], 30)[0]
    assert np.array_equal(phi, ref) and np.all(rho == 0.0)


def test_model_c_dt_max_separates_growth_from_decay():
    shape = (1, 8, 8)
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    cb = ((-1.0) ** (x + y)) * 1e-3
    lim = oracle.dt_max(MC, 2, 1.0, 4, [0.0, 0.0, 0.5])
    for f in range(2):
        init = [cb if g == f else np.zeros(shape) for g in range(2)]
        up = oracle.run(MC, init, 2, 1.0, lim * 1.02, 4, [0.0, 0.0, 0.5], 200)[f]
        dn = oracle.run(MC, init, 2, 1.0, lim * 0.98, 4, [0.0, 0.0, 0.5], 200)[f]
        assert np.max(np.abs(up)) > 1e-3 and np.max(np.abs(dn)) < 1e-3


# ------------------------------------------------- direct biharmonic pins --
# Cahn-Hilliard with the biharmonic's own stencil: fourth-derivative weights
# along each axis plus twice the mixed products of second-derivative stencils
# (Secs. "Advanced Derivative Support", "Compile-Time Stencil Generation").

@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_d4_weights_polynomial_exactness_off_grid(order):
    """Applied around an off-grid point x0, the stencil returns the exact
    fourth derivative of every polynomial of degree <= order + 3, and not of
    degree order + 4."""
    w4 = fourth_derivative_weights_exact(order)
    r4 = order // 2 + 1
    x0 = Fraction(3, 7)
    for deg in range(0, order + 5):
        f = lambda x: (x - x0 + Fraction(1, 3)) ** deg
        d4 = (Fraction(math.factorial(deg), math.factorial(deg - 4)) * Fraction(1, 3) ** (deg - 4)
              if deg >= 4 else Fraction(0))
        val = sum(w4[abs(j)] * f(x0 + j) for j in range(-r4, r4 + 1))
        if deg <= order + 3:
            assert val == d4, (order, deg)
        else:
            assert val != d4, (order, deg)


def test_d4_weights_golden_table():
    with open(os.path.join(GOLDEN, "centered_d4_weights.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for line in rows:
        p, vals = line.split(":")
        assert fourth_derivative_weights_exact(int(p)) == [Fraction(v) for v in vals.split()]


def _d2_sym(order, th):
    """Symbol of the second-derivative stencil, closed form in s = sin^2(th/2)."""
    s = math.sin(th / 2) ** 2
    return {2: -4 * s, 4: -4 * s * (1 + s / 3)}[order]


def _d4_sym(order, th):
    """Symbol of the fourth-derivative stencil, closed form in s = sin^2(th/2)."""
    s = math.sin(th / 2) ** 2
    return {2: 16 * s * s, 4: 16 * s * s * (1 + 2 * s / 3)}[order]


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("shape,ndim,modes", [
    ((1, 1, 24), 1, (0, 0, 5)),
    ((1, 18, 24), 2, (0, 2, 5)),
    ((1, 18, 24), 2, (0, 7, 3)),
    ((8, 10, 12), 3, (3, 1, 4)),
    ((8, 10, 12), 3, (1, 4, 2)),
])
def test_biharmonic_direct_fourier_symbol(order, shape, ndim, modes):
    """B of a separable Fourier mode is its symbol: sum_a D4(th_a)/dx^4 +
    2 sum_{a<b} D2(th_a) D2(th_b)/dx^4 (closed forms derived by hand)."""
    nz, ny, nx = shape
    dx = 0.7
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ths = [2 * math.pi * modes[2] / nx, 2 * math.pi * modes[1] / ny, 2 * math.pi * modes[0] / nz][:ndim]
    u = np.cos(ths[0] * x + 0.3)
    if ndim >= 2:
        u = u * np.sin(ths[1] * y + 0.1)
    if ndim == 3:
        u = u * np.cos(ths[2] * z)
    sym = sum(_d4_sym(order, t) for t in ths)
    sym += 2 * sum(_d2_sym(order, ths[a]) * _d2_sym(order, ths[b])
                   for a in range(ndim) for b in range(a + 1, ndim))
    sym /= dx ** 4
    bu = oracle.biharmonic_direct(u, ndim, dx, order)
    assert np.max(np.abs(bu - sym * u)) <= 1e-12 * (1 + abs(sym)) * 64 / dx ** 4
    # the same mode through the Cahn-Hilliard right-hand side (linear: c1 = c2 = 0)
    r = oracle.rhs(CH, [u], ndim, dx, order, [0.0, 0.0], biharmonic="direct")[0]
    assert np.max(np.abs(r + sym * u)) <= 1e-12 * (1 + abs(sym)) * 64 / dx ** 4


@pytest.mark.parametrize("shape,ndim", [((1, 1, 9), 1), ((1, 5, 6), 2), ((3, 4, 5), 3)])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_biharmonic_direct_exact_rational_brute_force(shape, ndim, order):
    """The FP64 oracle agrees with the exact-rational run to rounding error,
    and mass is conserved exactly by the exact run."""
    f = [np.random.default_rng(7).uniform(-0.3, 0.3, size=shape)]
    dx, dt, params = 0.9, 0.004, [0.8, 1.3]
    ex = run_exact(CH, f, ndim, dx, dt, order, params, 2, biharmonic="direct")
    got = oracle.run(CH, f, ndim, dx, dt, order, params, 2, biharmonic="direct")[0]
    exf = np.array([[[float(v) for v in row] for row in pl] for pl in ex[0]])
    assert np.max(np.abs(got - exf)) <= 1e-14
    m0 = sum(Fraction(float(v)) for v in f[0].ravel())
    assert sum(v for pl in ex[0] for row in pl for v in row) == m0


@pytest.mark.parametrize("shape,ndim", [((1, 4, 5), 2), ((3, 3, 4), 3)])
def test_biharmonic_direct_order2_is_composed(shape, ndim):
    """At accuracy 2 the fourth-derivative stencil is the square of the
    second-derivative one, so the direct and composed schemes are the same
    scheme: exactly equal in rational arithmetic."""
    f = [np.random.default_rng(8).uniform(-0.3, 0.3, size=shape)]
    a = run_exact(CH, f, ndim, 1.1, 0.003, 2, [1.0, 1.0], 2, biharmonic="direct")
    b = run_exact(CH, f, ndim, 1.1, 0.003, 2, [1.0, 1.0], 2)
    assert a == b
    c = run_exact(CH, f, ndim, 1.1, 0.003, 4, [1.0, 1.0], 1, biharmonic="direct")
    d = run_exact(CH, f, ndim, 1.1, 0.003, 4, [1.0, 1.0], 1)
    assert c != d


@pytest.mark.parametrize("order,ndim", [(2, 1), (4, 2), (6, 3), (4, 3)])
def test_biharmonic_direct_dt_max_is_nyquist_flip(order, ndim):
    """At dt_max the linear (c1 = c2 = 0) direct scheme maps the checkerboard
    to minus itself: 1 - dt_max * beta* = -1."""
    shape = {1: (1, 1, 8), 2: (1, 8, 8), 3: (4, 4, 4)}[ndim]
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    cb = (-1.0) ** (x + (y if ndim >= 2 else 0) + (z if ndim == 3 else 0))
    lim = oracle.dt_max(CH, ndim, 1.3, order, [0.0, 0.0], biharmonic="direct")
    out = oracle.run(CH, [cb], ndim, 1.3, lim, order, [0.0, 0.0], 1, biharmonic="direct")[0]
    assert np.max(np.abs(out + cb)) <= 1e-12


def test_biharmonic_direct_dimension_reduction():
    """A 2D grid with ny = 1 gives the 1D result: the mixed term vanishes."""
    u = np.random.default_rng(9).uniform(-1, 1, size=(1, 1, 29))
    for order in (2, 4, 6):
        a = oracle.biharmonic_direct(u, 1, 0.8, order)
        b = oracle.biharmonic_direct(u, 2, 0.8, order)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("order,composed,direct", [
    (2, Fraction(-1, 6), Fraction(-1, 6)),
    (4, Fraction(-1, 45), Fraction(-7, 240)),
])
def test_biharmonic_forms_leading_truncation_error(order, composed, direct):
    """Accuracy of the two forms along one axis: applied to exp(i theta j),
    each stencil gives theta^4 + C theta^(4 + order) + ...; C follows from
    the even moments of the weights (Taylor series of cos).  The composed form
    D2 D2 has C = 2 C2 with C2 the second-derivative constant; the direct
    fourth-derivative stencil has its own C (Fornberg's table: -1/6 at
    accuracy 2, -7/240 at accuracy 4), so at accuracy 4 the composed form is
    the more accurate one, with a wider stencil (radius 4 against 3)."""
    def coeff(w, k):  # theta^k coefficient of w_0 + 2 sum_j w_j cos(j theta), k even
        return sum(2 * wj * Fraction((-1) ** (k // 2) * j ** k, math.factorial(k))
                   for j, wj in enumerate(w) if j > 0)
    w2 = second_derivative_weights_exact(order)
    w4 = fourth_derivative_weights_exact(order)
    k = 4 + order
    c2 = coeff(w2, 2 + order)           # D2 = -theta^2 + c2 theta^(2+order) + ...
    assert coeff(w2, 2) == -1 and coeff(w4, 4) == 1
    assert 2 * (-1) * c2 == composed    # (D2)^2 = theta^4 - 2 c2 theta^(4+order) + ...
    assert coeff(w4, k) == direct


# ------------------------------------------------------------ Model H pins --
# Eq. model-h with the transverse projector one:
#   m_t = L mu - c3 div(m j),  mu = c2 m^3 - c1 m - L m;   j_t = L j + c3 m grad(mu).

MH = oracle.MH


def test_d1_weights_golden_table():
    with open(os.path.join(GOLDEN, "centered_d1_weights.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 4
    for line in rows:
        p, vals = line.split(":")
        w = first_derivative_weights_exact(int(p))
        assert w[0] == 0 and w[1:] == [Fraction(v) for v in vals.split()]


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_d1_weights_polynomial_exactness_off_grid(order):
    w1 = first_derivative_weights_exact(order)
    r = order // 2
    x0, s = Fraction(2, 9), Fraction(1, 4)
    for deg in range(0, order + 2):
        f = lambda x: (x - x0 + s) ** deg
        d1 = deg * s ** (deg - 1) if deg >= 1 else Fraction(0)
        val = sum(w1[j] * (f(x0 + j) - f(x0 - j)) for j in range(1, r + 1))
        if deg <= order:
            assert val == d1, (order, deg)
        else:
            assert val != d1, (order, deg)


@pytest.mark.parametrize("shape,ndim,order", [((1, 1, 9), 1, 4), ((1, 4, 5), 2, 2), ((1, 4, 4), 2, 6),
                                              ((3, 3, 4), 3, 2)])
def test_model_h_exact_rational_brute_force(shape, ndim, order):
    rng = np.random.default_rng(17)
    fields = [rng.uniform(-0.4, 0.4, size=shape) for _ in range(1 + ndim)]
    params, dt, nsteps = [0.9, 1.1, 0.5], 0.003, 3
    got = oracle.run(MH, fields, ndim, 0.8, dt, order, params, nsteps)
    ex = run_exact(MH, fields, ndim, 0.8, dt, order, params, nsteps)
    assert len(got) == 1 + ndim
    for g, e in zip(got, ex):
        e = np.array([[[float(v) for v in row] for row in pl] for pl in e])
        assert np.max(np.abs(g - e)) < 5e-15
    # m is conserved exactly: a Laplacian and a centred divergence sum to zero
    m0 = sum(Fraction(float(v)) for v in fields[0].ravel())
    assert sum(v for pl in ex[0] for row in pl for v in row) == m0


@pytest.mark.parametrize("order", [2, 4])
def test_model_h_without_coupling_is_cahn_hilliard_and_diffusion(order):
    """c3 = 0: m evolves exactly as Cahn-Hilliard (bitwise) and every j_a as
    the heat equation, whose single modes decay by (1 + dt lam)^n."""
    shape, ndim, dx, dt, n = (1, 16, 20), 2, 1.0, 0.002, 20
    rng = np.random.default_rng(18)
    m = rng.uniform(-0.05, 0.05, size=shape)
    jx, th = _mode(shape, ndim, (0, 3, 2))
    jy, _ = _mode(shape, ndim, (0, 3, 2))
    out = oracle.run(MH, [m, 0.1 * jx, -0.2 * jy], ndim, dx, dt, order, [1.0, 1.0, 0.0], n)
    ch = oracle.run(CH, [m], ndim, dx, dt, order, [1.0, 1.0], n)[0]
    assert np.array_equal(out[0], ch)
    g = (1 + dt * _eig(order, th, dx)) ** n
    assert np.max(np.abs(out[1] - 0.1 * g * jx)) <= 1e-15 * n * 8
    assert np.max(np.abs(out[2] + 0.2 * g * jy)) <= 1e-15 * n * 8


def test_model_h_coupling_one_step_closed_form():
    """1D, order 2, c1 = c2 = 0, m = m0 + e cos(th x), j = j0: with
    S = sin(th)/dx and lam = -4 sin^2(th/2)/dx^2 one step gives
      m' = m0 + e cos(th x) (1 - dt lam^2) + dt c3 j0 e S sin(th x)
      j' = j0 + dt c3 (m0 + e cos(th x)) lam e S sin(th x)
    (advection of m by j, and the push of j along grad mu)."""
    n, dx, dt, c3, m0, j0, e = 24, 0.7, 0.01, 0.5, 0.3, 0.8, 0.05
    x = np.arange(n)
    th = 2 * math.pi * 3 / n
    m = m0 + e * np.cos(th * x)
    j = np.full(n, j0)
    out = oracle.run(MH, [m[None, None, :], j[None, None, :]], 1, dx, dt, 2, [0.0, 0.0, c3], 1)
    S = math.sin(th) / dx
    lam = -4 * math.sin(th / 2) ** 2 / dx ** 2
    m1 = m0 + e * np.cos(th * x) * (1 - dt * lam * lam) + dt * c3 * j0 * e * S * np.sin(th * x)
    j1 = j0 + dt * c3 * (m0 + e * np.cos(th * x)) * lam * e * S * np.sin(th * x)
    assert np.max(np.abs(out[0][0, 0] - m1)) <= 1e-15
    assert np.max(np.abs(out[1][0, 0] - j1)) <= 1e-15


def test_model_h_dt_max_separates_growth_from_decay():
    """Linearised about small fields, m is Cahn-Hilliard and j diffuses: the
    checkerboard of m grows just above dt_max and decays just below it."""
    shape, ndim = (1, 8, 8), 2
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    cb = ((-1.0) ** (x + y)) * 1e-3
    zero = np.zeros(shape)
    params = [0.0, 0.0, 0.5]
    lim = oracle.dt_max(MH, ndim, 1.0, 4, params)
    assert lim == oracle.dt_max(CH, ndim, 1.0, 4, params[:2])
    up = oracle.run(MH, [cb, zero, zero], ndim, 1.0, lim * 1.02, 4, params, 200)[0]
    dn = oracle.run(MH, [cb, zero, zero], ndim, 1.0, lim * 0.98, 4, params, 200)[0]
    assert np.max(np.abs(up)) > 1e-3 and np.max(np.abs(dn)) < 1e-3
