"""Exact-rational brute force of the same scheme on tiny grids.

TEST INFRASTRUCTURE ONLY.  Every FP64 input (field values, dx, dt, model
parameters) is taken as the exact binary value it represents and every
operation is done in Fraction arithmetic, so the result is the scheme's
exact value; the FP64 oracle must agree with it to rounding error.  Pure
Python loops: use grids of a few dozen sites and a handful of steps.
"""
from fractions import Fraction

from .weights import (first_derivative_weights_exact, fourth_derivative_weights_exact,
                      second_derivative_weights_exact)


def _lap(u, shape, ndim, dx, w):
    nz, ny, nx = shape
    inv = 1 / (dx * dx)
    out = {}
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                acc = Fraction(0)
                for a in range(ndim):
                    for j in range(1, len(w)):
                        d = [0, 0, 0]
                        d[a] = j
                        up = u[((z + d[2]) % nz, (y + d[1]) % ny, (x + d[0]) % nx)]
                        um = u[((z - d[2]) % nz, (y - d[1]) % ny, (x - d[0]) % nx)]
                        acc += w[j] * inv * (up + um - 2 * u[(z, y, x)])
                out[(z, y, x)] = acc
    return out


def _axis(u, shape, a, scale, w):
    """One axis of a centred even-derivative stencil, times `scale`."""
    nz, ny, nx = shape
    out = {}
    for (z, y, x), u0 in u.items():
        acc = Fraction(0)
        for j in range(1, len(w)):
            d = [0, 0, 0]
            d[a] = j
            up = u[((z + d[2]) % nz, (y + d[1]) % ny, (x + d[0]) % nx)]
            um = u[((z - d[2]) % nz, (y - d[1]) % ny, (x - d[0]) % nx)]
            acc += w[j] * scale * (up + um - 2 * u0)
        out[(z, y, x)] = acc
    return out


def _d1(u, shape, a, dx, w1):
    """Centred first derivative along axis a (antisymmetric weights w1)."""
    nz, ny, nx = shape
    out = {}
    for (z, y, x) in u:
        acc = Fraction(0)
        for k in range(1, len(w1)):
            d = [0, 0, 0]
            d[a] = k
            up = u[((z + d[2]) % nz, (y + d[1]) % ny, (x + d[0]) % nx)]
            um = u[((z - d[2]) % nz, (y - d[1]) % ny, (x - d[0]) % nx)]
            acc += w1[k] / dx * (up - um)
        out[(z, y, x)] = acc
    return out


def biharmonic_direct_exact(u, shape, ndim, dx, w, w4):
    """sum_a D4_a u + 2 sum_{a<b} D2_a D2_b u in Fractions (u: dict site -> value)."""
    out = {k: Fraction(0) for k in u}
    for a in range(ndim):
        t = _axis(u, shape, a, 1 / dx ** 4, w4)
        for k in out:
            out[k] += t[k]
    for a in range(ndim):
        for b in range(a + 1, ndim):
            t = _axis(_axis(u, shape, b, 1 / (dx * dx), w), shape, a, 1 / (dx * dx), w)
            for k in out:
                out[k] += 2 * t[k]
    return out


def run_exact(kind, fields, ndim, dx, dt, order, params, nsteps, biharmonic="composed"):
    """Exact forward-Euler run.  fields: list of nested lists/arrays (nz, ny, nx).
    biharmonic="direct": Cahn-Hilliard as L g - B c with the direct stencil."""
    w = second_derivative_weights_exact(order)
    w4 = fourth_derivative_weights_exact(order)
    w1 = first_derivative_weights_exact(order)
    shape = (len(fields[0]), len(fields[0][0]), len(fields[0][0][0]))
    nz, ny, nx = shape
    keys = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)]
    F = [{k: Fraction(float(f[k[0]][k[1]][k[2]])) for k in keys} for f in fields]
    dx, dt = Fraction(dx), Fraction(dt)
    P = [Fraction(p) for p in params]
    for _ in range(nsteps):
        if kind == 1:
            c1, c2 = P[0], P[1]
            L = _lap(F[0], shape, ndim, dx, w)
            F = [{k: F[0][k] + dt * (L[k] + c1 * F[0][k] - c2 * F[0][k] ** 3) for k in keys}]
        elif kind == 5:
            c1, c2, c3 = P[0], P[1], P[2]
            m = F[0]
            Lm = _lap(m, shape, ndim, dx, w)
            mu = {k: c2 * m[k] ** 3 - c1 * m[k] - Lm[k] for k in keys}
            dm = _lap(mu, shape, ndim, dx, w)
            newF = []
            for a in range(ndim):
                ja = F[1 + a]
                div = _d1({k: m[k] * ja[k] for k in keys}, shape, a, dx, w1)
                dm = {k: dm[k] - c3 * div[k] for k in keys}
            newF.append({k: m[k] + dt * dm[k] for k in keys})
            for a in range(ndim):
                ja = F[1 + a]
                Lj = _lap(ja, shape, ndim, dx, w)
                gmu = _d1(mu, shape, a, dx, w1)
                newF.append({k: ja[k] + dt * (Lj[k] + c3 * m[k] * gmu[k]) for k in keys})
            F = newF
        elif kind == 2 and biharmonic == "direct":
            c1, c2 = P[0], P[1]
            Lg = _lap({k: c2 * F[0][k] ** 3 - c1 * F[0][k] for k in keys}, shape, ndim, dx, w)
            B = biharmonic_direct_exact(F[0], shape, ndim, dx, w, w4)
            F = [{k: F[0][k] + dt * (Lg[k] - B[k]) for k in keys}]
        elif kind == 2:
            c1, c2 = P[0], P[1]
            L = _lap(F[0], shape, ndim, dx, w)
            mu = {k: c2 * F[0][k] ** 3 - c1 * F[0][k] - L[k] for k in keys}
            Lm = _lap(mu, shape, ndim, dx, w)
            F = [{k: F[0][k] + dt * Lm[k] for k in keys}]
        elif kind == 4:
            c1, c2, c3 = P[0], P[1], P[2]
            phi, rho = F
            Lp = _lap(phi, shape, ndim, dx, w)
            Lg = _lap({k: rho[k] + c3 * phi[k] ** 2 for k in keys}, shape, ndim, dx, w)
            F = [{k: phi[k] + dt * (Lp[k] + c1 * phi[k] - c2 * phi[k] ** 3 - 2 * phi[k] * rho[k])
                  for k in keys},
                 {k: rho[k] + dt * Lg[k] for k in keys}]
        else:
            Du, Dv, Fr, kr = P[0], P[1], P[2], P[3]
            u, v = F
            Lu = _lap(u, shape, ndim, dx, w)
            Lv = _lap(v, shape, ndim, dx, w)
            F = [{k: u[k] + dt * (Du * Lu[k] - u[k] * v[k] ** 2 + Fr * (1 - u[k])) for k in keys},
                 {k: v[k] + dt * (Dv * Lv[k] + u[k] * v[k] ** 2 - (Fr + kr) * v[k]) for k in keys}]
    return [[[[f[(z, y, x)] for x in range(nx)] for y in range(ny)] for z in range(nz)] for f in F]
