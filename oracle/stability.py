"""Explicit-stability limit of the forward-Euler finite-difference step.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).  A reading of the paper:
it names no time integrator and gives no stability limit, so the limit is
taken from the linearised forward-Euler step at the stencil's Nyquist
(checkerboard) mode, the mode with the most negative Laplacian eigenvalue.
"""
from .weights import fourth_derivative_weights_exact, second_derivative_weights_exact

AC, CH, GS, MC, MH = 1, 2, 3, 4, 5


def dt_max(kind, ndim, dx, order, params, biharmonic="composed"):
    """Forward-Euler stability limit from the Nyquist-mode symbol.

    The most negative eigenvalue of the discrete Laplacian is lam* =
    ndim * sigma / dx^2 with sigma = w_0 + 2 sum_j w_j (-1)^j.  The
    linearised step is stable while dt * rho <= 2 where rho is
      AC: |lam*| + 2 c1        (linearisation about phi^2 <= c1/c2)
      CH: lam*^2 + 2 c1 |lam*|
          direct biharmonic: beta* + 2 c1 |lam*| with beta* = ndim tau / dx^4
          + ndim (ndim - 1) (sigma / dx^2)^2, tau = w4_0 + 2 sum_j w4_j (-1)^j
          (the direct operator's symbol at the Nyquist mode)
      GS: max(Du, Dv) |lam*| + F + k + 1     (u, v in [0, 1])
      MC: |lam*| + 2 c1        (as AC: linearisation about small phi, rho;
                                rho alone diffuses with |lam*|)
      MH: max(lam*^2 + 2 c1 |lam*|, |lam*|)  (m as CH, each j_a diffuses;
                                the couplings are products of small terms)
    """
    w = second_derivative_weights_exact(order)
    sigma = w[0] + 2 * sum(wj * (-1) ** j for j, wj in enumerate(w) if j > 0)
    lam = abs(float(sigma)) * ndim / (dx * dx)
    if biharmonic not in ("composed", "direct"):
        raise ValueError("biharmonic is 'composed' or 'direct'")
    direct = biharmonic == "direct"
    if direct and kind != CH:
        raise ValueError("the direct biharmonic applies to Cahn-Hilliard only")
    if kind == MH:
        # linearised about small m and j the couplings (products of small
        # quantities) drop out: m as Cahn-Hilliard, each j_a diffuses
        rho = max(lam * lam + 2 * abs(params[0]) * lam, lam)
    elif kind in (AC, MC):
        rho = lam + 2 * abs(params[0])
    elif kind == CH and direct:
        w4 = fourth_derivative_weights_exact(order)
        tau = w4[0] + 2 * sum(wj * (-1) ** j for j, wj in enumerate(w4) if j > 0)
        s1 = abs(float(sigma)) / (dx * dx)
        beta = ndim * abs(float(tau)) / dx ** 4 + ndim * (ndim - 1) * s1 * s1
        rho = beta + 2 * abs(params[0]) * lam
    elif kind == CH:
        rho = lam * lam + 2 * abs(params[0]) * lam
    else:
        rho = max(params[0], params[1]) * lam + params[2] + params[3] + 1.0
    return 2.0 / rho
