"""Oracle stencil weights, in exact rational arithmetic.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper derives finite-difference coefficients from polynomial
interpolation: for a derivative of order p (here the second derivative) and
accuracy n, a polynomial of degree q = p + n - 1 is fitted and the weights are
the solution of a linear system; centred stencils are reduced by symmetry
(Sec. "Compile-Time Stencil Generation").

For the centred second derivative with accuracy order p (even), the stencil
has radius r = p/2, points j = -r..r and symmetric weights w_{-j} = w_j.  The
stencil is exact on every polynomial of degree <= 2r, i.e. for the monomials
x^k applied at x = 0 with unit spacing:

    sum_{j=-r..r} w_j j^k = 2 if k == 2 else 0,      k = 0..2r.

Odd k hold automatically by symmetry, so the unknowns are w_0..w_r and the
equations are the even k = 0, 2, .., 2r: an (r+1) x (r+1) system that is
solved here by Gauss-Jordan elimination over Fractions.
"""
from fractions import Fraction


def second_derivative_weights_exact(order):
    """Exact centred second-derivative weights [w_0, w_1, .., w_r], r = order/2.

    Follows the polynomial-interpolation construction with symmetry reduction
    (Sec. "Compile-Time Stencil Generation").  `order` is the accuracy order
    p (even, >= 2).
    """
    if order < 2 or order % 2:
        raise ValueError("accuracy order must be an even integer >= 2")
    r = order // 2
    # Row for even moment k = 2m: w_0 * 0^k + sum_{j>=1} w_j * 2 * j^k.
    rows = []
    for m in range(r + 1):
        k = 2 * m
        row = [Fraction(1 if k == 0 else 0)]
        row += [Fraction(2 * j ** k) for j in range(1, r + 1)]
        rhs = Fraction(2 if k == 2 else 0)
        rows.append(row + [rhs])
    nvar = r + 1
    for col in range(nvar):
        piv = next(i for i in range(col, nvar) if rows[i][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        p = rows[col][col]
        rows[col] = [v / p for v in rows[col]]
        for i in range(nvar):
            if i != col and rows[i][col] != 0:
                f = rows[i][col]
                rows[i] = [a - f * b for a, b in zip(rows[i], rows[col])]
    return [rows[i][nvar] for i in range(nvar)]


def fourth_derivative_weights_exact(order):
    """Exact centred fourth-derivative weights [w_0, w_1, .., w_r4], r4 = order/2 + 1.

    The same construction for the derivative of order 4 (Sec. "Compile-Time
    Stencil Generation"): accuracy `order` (even, >= 2) needs a polynomial of
    degree 4 + order - 1, so the centred stencil has 2 r4 + 1 = order + 3
    points, and symmetry leaves the unknowns w_0..w_r4 with the even-moment
    equations

        sum_{j=-r4..r4} w_j j^k = 24 if k == 4 else 0,      k = 0, 2, .., 2 r4.
    """
    if order < 2 or order % 2:
        raise ValueError("accuracy order must be an even integer >= 2")
    r4 = order // 2 + 1
    rows = []
    for m in range(r4 + 1):
        k = 2 * m
        row = [Fraction(1 if k == 0 else 0)]
        row += [Fraction(2 * j ** k) for j in range(1, r4 + 1)]
        rows.append(row + [Fraction(24 if k == 4 else 0)])
    return _solve(rows)


def _solve(rows):
    """Gauss-Jordan elimination over Fractions of an augmented square system."""
    nvar = len(rows)
    rows = [list(r) for r in rows]
    for col in range(nvar):
        piv = next(i for i in range(col, nvar) if rows[i][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        p = rows[col][col]
        rows[col] = [v / p for v in rows[col]]
        for i in range(nvar):
            if i != col and rows[i][col] != 0:
                f = rows[i][col]
                rows[i] = [a - f * b for a, b in zip(rows[i], rows[col])]
    return [rows[i][nvar] for i in range(nvar)]


def first_derivative_weights_exact(order):
    """Exact centred first-derivative weights [0, w_1, .., w_r], r = order/2
    (antisymmetric: w_{-j} = -w_j, w_0 = 0).

    The same construction for the derivative of order 1: exact on the odd
    monomials up to degree 2r - 1, i.e. 2 sum_{j=1..r} w_j j^k = 1 if k == 1
    else 0 for k = 1, 3, .., 2r - 1 (even k hold by antisymmetry).
    """
    if order < 2 or order % 2:
        raise ValueError("accuracy order must be an even integer >= 2")
    r = order // 2
    rows = []
    for m in range(r):
        k = 2 * m + 1
        rows.append([Fraction(2 * j ** k) for j in range(1, r + 1)] + [Fraction(1 if k == 1 else 0)])
    return [Fraction(0)] + _solve(rows)


def first_derivative_weights(order):
    """FP64 first-derivative weights [0, w_1..w_r], each rounded once."""
    return [float(w) for w in first_derivative_weights_exact(order)]


def fourth_derivative_weights(order):
    """FP64 fourth-derivative weights [w_0..w_r4], each rounded to nearest once."""
    return [float(w) for w in fourth_derivative_weights_exact(order)]


def second_derivative_weights(order):
    """FP64 weights [w_0..w_r]: each exact rational rounded to nearest once."""
    return [float(w) for w in second_derivative_weights_exact(order)]
