"""CPU FP64 oracle for the explicit finite-difference phase-field step.

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct implementation of
what the GPU library computes (SymPhas 2.0, arXiv 2511.10508: Models A, B, C
and H, Eqs. model-a, model-b, model-c and model-h; Gray-Scott as named in the
Introduction), used by
the tests, by the smoke check and by the CPU-baseline leg of the benchmark.
The product library never imports or links it, and it imports nothing from
the product.

Layout: fields are numpy float64 arrays of shape (nz, ny, nx) (x fastest in
memory), one array per field.  A 2D grid is (1, ny, nx).

Pieces
  oracle/oracle.c   plain C loops (Laplacian, right-hand sides, forward Euler,
                    exact sums, energy density), built with gcc -O2
                    -ffp-contract=off into oracle/liboracle.so
  oracle/weights.py exact-rational stencil weights (polynomial interpolation)
  oracle/exact.py   Fraction-arithmetic brute force for tiny grids
  oracle/spectral.py the semi-implicit Fourier spectral step (numpy FFT)
"""
import ctypes
import os
import subprocess

import numpy as np

from .weights import (first_derivative_weights, first_derivative_weights_exact,
                      fourth_derivative_weights, fourth_derivative_weights_exact,
                      second_derivative_weights, second_derivative_weights_exact)

AC, CH, GS, MC, MH = 1, 2, 3, 4, 5
NFIELDS = {AC: 1, CH: 1, GS: 2, MC: 2}  # Model H: 1 + ndim (nfields())


def nfields(kind, ndim):
    return 1 + ndim if kind == MH else NFIELDS[kind]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A planted-mistake copy of the oracle (tests/test_oracle_mutants.py) is
# loaded in place of the real one through this variable.
_MUTANT = os.environ.get("PF_ORACLE_MUTANT_LIB")
_lib = None

# The spectral scheme (numpy); a planted-mistake copy replaces it through
# PF_ORACLE_SPECTRAL_MUTANT in the same way.
if os.environ.get("PF_ORACLE_SPECTRAL_MUTANT"):
    import importlib.util
    import sys
    _spec = importlib.util.spec_from_file_location("oracle.spectral",
                                                   os.environ["PF_ORACLE_SPECTRAL_MUTANT"])
    spectral = importlib.util.module_from_spec(_spec)
    _spec.loader.exec_module(spectral)
    sys.modules["oracle.spectral"] = spectral
else:
    from . import spectral  # noqa: E402

# The explicit-stability limit; a planted-mistake copy replaces it through
# PF_ORACLE_STABILITY_MUTANT in the same way.
if os.environ.get("PF_ORACLE_STABILITY_MUTANT"):
    import importlib.util
    import sys
    _spec = importlib.util.spec_from_file_location("oracle.stability",
                                                   os.environ["PF_ORACLE_STABILITY_MUTANT"])
    stability = importlib.util.module_from_spec(_spec)
    _spec.loader.exec_module(stability)
    sys.modules["oracle.stability"] = stability
else:
    from . import stability  # noqa: E402
dt_max = stability.dt_max


def build(force=False):
    """Compile oracle.c with gcc (FP64, no contraction, optional OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _MUTANT:
        lib = ctypes.CDLL(_MUTANT)
    else:
        build()
        lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    d, i32, i64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64
    pd, pi64 = P(d), P(i64)
    lib.orc_laplacian.argtypes = [i32, pi64, d, i32, pd, pd, pd]
    lib.orc_laplacian.restype = None
    lib.orc_rhs.argtypes = [i32, i32, pi64, d, i32, pd, pd, pd, pd]
    lib.orc_rhs.restype = None
    lib.orc_run.argtypes = [i32, i32, pi64, d, d, i32, pd, pd, pd, i64]
    lib.orc_run.restype = i32
    lib.orc_biharmonic_direct.argtypes = [i32, pi64, d, i32, pd, i32, pd, pd, pd]
    lib.orc_biharmonic_direct.restype = None
    lib.orc_rhs_chd.argtypes = [i32, pi64, d, i32, pd, i32, pd, pd, pd, pd]
    lib.orc_rhs_chd.restype = None
    lib.orc_run_chd.argtypes = [i32, pi64, d, d, i32, pd, i32, pd, pd, pd, i64]
    lib.orc_run_chd.restype = None
    lib.orc_rhs_mh.argtypes = [i32, pi64, d, i32, pd, pd, pd, pd, pd]
    lib.orc_rhs_mh.restype = None
    lib.orc_run_mh.argtypes = [i32, pi64, d, d, i32, pd, pd, pd, pd, i64]
    lib.orc_run_mh.restype = None
    lib.orc_exact_sum.argtypes = [pd, i64, i64]
    lib.orc_exact_sum.restype = d
    lib.orc_energy_density.argtypes = [i32, pi64, d, i32, pd, pd, pd, pd]
    lib.orc_energy_density.restype = None
    lib.orc_reduce.argtypes = [i32, i32, pi64, d, i32, pd, pd, pd, pd, pd]
    lib.orc_reduce.restype = i64
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(shape):
    """(nz, ny, nx) -> int64[3] {nx, ny, nz} and ndim (trailing extents of 1 dropped)."""
    nz, ny, nx = shape
    n = (ctypes.c_int64 * 3)(nx, ny, nz)
    return n


def _w(order):
    w = np.asarray(second_derivative_weights(order), dtype=np.float64)
    return w


def _w4(order):
    return np.asarray(fourth_derivative_weights(order), dtype=np.float64)


def _grid(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 2:
        a = a[None]
    if a.ndim != 3:
        raise ValueError("fields are (ny, nx) or (nz, ny, nx)")
    return a


def laplacian(u, ndim, dx, order):
    """Discrete star Laplacian of u (difference form), periodic."""
    lib = _load()
    u = _grid(u)
    out = np.empty_like(u)
    w = _w(order)
    lib.orc_laplacian(ndim, _dims(u.shape), dx, order // 2, _dptr(w), _dptr(u), _dptr(out))
    return out


def biharmonic_direct(u, ndim, dx, order):
    """Direct discrete biharmonic of u: fourth-derivative stencils along each
    axis plus twice the mixed second-derivative products, periodic."""
    lib = _load()
    u = _grid(u)
    out = np.empty_like(u)
    w, w4 = _w(order), _w4(order)
    lib.orc_biharmonic_direct(ndim, _dims(u.shape), dx, order // 2, _dptr(w), order // 2 + 1,
                              _dptr(w4), _dptr(u), _dptr(out))
    return out


def _stack(fields):
    fs = [_grid(f) for f in fields]
    shape = fs[0].shape
    if any(f.shape != shape for f in fs):
        raise ValueError("all fields must have the same shape")
    return np.ascontiguousarray(np.stack(fs)), shape


def _check_biharmonic(kind, biharmonic):
    if biharmonic not in ("composed", "direct"):
        raise ValueError("biharmonic is 'composed' or 'direct'")
    if biharmonic == "direct" and kind != CH:
        raise ValueError("the direct biharmonic applies to Cahn-Hilliard only")
    return biharmonic == "direct"


def rhs(kind, fields, ndim, dx, order, params, biharmonic="composed"):
    """Right-hand sides of Eq. model-a (AC), Eq. model-b (CH), Gray-Scott or
    Eq. model-c (MC: phi then rho).  biharmonic="direct": Cahn-Hilliard with
    the direct biharmonic stencil in place of the Laplacian applied twice."""
    lib = _load()
    direct = _check_biharmonic(kind, biharmonic)
    st, shape = _stack(fields)
    if st.shape[0] != nfields(kind, ndim):
        raise ValueError("wrong number of fields")
    out = np.empty_like(st)
    w = _w(order)
    p = np.asarray(list(params) + [0.0] * (4 - len(params)), dtype=np.float64)
    if kind == MH:
        w1 = np.asarray(first_derivative_weights(order), dtype=np.float64)
        lib.orc_rhs_mh(ndim, _dims(shape), dx, order // 2, _dptr(w), _dptr(w1), _dptr(p),
                       _dptr(st), _dptr(out))
        return [out[f] for f in range(st.shape[0])]
    if direct:
        w4 = _w4(order)
        lib.orc_rhs_chd(ndim, _dims(shape), dx, order // 2, _dptr(w), order // 2 + 1, _dptr(w4),
                        _dptr(p), _dptr(st), _dptr(out))
        return [out[0]]
    lib.orc_rhs(kind, ndim, _dims(shape), dx, order // 2, _dptr(w), _dptr(p), _dptr(st), _dptr(out))
    return [out[f] for f in range(st.shape[0])]


def run(kind, fields, ndim, dx, dt, order, params, nsteps, biharmonic="composed"):
    """nsteps forward-Euler steps from `fields` (list of arrays); returns new list.
    biharmonic as in rhs()."""
    lib = _load()
    direct = _check_biharmonic(kind, biharmonic)
    st, shape = _stack(fields)
    if st.shape[0] != nfields(kind, ndim):
        raise ValueError("wrong number of fields")
    w = _w(order)
    p = np.asarray(list(params) + [0.0] * (4 - len(params)), dtype=np.float64)
    if kind == MH:
        w1 = np.asarray(first_derivative_weights(order), dtype=np.float64)
        lib.orc_run_mh(ndim, _dims(shape), dx, dt, order // 2, _dptr(w), _dptr(w1), _dptr(p),
                       _dptr(st), int(nsteps))
        return [st[f].copy() for f in range(st.shape[0])]
    if direct:
        w4 = _w4(order)
        lib.orc_run_chd(ndim, _dims(shape), dx, dt, order // 2, _dptr(w), order // 2 + 1,
                        _dptr(w4), _dptr(p), _dptr(st), int(nsteps))
        return [st[0].copy()]
    rc = lib.orc_run(kind, ndim, _dims(shape), dx, dt, order // 2, _dptr(w), _dptr(p),
                     _dptr(st), int(nsteps))
    if rc != 0:
        raise ValueError("bad model kind")
    return [st[f].copy() for f in range(st.shape[0])]


def exact_sum(x):
    """Correctly rounded exact sum of a float64 array (finite values)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return lib.orc_exact_sum(_dptr(x), x.size, 1)


def energy_density(x, ndim, dx, order, params):
    """Per-site Landau free-energy density with the discrete gradient term."""
    lib = _load()
    x = _grid(x)
    e = np.empty_like(x)
    w = _w(order)
    p = np.asarray(list(params) + [0.0] * (4 - len(params)), dtype=np.float64)
    lib.orc_energy_density(ndim, _dims(x.shape), dx, order // 2, _dptr(w), _dptr(p), _dptr(x), _dptr(e))
    return e


def reduce(kind, fields, ndim, dx, order, params):
    """(mass list, energy or None, nonfinite count) of a state, summed exactly
    (Model H: the mass and non-finite count of m only)."""
    lib = _load()
    st, shape = _stack(fields)
    w = _w(order)
    p = np.asarray(list(params) + [0.0] * (4 - len(params)), dtype=np.float64)
    mass = np.zeros(2)
    energy = np.zeros(1)
    bad = lib.orc_reduce(kind, ndim, _dims(shape), dx, order // 2, _dptr(w), _dptr(p),
                         _dptr(st), _dptr(mass), _dptr(energy))
    if bad:
        return None, None, int(bad)
    m = [float(mass[f]) for f in range(1 if kind == MH else NFIELDS[kind])]
    return m, (float(energy[0]) if kind in (AC, CH) else None), 0


