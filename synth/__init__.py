"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds none of the method's arithmetic: it only produces initial
fields and request traces.  Both the oracle tests and the GPU tests draw
their inputs from here, so the two implementations see identical data.

Counter-based generator
-----------------------
Every random value is a pure function of (seed, stream, index), so any window
of a field can be produced without producing the whole field.  The mixing
function is the SplitMix64 output finaliser (Steele, Lea and Flood,
"Fast Splittable Pseudorandom Number Generators", OOPSLA 2014), with the
golden-ratio increment G = 0x9E3779B97F4A7C15:

    mix(z)  = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB;  z ^ (z >> 31)
    key     = mix(seed + (stream + 1) * G)            (mod 2^64)
    h(i)    = mix(key + (i + 1) * G)                  (mod 2^64)
    u01(i)  = (h(i) >> 11) * 2^-53                    in [0, 1)
    x(i)    = a + (b - a) * u01(i)                    FP64, two roundings

i is the site's linear index x + nx*(y + ny*z).  FP32 storage rounds x(i) to
nearest.  Streams: 0 = first field, 1 = second field, 2 = Gray-Scott cube
corners.

Initial-condition recipes (one per workload)
  uniform(lo, hi)        Allen-Cahn phi0 ~ U[-0.1, 0.1]; Cahn-Hilliard
                         c0 = 0 + U[-0.05, 0.05]
  gray_scott_cubes       u = 1, v = 0 except ncubes cubes of side s with
                         u = 0.5, v = 0.25 at seeded corners (periodic wrap),
                         then U[-0.01, 0.01] added to u and v.
"""
import math

import numpy as np

G = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1

IC_UNIFORM = 1
IC_GS_CUBES = 2
IC_CONST = 3


def mix_int(z):
    """SplitMix64 finaliser on a Python int (mod 2^64)."""
    z &= MASK
    z ^= z >> 30
    z = (z * M1) & MASK
    z ^= z >> 27
    z = (z * M2) & MASK
    return z ^ (z >> 31)


def _mix_np(z):
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(M1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(M2)
    z ^= z >> np.uint64(31)
    return z


def stream_key(seed, stream):
    return mix_int((seed + (stream + 1) * G) & MASK)


def u01(seed, stream, idx):
    """Uniform [0,1) doubles for an int64 array of linear indices."""
    key = np.uint64(stream_key(seed, stream))
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + (idx + np.uint64(1)) * np.uint64(G)
        h = _mix_np(z)
    return (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_values(seed, stream, idx, lo, hi):
    """lo + (hi - lo) * u01 in FP64 (the product is rounded, then the sum)."""
    u = u01(seed, stream, idx)
    return np.float64(lo) + np.float64(hi - lo) * u


def window_indices(shape, origin=(0, 0, 0), wshape=None):
    """Linear indices (periodic) of a window of a (nz, ny, nx) grid.

    origin and wshape are (z0, y0, x0) and (wz, wy, wx); coordinates wrap.
    """
    nz, ny, nx = shape
    if wshape is None:
        wshape = shape
    z = (np.arange(wshape[0], dtype=np.int64) + origin[0]) % nz
    y = (np.arange(wshape[1], dtype=np.int64) + origin[1]) % ny
    x = (np.arange(wshape[2], dtype=np.int64) + origin[2]) % nx
    return (x[None, None, :] + nx * (y[None, :, None] + ny * z[:, None, None]))


def uniform_field(seed, stream, shape, lo, hi, origin=(0, 0, 0), wshape=None):
    idx = window_indices(shape, origin, wshape)
    return uniform_values(seed, stream, idx.ravel(), lo, hi).reshape(idx.shape)


def cube_corners(seed, shape, ncubes):
    """Corner (z, y, x) of each Gray-Scott cube: floor(u01 * n) per axis."""
    nz, ny, nx = shape
    out = []
    for c in range(ncubes):
        ks = np.array([3 * c, 3 * c + 1, 3 * c + 2], dtype=np.uint64)
        u = u01(seed, 2, ks)
        cx = min(int(math.floor(u[0] * nx)), nx - 1)
        cy = min(int(math.floor(u[1] * ny)), ny - 1)
        cz = min(int(math.floor(u[2] * nz)), nz - 1)
        out.append((cz, cy, cx))
    return out


def gray_scott_fields(seed, shape, ncubes=20, side=16, noise=0.01,
                      inside=(0.5, 0.25), outside=(1.0, 0.0),
                      origin=(0, 0, 0), wshape=None):
    """(u, v) for the Gray-Scott cube recipe, optionally on a periodic window."""
    nz, ny, nx = shape
    if wshape is None:
        wshape = shape
    z = (np.arange(wshape[0], dtype=np.int64) + origin[0]) % nz
    y = (np.arange(wshape[1], dtype=np.int64) + origin[1]) % ny
    x = (np.arange(wshape[2], dtype=np.int64) + origin[2]) % nx
    inside_mask = np.zeros(wshape, dtype=bool)
    sz, sy, sx = min(side, nz), min(side, ny), min(side, nx)
    for cz, cy, cx in cube_corners(seed, shape, ncubes):
        mz = ((z - cz) % nz) < sz
        my = ((y - cy) % ny) < sy
        mx = ((x - cx) % nx) < sx
        inside_mask |= mz[:, None, None] & my[None, :, None] & mx[None, None, :]
    idx = (x[None, None, :] + nx * (y[None, :, None] + ny * z[:, None, None])).ravel()
    base_u = np.where(inside_mask, inside[0], outside[0]).astype(np.float64)
    base_v = np.where(inside_mask, inside[1], outside[1]).astype(np.float64)
    nu = uniform_values(seed, 0, idx, -noise, noise).reshape(wshape)
    nv = uniform_values(seed, 1, idx, -noise, noise).reshape(wshape)
    return base_u + nu, base_v + nv


def initial_fields(kind, shape, seed, ic=None, ic_params=None, origin=(0, 0, 0), wshape=None,
                   ndim=None):
    """Initial state for a model kind (1 AC, 2 CH, 3 GS, 4 MC, 5 MH) as FP64
    arrays; Model H has 1 + ndim fields (ndim required)."""
    return _initial_fields(kind, shape, seed, ic, ic_params, origin, wshape, ndim)


def _initial_fields(kind, shape, seed, ic, ic_params, origin, wshape, ndim):
    """Initial state for a model kind as FP64 arrays.

    ic / ic_params follow the library's pf_init convention:
      IC_UNIFORM  params (lo, hi): field f from stream f
      IC_GS_CUBES params (ncubes, side, noise)
      IC_CONST    params (value per field)
    """
    if ic is None:
        ic = IC_GS_CUBES if kind == 3 else IC_UNIFORM
    if kind == 5 and ndim is None:
        raise ValueError("Model H needs ndim (1 + ndim fields)")
    nf = 1 + ndim if kind == 5 else 2 if kind in (3, 4) else 1
    if ic == IC_UNIFORM:
        lo, hi = (ic_params or (-0.05, 0.05))[:2]
        return [uniform_field(seed, f, shape, lo, hi, origin, wshape) for f in range(nf)]
    if ic == IC_GS_CUBES:
        p = list(ic_params or (20, 16, 0.01))
        return list(gray_scott_fields(seed, shape, int(p[0]), int(p[1]), float(p[2]),
                                      origin=origin, wshape=wshape))
    if ic == IC_CONST:
        vals = list(ic_params)
        ws = wshape or shape
        return [np.full(ws, float(vals[f])) for f in range(nf)]
    raise ValueError("unknown initial condition")


def serving_trace(nreq, seed=505, rate=None, dims=(2, 3), fp32=True):
    """The mixed serving workload: a list of request dicts.

    Model uniform over {AC, CH, GS}; dimension 2D/3D at 50/50; side
    log-uniform 64..2048 (2D) or 32..256 (3D); steps log-uniform 100..10000;
    order uniform over {2, 4}; parameters jittered by U[0.8, 1.2] around the
    base workloads (AC c1=c2=1 dt=0.05; CH c1=c2=1 dt=0.01; GS Du=0.2 Dv=0.1
    F=0.04 k=0.06 dt=0.5).  Arrival times are Poisson with the given rate
    (requests/s); rate None gives all arrivals at t = 0.  The requests
    themselves do not depend on the rate (every request draws its
    inter-arrival gap, used or not), so traces at different rates hold the
    same requests.  The time-step limit is not applied here: the caller
    redraws dt against its own limit.
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(nreq):
        kind = int(rng.integers(1, 4))
        ndim = int(dims[int(rng.integers(0, len(dims)))])
        if ndim == 2:
            side = int(round(math.exp(rng.uniform(math.log(64), math.log(2048)))))
            shape = (1, side, side)
        else:
            side = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
            shape = (side, side, side)
        steps = int(round(math.exp(rng.uniform(math.log(100), math.log(10000)))))
        order = int(rng.choice([2, 4]))
        jit = rng.uniform(0.8, 1.2, size=5)
        if kind == 1:
            params, dt = [1.0 * jit[0], 1.0 * jit[1]], 0.05 * jit[4]
        elif kind == 2:
            params, dt = [1.0 * jit[0], 1.0 * jit[1]], 0.01 * jit[4]
        else:
            params, dt = [0.2 * jit[0], 0.1 * jit[1], 0.04 * jit[2], 0.06 * jit[3]], 0.5 * jit[4]
        gap = float(rng.exponential(1.0))
        if rate:
            t += gap / rate
        out.append(dict(id=i, kind=kind, ndim=ndim, shape=shape, steps=steps, order=order,
                        params=params, dt=float(dt), seed=int(mix_int(seed * 1000003 + i) >> 1),
                        arrival=t, fp32=fp32,
                        cube_side=max(2, int(round(16 * side / 512)))))
    return out
