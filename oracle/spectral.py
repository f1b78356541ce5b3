"""Semi-implicit Fourier spectral step, FP64 (numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): used by the tests, the
smoke check and the benchmark's CPU leg, never by the product library.

The paper builds spectral schemes by separating the linear terms of an
equation, solved in Fourier space, from the nonlinear terms, evolved in real
space (Sec. "Construction of Semi-Implicit Fourier Spectral Scheme", citing
the semi-implicit Fourier method of Chen and Shen, 1998).  For the two scalar
models on a periodic grid of n_a sites of spacing dx per axis, with the
continuous wavenumbers k_a = 2 pi m_a / (n_a dx) (m_a the signed discrete
frequency) and K2 = sum over axes of k_a^2, one step is

  Model A (Eq. model-a):  phi^ <- (phi^ + dt N^) / (1 + dt K2),      N = c1 phi - c2 phi^3
  Model B (Eq. model-b):  c^   <- (c^ - dt K2 g^) / (1 + dt K2^2),    g = c2 c^3 - c1 c

(^ the discrete Fourier transform): the Laplacian terms are taken at the new
time, the local polynomial at the old one.  numpy's FFT is the library
primitive for the transform; everything else is written out here.
"""
import numpy as np

AC, CH = 1, 2


def _axes(ndim):
    return tuple(range(3 - ndim, 3))


def k_squared(shape, ndim, dx):
    """K2 on the half-spectrum layout of a real transform over the last
    ndim axes of a (nz, ny, nx) grid (x halved)."""
    nz, ny, nx = shape
    kx = 2 * np.pi * np.fft.rfftfreq(nx, d=dx)
    K2 = np.zeros((nz if ndim == 3 else 1, ny if ndim >= 2 else 1, kx.size))
    K2 += kx[None, None, :] ** 2
    if ndim >= 2:
        ky = 2 * np.pi * np.fft.fftfreq(ny, d=dx)
        K2 += ky[None, :, None] ** 2
    if ndim == 3:
        kz = 2 * np.pi * np.fft.fftfreq(nz, d=dx)
        K2 += kz[:, None, None] ** 2
    return K2


def nonlinear(kind, u, params):
    """The explicit real-space term: N (Model A) or g (Model B)."""
    c1, c2 = params[0], params[1]
    if kind == AC:
        return c1 * u - c2 * (u * u * u)
    if kind == CH:
        return c2 * (u * u * u) - c1 * u
    raise ValueError("the spectral scheme covers Models A and B")


def step(kind, u, ndim, dx, dt, params, K2=None):
    """One semi-implicit step of the field u, shape (nz, ny, nx)."""
    u = np.asarray(u, dtype=np.float64)
    ax = _axes(ndim)
    if K2 is None:
        K2 = k_squared(u.shape, ndim, dx)
    uh = np.fft.rfftn(u, axes=ax)
    nh = np.fft.rfftn(nonlinear(kind, u, params), axes=ax)
    if kind == AC:
        uh = (uh + dt * nh) / (1.0 + dt * K2)
    else:
        uh = (uh - dt * K2 * nh) / (1.0 + dt * K2 * K2)
    return np.fft.irfftn(uh, s=[u.shape[a] for a in ax], axes=ax)


def dt_max(kind, params):
    """Stability limit of the scheme: only the local term is explicit.
    Linearised about the separated states u^2 = c1/c2, the explicit term has
    slope a = -2 c1 (Model A: N' = c1 - 3 c2 u^2) or a = 2 c1 (Model B:
    g' = 3 c2 u^2 - c1), so a mode is multiplied by
      Model A: (1 + dt a) / (1 + dt K2),      bounded by 1 for all K2 iff dt <= 1 / c1
      Model B: (1 - dt a K2) / (1 + dt K2^2), bounded by 1 for all K2 iff
               dt (a K2 - K2^2) <= 2 at K2 = a / 2, i.e. dt <= 8 / a^2 = 2 / c1^2.
    c1 = 0 leaves no limit (inf)."""
    c1 = abs(params[0])
    if c1 == 0.0:
        return float("inf")
    return 1.0 / c1 if kind == AC else 2.0 / (c1 * c1)


def run(kind, field, ndim, dx, dt, params, nsteps):
    """nsteps semi-implicit steps from `field` ((nz, ny, nx) or (ny, nx))."""
    u = np.asarray(field, dtype=np.float64)
    if u.ndim == 2:
        u = u[None]
    K2 = k_squared(u.shape, ndim, dx)
    for _ in range(nsteps):
        u = step(kind, u, ndim, dx, dt, params, K2)
    return u
