"""Seeded synthetic initial fields in *primitive* form (input data only).

Every recipe returns pressure, temperature, mass fractions and velocity on
the interior cells of a periodic box, arrays laid out [z][y][x] (x fastest),
species and velocity components first: Y[ns][nz][ny][nx], u[3][nz][ny][nx].
Conversion to the conserved state (density, momentum, total energy) is done
separately by each implementation from its own thermodynamics.

Recipes
  sines : sums of three seeded Fourier modes for T (300..1500 K) and for each
          velocity component (amplitude 10 m/s), a two-composition blend for Y.
          The small-box workloads (16^3, the batched boxes, the 64^3 adjoint).
  turb  : solenoidal random-phase velocity with a k^-5/3 shell spectrum and a
          set rms, a periodic two-front planar flame slab in T (300->1800 K,
          fronts 20 cells thick) with 1% multiplicative noise, and an
          unburnt/burnt composition blend following the progress variable.
"""
import numpy as np

P_ATM = 101325.0


def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def _grid(shape, dx):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) * dx[2], np.arange(ny) * dx[1], np.arange(nx) * dx[0], indexing="ij")
    return x, y, z


def _wavevec(rng):
    while True:
        k = rng.integers(-2, 3, size=3)
        if np.any(k != 0):
            return k


def sines(shape, dx, ns, seed):
    nz, ny, nx = shape
    dx = np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,))
    L = np.array([nx, ny, nz]) * dx
    x, y, z = _grid(shape, dx)
    rng = _rng(seed, 101)

    def phase(k, phi):
        return 2 * np.pi * (k[0] * x / L[0] + k[1] * y / L[1] + k[2] * z / L[2]) + phi

    s = np.zeros(shape)
    for _ in range(3):
        k = _wavevec(rng)
        s += np.sin(phase(k, rng.uniform(0, 2 * np.pi))) / 3.0
    T = 300.0 + 600.0 * (1.0 + s)
    Ya = rng.dirichlet(np.ones(ns))
    Yb = rng.dirichlet(np.ones(ns))
    kw = _wavevec(rng)
    w = 0.5 * (1.0 + np.sin(phase(kw, rng.uniform(0, 2 * np.pi))))
    Y = w[None] * Ya[:, None, None, None] + (1.0 - w[None]) * Yb[:, None, None, None]
    u = np.zeros((3,) + shape)
    for c in range(3):
        for _ in range(3):
            k = _wavevec(rng)
            u[c] += (10.0 / 3.0) * np.sin(phase(k, rng.uniform(0, 2 * np.pi)))
    p = np.full(shape, P_ATM)
    return dict(p=p, T=T, Y=Y, u=u)


def turb(shape, dx, ns, seed, kmax=16, urms=5.0, width_cells=10.0, noise=0.01):
    nz, ny, nx = shape
    dx = float(dx)
    L = np.array([nx, ny, nz]) * dx
    rng = _rng(seed, 202)
    # random-phase solenoidal field with E(k) ~ k^-5/3 on integer shells
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shell = np.rint(kmag).astype(np.int64)
    active = (shell >= 1) & (shell <= kmax)
    counts = np.bincount(shell[active], minlength=kmax + 1).astype(np.float64)
    amp = np.zeros(shape)
    sh = shell[active]
    amp[active] = np.sqrt(sh.astype(np.float64) ** (-5.0 / 3.0) / counts[sh])
    coef = (rng.standard_normal((3,) + shape) + 1j * rng.standard_normal((3,) + shape)) * amp[None]
    kvec = np.stack([KX, KY, KZ])
    k2 = np.where(kmag > 0, kmag ** 2, 1.0)
    coef = coef - kvec * (np.sum(kvec * coef, axis=0) / k2)[None]
    u = np.real(np.fft.ifftn(coef, axes=(1, 2, 3)))
    # ifft of a non-Hermitian spectrum: the real part is still solenoidal
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    u *= urms / np.sqrt(np.mean(np.sum(u ** 2, axis=0)) / 3.0)
    # periodic two-front slab along x
    x = (np.arange(nx) + 0.5) * dx
    delta = width_cells * dx
    prof = np.zeros(nx)
    for n in range(-2, 3):
        xs = x + n * L[0]
        prof += np.tanh((xs - L[0] / 4) / delta) - np.tanh((xs - 3 * L[0] / 4) / delta)
    prof = np.clip(prof, 0.0, 2.0) / 2.0
    T_clean = 300.0 + 1500.0 * prof
    T = np.broadcast_to(T_clean[None, None, :], shape).copy()
    T *= 1.0 + noise * rng.standard_normal(shape)
    c = np.broadcast_to(prof[None, None, :], shape)
    Yu = rng.dirichlet(np.ones(ns))
    Yb = rng.dirichlet(np.ones(ns))
    Y = (1.0 - c)[None] * Yu[:, None, None, None] + c[None] * Yb[:, None, None, None]
    p = np.full(shape, P_ATM)
    return dict(p=p, T=T, Y=Y, u=u)


def tile(fields, reps):
    """Periodic tiling of a field set (reps along z, y, x)."""
    rz, ry, rx = reps
    out = {}
    for k, v in fields.items():
        if v.ndim == 3:
            out[k] = np.tile(v, (rz, ry, rx))
        else:
            out[k] = np.tile(v, (1, rz, ry, rx))
    return out
