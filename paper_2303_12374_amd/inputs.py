"""Seeded synthetic inputs for the staggered-grid stencil step.

This module is shared by the CPU oracle (test infrastructure) and by the GPU
path's callers (tests, benchmark, server traces).  It holds no arithmetic of
the method itself: only random numbers, analytic field values at the grid's
staggered positions, the vertical grid, and the padded-array embedding.

Grid conventions (the paper states the problem as fields on a 3-D grid with
grid dimensions, spacings, viscosity and precision; Section "Application" and
"Tunable Parameters").  The readings below are this library's:

* interior sizes ``itot, jtot, ktot``; ``gh`` ghost cells per side in x and
  y (1, or 3 for the fifth-order advection scheme), one in z;
* index ``idx(i, j, k) = off + i + j*jstride + k*kstride`` with
  ``i in [1-gh, itot+gh]``, ``j in [1-gh, jtot+gh]``, ``k in [0, ktot+1]``,
  interior ``i in [1, itot]`` etc.;
* Arakawa-C staggering: u at (xh_i, y_j, z_k), v at (x_i, yh_j, z_k),
  w at (x_i, y_j, zh_k) with ``xh_i = (i-1) dx`` and ``x_i = (i-1/2) dx``;
* ``Lx = Ly = 1`` so ``dx = 1/itot``, ``dy = 1/jtot``;
* z is centers-primary: ``z_k = Lz (1 - tanh(g (1 - (k-1/2)/ktot)) / tanh g)``
  for the stretched grid (uniform ``z_k = (k-1/2) Lz/ktot`` when ``g = 0``),
  ghost centers by reflection about the walls, and faces at the midpoints of
  neighbouring centers; ``Lz = ktot / max(itot, jtot)``.

Random numbers: counter-based SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014).  The value for
counter ``key`` is the generator's output after one step from state ``key``:
``z = key + 0x9E3779B97F4A7C15``, then the published finaliser
``z = (z ^ z>>30) * 0xBF58476D1CE4E5B9; z = (z ^ z>>27) * 0x94D049BB133111EB;
z ^= z>>31``; the uniform double is ``(z >> 11) * 2**-53`` in [0, 1).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA_SM = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

FIELD_U, FIELD_V, FIELD_W = 0, 1, 2
MEAN_FLOW = (1.0, 0.5, 0.0)


def splitmix64(keys: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state ``keys`` (uint64 array), wrapping arithmetic."""
    z = np.asarray(keys, dtype=np.uint64) + GAMMA_SM
    t = z >> np.uint64(30)
    z ^= t
    z *= M1
    np.right_shift(z, np.uint64(27), out=t)
    z ^= t
    z *= M2
    np.right_shift(z, np.uint64(31), out=t)
    z ^= t
    return z


def uniform01(keys: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from counters ``keys``."""
    return (splitmix64(keys) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def field_key_base(seed: int, field: int) -> np.uint64:
    """Counter base of one field: ``(seed*8 + field) << 40``."""
    return np.uint64(((seed * 8 + field) << 40) & 0xFFFFFFFFFFFFFFFF)


def uniform_field(seed: int, field: int, itot: int, jtot: int, ktot: int) -> np.ndarray:
    """U[-1, 1) noise on the interior, shape (ktot, jtot, itot), C order.

    Counter of interior point (i', j', k') (0-based) is
    ``base + i' + itot*(j' + jtot*k')``.
    """
    with np.errstate(over="ignore"):
        n = itot * jtot * ktot
        keys = field_key_base(seed, field) + np.arange(n, dtype=np.uint64)
        r = uniform01(keys)
    return (2.0 * r - 1.0).reshape(ktot, jtot, itot)


def _phase(seed: int, field: int, n: int, which: int) -> float:
    """Phase in [0, 2 pi) for mode ``n`` and axis ``which`` of a sinusoid field."""
    with np.errstate(over="ignore"):
        key = field_key_base(seed, field) + np.uint64((1 << 39) + 3 * n + which)
        return float(uniform01(np.array([key], dtype=np.uint64))[0]) * 2.0 * math.pi


# --------------------------------------------------------------------------
# vertical grid
# --------------------------------------------------------------------------

def domain_height(itot: int, jtot: int, ktot: int) -> float:
    """Lz = ktot / max(itot, jtot): cells of unit mean aspect ratio."""
    return ktot / max(itot, jtot)


def zgrid(ktot: int, Lz: float, gamma: float = 1.5) -> dict:
    """Centers-primary vertical grid with ghost levels, arrays of length ktot+2.

    Returns z, zh, dz, dzh, dzi, dzhi.  ``gamma == 0`` gives a uniform grid.
    Faces are midpoints of neighbouring centers; the ghost center below the
    bottom wall and above the top wall are reflections of the first and last
    interior centers; ``zh[0]`` is the reflection of ``zh[2]`` about the
    bottom wall.  Metric ghosts not defined by a difference copy their
    neighbour (``dz[0]=dz[1]``, ``dz[ktot+1]=dz[ktot]``, ``dzh[0]=dzh[1]``).
    """
    kc = ktot + 2
    z = np.zeros(kc)
    k = np.arange(1, ktot + 1, dtype=np.float64)
    if gamma == 0.0:
        z[1:ktot + 1] = (k - 0.5) * (Lz / ktot)
    else:
        # the C library's tanh, one level at a time: numpy's vector tanh can
        # differ from it in the last bit, and the served form computes the
        # same grid in C
        z[1:ktot + 1] = [Lz * (1.0 - math.tanh(gamma * (1.0 - (kk - 0.5) / ktot)) / math.tanh(gamma)) for kk in k]
    z[0] = -z[1]
    z[ktot + 1] = 2.0 * Lz - z[ktot]
    zh = np.zeros(kc)
    zh[1:ktot + 2] = 0.5 * (z[0:ktot + 1] + z[1:ktot + 2])
    zh[0] = -zh[2] if ktot >= 1 else 0.0
    dz = np.zeros(kc)
    dz[1:ktot + 1] = zh[2:ktot + 2] - zh[1:ktot + 1]
    dz[0] = dz[1]
    dz[ktot + 1] = dz[ktot]
    dzh = np.zeros(kc)
    dzh[1:ktot + 2] = z[1:ktot + 2] - z[0:ktot + 1]
    dzh[0] = dzh[1]
    return dict(z=z, zh=zh, dz=dz, dzh=dzh, dzi=1.0 / dz, dzhi=1.0 / dzh, Lz=Lz, gamma=gamma)


def coords(itot: int, jtot: int, zg: dict, gh: int = 1) -> dict:
    """Cell-center and face coordinates, ghost cells included (length n+2*gh,
    entry 0 is index 1-gh)."""
    dx, dy = 1.0 / itot, 1.0 / jtot
    i = np.arange(1 - gh, itot + gh + 1, dtype=np.float64)
    j = np.arange(1 - gh, jtot + gh + 1, dtype=np.float64)
    return dict(x=(i - 0.5) * dx, xh=(i - 1.0) * dx, y=(j - 0.5) * dy, yh=(j - 1.0) * dy,
                z=zg["z"], zh=zg["zh"])


def staggered_positions(field: int, itot: int, jtot: int, zg: dict, gh: int = 1):
    """Broadcastable (Z, Y, X) coordinate arrays of one field, ghosts included."""
    c = coords(itot, jtot, zg, gh)
    X = c["xh"] if field == FIELD_U else c["x"]
    Y = c["yh"] if field == FIELD_V else c["y"]
    Z = c["zh"] if field == FIELD_W else c["z"]
    return Z[:, None, None], Y[None, :, None], X[None, None, :]


# --------------------------------------------------------------------------
# field recipes
# --------------------------------------------------------------------------

def random_fields(seed: int, itot: int, jtot: int, ktot: int, mean=MEAN_FLOW):
    """u, v, w interior = U[-1, 1) noise + mean flow (1.0, 0.5, 0)."""
    return [uniform_field(seed, f, itot, jtot, ktot) + mean[f] for f in range(3)]


FIELD_EVISC = 3


def evisc_field(seed: int, itot: int, jtot: int, ktot: int, mean: float = 1e-3, amp: float = 0.5):
    """A positive eddy-viscosity field at cell centers:
    ``mean * (1 + amp * U[-1, 1))`` from stream 3 of ``seed``."""
    return mean * (1.0 + amp * uniform_field(seed, FIELD_EVISC, itot, jtot, ktot))


def sinusoid_fields(seed: int, itot: int, jtot: int, ktot: int, zg: dict,
                    nmodes: int = 8, noise: float = 0.1, mean=MEAN_FLOW):
    """Sum of modes n = 1..nmodes with amplitude 1/n plus seeded noise.

    f = mean + sum_n (1/n) sin(2 pi n x + a_n) cos(2 pi n y + b_n) cos(pi n z / Lz + d_n)
        + noise * U[-1, 1), evaluated at each field's staggered position.
    """
    out = []
    Lz = zg["Lz"]
    for f in range(3):
        Z, Y, X = staggered_positions(f, itot, jtot, zg)
        Z, Y, X = Z[1:ktot + 1, 0, 0], Y[0, 1:jtot + 1, 0], X[0, 0, 1:itot + 1]
        # each mode is a separable product, so the sum over modes is a
        # (ktot x nmodes) @ (nmodes x jtot*itot) matrix product
        zm = np.empty((ktot, nmodes))
        xy = np.empty((nmodes, jtot * itot))
        for n in range(1, nmodes + 1):
            a, b, d = (_phase(seed, f, n, w) for w in range(3))
            zm[:, n - 1] = np.cos(math.pi * n * Z / Lz + d)
            xy[n - 1] = ((1.0 / n) * np.outer(np.cos(2 * math.pi * n * Y + b),
                                              np.sin(2 * math.pi * n * X + a))).ravel()
        acc = (zm @ xy).reshape(ktot, jtot, itot)
        acc += mean[f]
        acc += noise * uniform_field(seed, f, itot, jtot, ktot)
        out.append(acc)
    return out


# --------------------------------------------------------------------------
# padded layout
# --------------------------------------------------------------------------

def plain_layout(itot: int, jtot: int, ktot: int, gh: int = 1):
    """Unpadded layout: jstride = itot+2*gh, kstride = jstride*(jtot+2*gh),
    and off such that idx(1-gh, 1-gh, 0) = 0."""
    js = itot + 2 * gh
    ks = js * (jtot + 2 * gh)
    off = (gh - 1) * (js + 1)
    return off, js, ks, ks * (ktot + 2)


def padded_view(buf: np.ndarray, itot: int, jtot: int, ktot: int, off: int, js: int, ks: int,
                gh: int = 1):
    """Strided (ktot+2, jtot+2*gh, itot+2*gh) view of a flat buffer in the
    index layout; view[k, j, i] is element (i+1-gh, j+1-gh, k)."""
    item = buf.itemsize
    start = off - (gh - 1) * (js + 1)
    return np.lib.stride_tricks.as_strided(
        buf[start:], shape=(ktot + 2, jtot + 2 * gh, itot + 2 * gh), strides=(ks * item, js * item, item))


def interior_view(buf: np.ndarray, itot: int, jtot: int, ktot: int, off: int, js: int, ks: int,
                  gh: int = 1):
    """The (ktot, jtot, itot) interior of a flat buffer in the index layout."""
    return padded_view(buf, itot, jtot, ktot, off, js, ks, gh)[1:ktot + 1, gh:jtot + gh, gh:itot + gh]


def embed(interior: np.ndarray, off: int, js: int, ks: int, alloc: int,
          dtype=np.float64, fill=np.nan, gh: int = 1) -> np.ndarray:
    """Flat buffer of ``alloc`` elements holding ``interior`` at [1..n] in each axis.

    Ghost and padding cells hold ``fill`` (NaN by default) so that a read of
    a cell the caller did not define shows up in the result.
    """
    ktot, jtot, itot = interior.shape
    buf = np.full(alloc, fill, dtype=dtype)
    interior_view(buf, itot, jtot, ktot, off, js, ks, gh)[...] = interior
    return buf


def analytic_padded(fn, field: int, itot: int, jtot: int, ktot: int, zg: dict,
                    off: int, js: int, ks: int, alloc: int, gh: int = 1) -> np.ndarray:
    """Flat FP64 buffer with ``fn(x, y, z)`` at every cell, ghosts included.
    ``field`` 3 is a cell-center scalar (the position of v's x, u's y and z)."""
    Z, Y, X = staggered_positions(field, itot, jtot, zg, gh)
    vals = np.broadcast_to(fn(X, Y, Z), (ktot + 2, jtot + 2 * gh, itot + 2 * gh))
    buf = np.full(alloc, np.nan)
    padded_view(buf, itot, jtot, ktot, off, js, ks, gh)[...] = vals
    return buf


# --------------------------------------------------------------------------
# batched and served workloads
# --------------------------------------------------------------------------

BATCH_SIZES = (32, 64, 96, 128, 192)


def batch_shapes(seed: int = 3, n_random: int = 48, n_aniso: int = 8):
    """Grid shapes (itot, jtot, ktot) of the batched workload.

    ``n_random`` grids draw each axis independently and uniformly from
    {32, 64, 96, 128, 192} (counters of stream 7 of ``seed``), followed by
    ``n_aniso`` anisotropic 256 x 256 x 32 grids.
    """
    with np.errstate(over="ignore"):
        keys = field_key_base(seed, 7) + np.arange(3 * n_random, dtype=np.uint64)
        r = uniform01(keys)
    idx = np.minimum((r * len(BATCH_SIZES)).astype(np.int64), len(BATCH_SIZES) - 1)
    shapes = [tuple(int(BATCH_SIZES[i]) for i in idx[3 * n:3 * n + 3]) for n in range(n_random)]
    return shapes + [(256, 256, 32)] * n_aniso
