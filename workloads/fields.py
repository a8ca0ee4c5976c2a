"""Seeded random permeability fields.

Recipe (the paper fixes none of it; its own fields are SPE10/SPE11 data and a
cross pattern that is only in a figure):

* ``grf``: Gaussian random field with Gaussian covariance
  ``sigma^2 exp(-1/2 sum_a (r_a/ell_a)^2)``.  White noise from
  ``numpy.random.default_rng(seed).standard_normal`` on a periodic grid padded
  by ``ceil(4*ell_a)`` cells per axis is filtered in Fourier space by the square
  root of the covariance's spectrum, cropped to the requested shape and then
  standardised to sample mean 0 and sample standard deviation ``sigma``.
* ``layered_log10k``: one ``U[-3, 3]`` draw of log10 K per z-layer plus a GRF
  given in natural-log units, clipped to ``[-3, 3]`` (contrast exactly 1e6 when
  both clips are reached).
* ``cross_log_kappa``: the periodic cross pattern (no randomness).

Arrays are indexed ``[z, y, x]`` (C order), so the flat index of cell
``(i, j, k)`` is ``i + nx*(j + ny*k)``.
"""
import math

import numpy as np


def grf(shape, ell, sigma, seed):
    """Return a Gaussian random field of the given ``shape`` (C order).

    ``ell`` is one correlation length per axis (same order as ``shape``) or a
    scalar.  Deterministic for a given ``seed``.
    """
    shape = tuple(int(s) for s in shape)
    if np.isscalar(ell):
        ell = (float(ell),) * len(shape)
    ell = tuple(float(e) for e in ell)
    pad = tuple(n + int(math.ceil(4.0 * e)) for n, e in zip(shape, ell))
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(pad)
    # periodic distance to the origin along each axis
    r2 = np.zeros(pad)
    for ax, (P, e) in enumerate(zip(pad, ell)):
        d = np.arange(P, dtype=np.float64)
        d = np.minimum(d, P - d) / e
        sh = [1] * len(pad)
        sh[ax] = P
        r2 = r2 + (d ** 2).reshape(sh)
    cov = np.exp(-0.5 * r2)
    spec = np.maximum(np.fft.rfftn(cov).real, 0.0)
    field = np.fft.irfftn(np.sqrt(spec) * np.fft.rfftn(noise), s=pad, axes=tuple(range(len(pad))))
    field = field[tuple(slice(0, n) for n in shape)]
    field = field - field.mean()
    field = field / field.std() * sigma
    return np.ascontiguousarray(field)


def layered_log10k(nx, ny, nz, ell_xyz, sigma, seed, lo=-3.0, hi=3.0):
    """log10 K for the layered high-contrast model, shape ``[nz, ny, nx]``.

    Layers are z-planes.  The per-layer draws come from a generator seeded with
    ``(seed, 1)`` so they are independent of the GRF noise.
    """
    g = grf((nz, ny, nx), (ell_xyz[2], ell_xyz[1], ell_xyz[0]), sigma, seed)
    u = np.random.default_rng([seed, 1]).uniform(lo, hi, size=nz)
    return np.clip(u[:, None, None] + g / math.log(10.0), lo, hi)


def cross_log_kappa(nx, ny, nz, base=8, lo=3, hi=4, kappa_hi=1.0e6):
    """ln kappa of the periodic high-contrast cross pattern, shape ``[nz, ny, nx]``.

    Reading of the cross-shaped field of the paper's scalability study (its
    exact pattern is only drawn in a figure): the grid is tiled by
    ``base^3`` tiles; inside a tile, a cell belongs to the cross when at least
    two of its three tile coordinates lie in the central band ``[lo, hi]``,
    i.e. three orthogonal bars through the tile centre.  Replicated over the
    tiles, the bars join into straight channels along x, y and z that cross
    the whole grid.  ``kappa = kappa_hi`` on the cross and 1 elsewhere.
    """
    def band(nn):
        a = np.arange(nn) % base
        return ((a >= lo) & (a <= hi)).astype(np.int64)
    cnt = (band(nz)[:, None, None] + band(ny)[None, :, None] + band(nx)[None, None, :])
    return np.where(cnt >= 2, math.log(kappa_hi), 0.0)
