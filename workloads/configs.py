"""The six synthetic workloads (and scaled-down variants for tests).

Every workload is fully determined by its name and seed:

``c1``  2-D 64x64, ``K = exp(g)``, ``g`` GRF (sigma 1, ell 8).  ``p = 0`` on
        the x = 0 edge, no-flow elsewhere; ``f = +1`` in cell (0,0) and ``-1`` in
        cell (63,63) (the compatibility constant is 0: the Dirichlet edge makes
        ``A`` nonsingular).  4x4 blocks of 16x16 cells.  PCG tol 1e-10.
``c2``  64^3 layered log10 K in [-3, 3] + GRF (sigma 1.5, ell 16x16x2), clipped
        (contrast 1e6).  ``p = 1`` on x = 0, ``p = 0`` on x = 64, ``f = 0``.
        512 blocks of 8^3.  tol 1e-8.
``c3``  128x128x64 hexahedra with vertices displaced by U(-0.3, 0.3)^3,
        ``ln K`` GRF (sigma 2, ell 8), ``p = 0`` on x = 0, 16 right-hand sides
        from injector/producer pairs (+1/-1 at 32 distinct seeded cells).
        Recursive bisection into parts of 200..800 cells.  tol 1e-8.
``c4``  128^3, ``K = exp(g)`` (sigma 1, ell 8), ``p = 0`` on x = 0, ``+1`` at
        cell (0,0,0), ``-1`` at (127,127,127).  4096 blocks of 8^3.  tol 1e-8.
``c5``  96^3, ``ln K`` GRF (sigma 2, ell 12x12x4), ``p = 1`` on x = 0,
        ``p = 0`` on x = 96.  1728 blocks of 8^3.  1000 seeded observation
        cells; observed pressures come from a forward solve with
        ``ln K + 0.1 g'`` (``g'`` an independent GRF, seed + 1).
``c6``  64^3 periodic cross pattern (``cross_log_kappa``: kappa = 1e6 on three
        orthogonal 2-cell-thick bars through the centre of every 8^3 tile, 1
        elsewhere), ``p = 0`` on y = 0, ``p = 1`` on y = 64, no-flow elsewhere,
        ``f = 0``.  512 blocks of 8^3.  tol 1e-8.

``theta`` (c2, c6): the contrast sweep ``K -> K^theta`` (``ln K`` scaled by
theta), so a field of contrast c gets contrast ``c^theta``.

The seed defaults to the config number.  ``scale`` shrinks a config
(dimensions divided, blocks kept) for fast tests.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .fields import cross_log_kappa, grf, layered_log10k
from .grids import cartesian_faces, distorted_hex_faces
from .tpfa import Faces, assemble, CSR

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5", "c6")


@dataclass
class Problem:
    name: str
    dims: tuple                 # (nx, ny, nz)
    A: CSR
    b: np.ndarray               # float64[n] or [n, nrhs] (column per RHS)
    faces: Faces
    logK: np.ndarray            # natural log of permeability, float64[n]
    partition: tuple            # ("blocks", (bx, by, bz)) or ("bisect", lo, hi, seed)
    tol: float
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.A.n

    @property
    def nrhs(self):
        return 1 if self.b.ndim == 1 else self.b.shape[1]


def _point_sources(n, cells_vals):
    s = np.zeros(n)
    for c, v in cells_vals:
        s[c] += v
    return s


def cartesian_problem(name, nx, ny, nz, logK, dirichlet, sources, block, tol, extra=None):
    n = nx * ny * nz
    faces = Faces.from_dict(cartesian_faces(nx, ny, nz, dirichlet))
    A, f = assemble(faces, np.exp(logK.ravel()), n, sources)
    return Problem(name=name, dims=(nx, ny, nz), A=A, b=f, faces=faces,
                   logK=logK.ravel().copy(), partition=("blocks", tuple(block)),
                   tol=tol, extra=extra or {})


def make_c1(seed=1, nx=64, ny=64, block=(16, 16, 1)):
    g = grf((ny, nx), 8.0, 1.0, seed)
    n = nx * ny
    src = _point_sources(n, [(0, 1.0), (n - 1, -1.0)])
    return cartesian_problem("c1", nx, ny, 1, g, [(0, 0, 0.0)], src, block, 1e-10)


def make_c2(seed=2, nx=64, ny=64, nz=64, block=(8, 8, 8), theta=1.0):
    log10k = layered_log10k(nx, ny, nz, (16.0, 16.0, 2.0), 1.5, seed)
    logK = theta * log10k * np.log(10.0)
    return cartesian_problem("c2", nx, ny, nz, logK, [(0, 0, 1.0), (0, 1, 0.0)],
                             None, block, 1e-8)


def make_c4(seed=4, nx=128, ny=128, nz=128, block=(8, 8, 8)):
    g = grf((nz, ny, nx), 8.0, 1.0, seed)
    n = nx * ny * nz
    src = _point_sources(n, [(0, 1.0), (n - 1, -1.0)])
    return cartesian_problem("c4", nx, ny, nz, g, [(0, 0, 0.0)], src, block, 1e-8)


def make_c5(seed=5, nx=96, ny=96, nz=96, block=(8, 8, 8), n_obs=1000, n_fd=20):
    g = grf((nz, ny, nx), (4.0, 12.0, 12.0), 2.0, seed)
    n = nx * ny * nz
    rng = np.random.default_rng([seed, 3])
    obs = np.sort(rng.choice(n, size=min(n_obs, n), replace=False)).astype(np.int64)
    g_pert = g + 0.1 * grf((nz, ny, nx), (4.0, 12.0, 12.0), 2.0, seed + 1)
    extra = dict(obs=obs, logK_pert=g_pert.ravel().copy(), n_fd=n_fd,
                 fd_seed=[seed, 4], fd_h=1e-6, adjoint_tol=1e-12)
    return cartesian_problem("c5", nx, ny, nz, g, [(0, 0, 1.0), (0, 1, 0.0)],
                             None, block, 1e-10, extra)


def make_c3(seed=3, nx=128, ny=128, nz=64, n_pairs=16, lo=200, hi=800):
    n = nx * ny * nz
    g = grf((nz, ny, nx), 8.0, 2.0, seed)
    faces = Faces.from_dict(distorted_hex_faces(nx, ny, nz, 0.3, seed, [(0, 0, 0.0)]))
    rng = np.random.default_rng([seed, 5])
    wells = rng.choice(n, size=2 * n_pairs, replace=False).astype(np.int64)
    src = np.zeros((n, n_pairs))
    for r in range(n_pairs):
        src[wells[2 * r], r] += 1.0
        src[wells[2 * r + 1], r] -= 1.0
    A, f = assemble(faces, np.exp(g.ravel()), n, src)
    return Problem(name="c3", dims=(nx, ny, nz), A=A, b=f, faces=faces,
                   logK=g.ravel().copy(), partition=("bisect", lo, hi, seed),
                   tol=1e-8, extra=dict(wells=wells))


def make_c6(seed=6, nx=64, ny=64, nz=64, block=(8, 8, 8), theta=1.0):
    logK = theta * cross_log_kappa(nx, ny, nz)
    return cartesian_problem("c6", nx, ny, nz, logK, [(1, 0, 0.0), (1, 1, 1.0)],
                             None, block, 1e-8)


_MAKERS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "c5": make_c5,
           "c6": make_c6}


def make_config(name, seed: Optional[int] = None, **kw):
    """Build a named workload; keyword arguments override its sizes."""
    maker = _MAKERS[name]
    if seed is None:
        return maker(**kw)
    return maker(seed=seed, **kw)
