"""Grid geometry -> TPFA face lists.

A face list describes the two-point flux discretization independently of the
permeability: for face ``f`` between cells ``k[f]`` and ``l[f]`` the
half-transmissibilities are ``t_k = K[k] * gk[f]`` and ``t_l = K[l] * gl[f]``
with geometric factors ``g = (c . n) / |c|^2`` (``c`` from the cell centre to
the face centre, ``n`` the outward area vector).  A Dirichlet boundary face has
``l = -1``, ``gl = 0`` and boundary value ``pD``.

Cartesian grids use unit cubes (unit squares in 2-D), so every geometric factor
is ``1 / 0.5 = 2``.
"""
import numpy as np


def cell_index(i, j, k, nx, ny):
    """Flat index of cell (i, j, k) with x fastest."""
    return i + nx * (j + ny * k)


def _grid_ids(nx, ny, nz):
    return np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)


def cartesian_faces(nx, ny, nz=1, dirichlet=()):
    """Face list of a uniform unit-cell Cartesian grid.

    ``dirichlet`` is a sequence of ``(axis, side, value)``: axis 0/1/2 = x/y/z,
    side 0 = the low boundary (e.g. x = 0), side 1 = the high boundary.
    All other boundary faces are no-flow.
    Returns a dict with arrays ``k, l, gk, gl, pD``.
    """
    ids = _grid_ids(nx, ny, nz)
    ks, ls = [], []
    # interior faces along x, y, z (in that order)
    ks.append(ids[:, :, :-1].ravel()); ls.append(ids[:, :, 1:].ravel())
    ks.append(ids[:, :-1, :].ravel()); ls.append(ids[:, 1:, :].ravel())
    if nz > 1:
        ks.append(ids[:-1, :, :].ravel()); ls.append(ids[1:, :, :].ravel())
    k = np.concatenate(ks)
    l = np.concatenate(ls)
    nint = k.size
    gk = np.full(nint, 2.0)
    gl = np.full(nint, 2.0)
    pD = np.zeros(nint)
    bk, bv = [], []
    for axis, side, value in dirichlet:
        sl = [slice(None)] * 3
        # ids is [z, y, x]; axis 0 (x) is the last array axis
        arr_axis = 2 - axis
        sl[arr_axis] = 0 if side == 0 else -1
        cells = ids[tuple(sl)].ravel()
        bk.append(cells)
        bv.append(np.full(cells.size, float(value)))
    if bk:
        bk = np.concatenate(bk)
        bv = np.concatenate(bv)
        k = np.concatenate([k, bk])
        l = np.concatenate([l, np.full(bk.size, -1, dtype=np.int64)])
        gk = np.concatenate([gk, np.full(bk.size, 2.0)])
        gl = np.concatenate([gl, np.zeros(bk.size)])
        pD = np.concatenate([pD, bv])
    return dict(k=k, l=l, gk=gk, gl=gl, pD=pD)


def distorted_vertices(nx, ny, nz, jitter, seed):
    """Lattice vertices ``[nz+1, ny+1, nx+1, 3]`` (xyz) displaced by U(-j, j)^3."""
    rng = np.random.default_rng([seed, 2])
    z, y, x = np.meshgrid(np.arange(nz + 1.0), np.arange(ny + 1.0),
                          np.arange(nx + 1.0), indexing="ij")
    v = np.stack([x, y, z], axis=-1)
    return v + rng.uniform(-jitter, jitter, size=v.shape)


def _quad(a, b, c, d):
    """Centre and area vector of the quad a-b-c-d (half the diagonal cross product)."""
    centre = 0.25 * (a + b + c + d)
    area = 0.5 * np.cross(c - a, d - b)
    return centre, area


def distorted_hex_faces(nx, ny, nz, jitter, seed, dirichlet=()):
    """Face list of a hexahedral grid with randomly displaced vertices.

    Cell centre = mean of its 8 vertices; face centre = mean of its 4 vertices;
    area vector = half the cross product of the face diagonals, oriented along
    +x / +y / +z.  ``dirichlet`` as in :func:`cartesian_faces`.
    Raises if any half-transmissibility factor is not positive.
    """
    V = distorted_vertices(nx, ny, nz, jitter, seed)
    cc = 0.125 * (V[:-1, :-1, :-1] + V[:-1, :-1, 1:] + V[:-1, 1:, :-1] + V[:-1, 1:, 1:]
                  + V[1:, :-1, :-1] + V[1:, :-1, 1:] + V[1:, 1:, :-1] + V[1:, 1:, 1:])
    # x-faces at vertex plane i: quad (j,k),(j+1,k),(j+1,k+1),(j,k+1) -> +x
    fx_c, fx_a = _quad(V[:-1, :-1, :], V[:-1, 1:, :], V[1:, 1:, :], V[1:, :-1, :])
    # y-faces at plane j: (i,k),(i,k+1),(i+1,k+1),(i+1,k) -> +y
    fy_c, fy_a = _quad(V[:-1, :, :-1], V[1:, :, :-1], V[1:, :, 1:], V[:-1, :, 1:])
    # z-faces at plane k: (i,j),(i+1,j),(i+1,j+1),(i,j+1) -> +z
    fz_c, fz_a = _quad(V[:, :-1, :-1], V[:, :-1, 1:], V[:, 1:, 1:], V[:, 1:, :-1])
    ids = _grid_ids(nx, ny, nz)

    def factor(centre, fc, n):
        c = fc - centre
        return np.einsum("...a,...a->...", c, n) / np.einsum("...a,...a->...", c, c)

    ks, ls, gks, gls = [], [], [], []
    # x interior: face plane i+1 between cell i (low) and i+1 (high)
    ks.append(ids[:, :, :-1]); ls.append(ids[:, :, 1:])
    gks.append(factor(cc[:, :, :-1], fx_c[:, :, 1:-1], fx_a[:, :, 1:-1]))
    gls.append(factor(cc[:, :, 1:], fx_c[:, :, 1:-1], -fx_a[:, :, 1:-1]))
    ks.append(ids[:, :-1, :]); ls.append(ids[:, 1:, :])
    gks.append(factor(cc[:, :-1, :], fy_c[:, 1:-1, :], fy_a[:, 1:-1, :]))
    gls.append(factor(cc[:, 1:, :], fy_c[:, 1:-1, :], -fy_a[:, 1:-1, :]))
    ks.append(ids[:-1, :, :]); ls.append(ids[1:, :, :])
    gks.append(factor(cc[:-1, :, :], fz_c[1:-1, :, :], fz_a[1:-1, :, :]))
    gls.append(factor(cc[1:, :, :], fz_c[1:-1, :, :], -fz_a[1:-1, :, :]))
    k = np.concatenate([a.ravel() for a in ks])
    l = np.concatenate([a.ravel() for a in ls])
    gk = np.concatenate([a.ravel() for a in gks])
    gl = np.concatenate([a.ravel() for a in gls])
    pD = np.zeros(k.size)
    bounds = {
        (0, 0): (ids[:, :, 0], cc[:, :, 0], fx_c[:, :, 0], -fx_a[:, :, 0]),
        (0, 1): (ids[:, :, -1], cc[:, :, -1], fx_c[:, :, -1], fx_a[:, :, -1]),
        (1, 0): (ids[:, 0, :], cc[:, 0, :], fy_c[:, 0, :], -fy_a[:, 0, :]),
        (1, 1): (ids[:, -1, :], cc[:, -1, :], fy_c[:, -1, :], fy_a[:, -1, :]),
        (2, 0): (ids[0], cc[0], fz_c[0], -fz_a[0]),
        (2, 1): (ids[-1], cc[-1], fz_c[-1], fz_a[-1]),
    }
    for axis, side, value in dirichlet:
        cells, cen, fc, n = bounds[(axis, side)]
        g = factor(cen, fc, n).ravel()
        k = np.concatenate([k, cells.ravel()])
        l = np.concatenate([l, np.full(g.size, -1, dtype=np.int64)])
        gk = np.concatenate([gk, g])
        gl = np.concatenate([gl, np.zeros(g.size)])
        pD = np.concatenate([pD, np.full(g.size, float(value))])
    if not (np.all(gk > 0) and np.all(gl[l >= 0] > 0)):
        raise ValueError("distorted grid produced a nonpositive half-transmissibility")
    return dict(k=k.astype(np.int64), l=l.astype(np.int64), gk=gk, gl=gl, pD=pD)
