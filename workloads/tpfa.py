"""TPFA assembly of the fine system ``A p = f`` from a face list.

Cell-centred two-point flux approximation (the discretization behind the
paper's experiments, Sec. 2 end and Sec. 7): an interior face ``(k, l)`` has
transmissibility ``T = t_k t_l / (t_k + t_l)`` and contributes ``+T`` to
``a_kk`` and ``a_ll`` and ``-T`` to ``a_kl = a_lk``; a Dirichlet face of cell
``k`` adds ``t_k`` to ``a_kk`` and ``t_k * pD`` to ``f_k``; no-flow faces add
nothing.  The result is symmetric bitwise (each ``T`` is computed once) with
negative off-diagonals and nonnegative row sums.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    """Square sparse matrix in CSR form, columns ascending within each row."""
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def matvec(self, x):
        return self.to_scipy() @ x


@dataclass
class Faces:
    """TPFA face list (see ``grids``): ``l == -1`` marks a Dirichlet face."""
    k: np.ndarray
    l: np.ndarray
    gk: np.ndarray
    gl: np.ndarray
    pD: np.ndarray

    @classmethod
    def from_dict(cls, d):
        return cls(k=np.asarray(d["k"], np.int64), l=np.asarray(d["l"], np.int64),
                   gk=np.asarray(d["gk"], np.float64), gl=np.asarray(d["gl"], np.float64),
                   pD=np.asarray(d["pD"], np.float64))

    @property
    def n_faces(self):
        return int(self.k.size)


def transmissibilities(faces, K):
    """Half-transmissibilities and face transmissibility for permeability ``K``.

    Returns ``(t_k, t_l, T)``; for Dirichlet faces ``t_l = 0`` and ``T = 0``.
    """
    interior = faces.l >= 0
    tk = K[faces.k] * faces.gk
    tl = np.zeros_like(tk)
    tl[interior] = K[faces.l[interior]] * faces.gl[interior]
    T = np.zeros_like(tk)
    T[interior] = tk[interior] * tl[interior] / (tk[interior] + tl[interior])
    return tk, tl, T


def assemble(faces, K, n, sources=None):
    """Assemble CSR ``A`` and right-hand side ``f`` (Dirichlet lifting + sources).

    ``sources``: optional float64[n] (or [n, r]) added to ``f``.
    """
    K = np.asarray(K, dtype=np.float64).ravel()
    tk, tl, T = transmissibilities(faces, K)
    interior = faces.l >= 0
    kk = faces.k[interior]
    ll = faces.l[interior]
    Ti = T[interior]
    bnd = ~interior
    diag = (np.bincount(kk, weights=Ti, minlength=n)
            + np.bincount(ll, weights=Ti, minlength=n)
            + np.bincount(faces.k[bnd], weights=tk[bnd], minlength=n))
    rows = np.concatenate([kk, ll, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([ll, kk, np.arange(n, dtype=np.int64)])
    vals = np.concatenate([-Ti, -Ti, diag])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if np.any((rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])):
        raise ValueError("duplicate face between the same pair of cells")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    A = CSR(n=n, row_ptr=row_ptr, col=cols.astype(np.int32), val=vals)
    f = np.bincount(faces.k[bnd], weights=tk[bnd] * faces.pD[bnd], minlength=n).astype(np.float64)
    if sources is not None:
        src = np.asarray(sources, dtype=np.float64)
        if src.ndim == 1:
            f = f + src
        else:
            f = f[:, None] + src
    return A, f
