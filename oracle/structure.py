"""Permutation, interface edge sets and mortar numbering (paper Sec. 3.1-3.2).

* Permutation ``P`` (eq. linear-system-perm): unknowns reordered by subdomain;
  inside a subdomain they keep ascending original index.  ``perm[new] = old``.
* Interface edges (eq. Eij, eq. E): stored couplings ``a_kl != 0`` with
  ``part[k] < part[l]``; the pair ``(k, l)`` and ``(l, k)`` is one edge.  Edges
  are ordered by ``(part[k], part[l], k, l)`` in original indices, so each
  ``E_ij`` is ordered consistently from both sides.
* Mortar space (Sec. 5.4, piecewise constant): one basis function per
  subdomain pair ``(i, j)``, numbered in lexicographic order of ``(i, j)``;
  one function per pair even when ``E_ij`` is disconnected.  With
  ``mortar="edge"`` every edge gets its own basis function (``Lambda = R^E``,
  the case in which the method reproduces ``A`` exactly, Sec. 3.3).
* ``I_i`` (Sec. 3.4): the basis functions whose support meets ``E_i``,
  ascending.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Structure:
    n: int
    nparts: int
    part: np.ndarray        # int32[n]
    perm: np.ndarray        # int32[n], perm[new] = old
    sub_ptr: np.ndarray     # int64[m+1]
    edge_k: np.ndarray      # int32[|E|], endpoint in the lower subdomain (original index)
    edge_l: np.ndarray      # int32[|E|], endpoint in the higher subdomain
    edge_a: np.ndarray      # float64[|E|], a_kl (the diagonal of W)
    iface_ptr: np.ndarray   # int64[N_Lambda+1], edges of basis function n
    iface_ij: np.ndarray    # int32[N_Lambda, 2], (i, j) with i < j
    I: list                 # I[i] = ascending int array of basis functions touching i

    @property
    def n_iface(self):
        return self.iface_ij.shape[0]

    @property
    def n_edges(self):
        return self.edge_k.size

    def omega(self, i):
        """Original indices of subdomain i, ascending."""
        return self.perm[self.sub_ptr[i]:self.sub_ptr[i + 1]]


class PositiveCouplingError(ValueError):
    pass


def build_structure(A, part, mortar="interface"):
    """Build the index structure of AlgMortar for CSR ``A`` and ``part``."""
    n = A.n
    part = np.asarray(part, dtype=np.int64)
    m = int(part.max()) + 1
    counts = np.bincount(part, minlength=m)
    if np.any(counts == 0):
        raise ValueError("empty subdomain")
    perm = np.lexsort((np.arange(n), part)).astype(np.int32)
    sub_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=sub_ptr[1:])

    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
    cols = A.col.astype(np.int64)
    vals = A.val
    sel = (vals != 0) & (part[rows] < part[cols])
    k, l, a = rows[sel], cols[sel], vals[sel]
    if np.any(a > 0):
        raise PositiveCouplingError("positive inter-subdomain coupling violates W < 0")
    order = np.lexsort((l, k, part[l], part[k]))
    k, l, a = k[order], l[order], a[order]
    pi, pj = part[k], part[l]
    ne = k.size
    if mortar == "interface":
        new = np.ones(ne, dtype=bool)
        new[1:] = (pi[1:] != pi[:-1]) | (pj[1:] != pj[:-1])
        starts = np.flatnonzero(new)
    elif mortar == "edge":
        starts = np.arange(ne)
    else:
        raise ValueError(mortar)
    iface_ptr = np.append(starts, ne).astype(np.int64)
    iface_ij = np.stack([pi[starts], pj[starts]], axis=1).astype(np.int32)
    I = [[] for _ in range(m)]
    for nidx, (i, j) in enumerate(iface_ij):
        I[i].append(nidx)
        I[j].append(nidx)
    I = [np.array(sorted(x), dtype=np.int64) for x in I]
    return Structure(n=n, nparts=m, part=part.astype(np.int32), perm=perm, sub_ptr=sub_ptr,
                     edge_k=k.astype(np.int32), edge_l=l.astype(np.int32), edge_a=a,
                     iface_ptr=iface_ptr, iface_ij=iface_ij, I=I)
