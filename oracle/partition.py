"""Graph partition of G(A) (paper Sec. 3.1, "Graph partition").

The paper partitions the adjacency graph with METIS/ParMETIS (Sec. 6), which is
neither available here nor bit-reproducible.  Two deterministic rules replace
it (reading recorded in the design notes):

* ``partition_blocks``: Cartesian blocks, part id
  ``i/bx + (nx/bx) * (j/by + (ny/by) * (k/bz))`` for cell ``(i, j, k)``.
* ``partition_bisect``: integer recursive bisection by a double breadth-first
  search, for irregular graphs.  Sets are processed depth-first, left child
  first; a set of at most ``hi`` cells becomes a part (numbered in emission
  order).  A larger set is split on its induced subgraph:

  1. ``u`` = vertex farthest (BFS hops) from the set's smallest vertex,
     ties to the smallest id;
  2. ``v`` = vertex farthest from ``u``, ties to the smallest id;
  3. ``key = d_u - d_v`` for vertices reachable from ``u``; every other
     vertex gets ``2**40 + c`` where ``c`` numbers the remaining connected
     components in order of their smallest vertex;
  4. vertices are sorted by ``(key, id)``;
  5. the first ``cut = clamp(n*rho // 100, lo, n - lo)`` go left, with
     ``rho = 40 + splitmix64(seed ^ node) % 21`` and ``node`` the heap index
     of the set (root 1, children ``2 node`` and ``2 node + 1``).

Only integer arithmetic decides anything, so any correct implementation of
these rules yields the same map.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse import csgraph

MASK64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output for input state ``x`` (Steele, Lea and Flood 2014;
    constants as published by Vigna): one increment by the golden-ratio
    constant followed by the two xor-shift-multiply rounds and a final
    xor-shift."""
    z = (int(x) + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def partition_blocks(dims, block):
    """Block partition of an ``nx x ny x nz`` grid (x fastest) into
    ``bx x by x bz`` blocks.  Returns (part int32[N], nparts)."""
    nx, ny, nz = dims
    bx, by, bz = block
    if nx % bx or ny % by or nz % bz:
        raise ValueError("block sizes must divide the grid")
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mx, my = nx // bx, ny // by
    part = (i // bx) + mx * ((j // by) + my * (k // bz))
    return part.ravel().astype(np.int32), mx * my * (nz // bz)


def _adjacency(row_ptr, col, val, n):
    """Symmetric adjacency of G(A): (k, l) with k != l and a_kl != 0."""
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    keep = (rows != col) & (val != 0)
    G = sp.csr_matrix((np.ones(int(keep.sum()), dtype=np.int8),
                       (rows[keep], col[keep])), shape=(n, n))
    return G


def _hops(G, src):
    d = csgraph.shortest_path(G, method="D", unweighted=True, directed=False, indices=src)
    return d


def _farthest(d):
    reach = np.isfinite(d)
    dm = np.where(reach, d, -1.0)
    return int(np.flatnonzero(dm == dm.max())[0])


def _split(Gsub, node, seed, lo):
    """Order of the local vertices and the cut position for one set."""
    n = Gsub.shape[0]
    d0 = _hops(Gsub, 0)
    u = _farthest(d0)
    du = _hops(Gsub, u)
    v = _farthest(du)
    dv = _hops(Gsub, v)
    reach = np.isfinite(du)
    key = np.zeros(n, dtype=np.int64)
    key[reach] = (du[reach] - dv[reach]).astype(np.int64)
    if not reach.all():
        _, labels = csgraph.connected_components(Gsub, directed=False)
        others = np.flatnonzero(~reach)
        # number the other components by their smallest vertex
        first = {}
        for x in others:
            lab = labels[x]
            if lab not in first:
                first[lab] = len(first)
        key[others] = (1 << 40) + np.array([first[labels[x]] for x in others], dtype=np.int64)
    order = np.lexsort((np.arange(n), key))
    rho = 40 + splitmix64((seed ^ node) & MASK64) % 21
    cut = min(max((n * rho) // 100, lo), n - lo)
    return order, cut


def partition_bisect(row_ptr, col, val, n, lo=200, hi=800, seed=0):
    """Recursive double-BFS bisection (rules in the module docstring).

    Returns (part int32[N], nparts).  Requires ``hi >= 2*lo`` so every split
    is feasible.
    """
    if hi < 2 * lo:
        raise ValueError("need hi >= 2*lo")
    G = _adjacency(np.asarray(row_ptr), np.asarray(col), np.asarray(val), n)
    part = np.full(n, -1, dtype=np.int32)
    nparts = 0
    stack = [(1, np.arange(n, dtype=np.int64))]
    while stack:
        node, cells = stack.pop()
        if cells.size <= hi:
            part[cells] = nparts
            nparts += 1
            continue
        Gsub = G[cells][:, cells]
        order, cut = _split(Gsub, node, seed, lo)
        left = np.sort(cells[order[:cut]])
        right = np.sort(cells[order[cut:]])
        stack.append((2 * node + 1, right))
        stack.append((2 * node, left))
    return part, nparts
