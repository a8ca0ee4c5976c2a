"""Pins for the oracle's partitioners and interface structure (paper Sec. 3.1)."""
import numpy as np
import pytest

from oracle import partition_blocks, partition_bisect, splitmix64, build_structure
from oracle.partition import MASK64
from workloads import make_config
from workloads.grids import cartesian_faces
from workloads.tpfa import Faces, assemble


def test_splitmix64_published_values():
    # reference outputs of the SplitMix64 generator (state 0, and the
    # first three outputs from state 1234567)
    assert splitmix64(0) == 0xE220A8397B1DCDAF
    gamma = 0x9E3779B97F4A7C15
    s = 1234567
    outs = []
    for _ in range(3):
        outs.append(splitmix64(s))
        s = (s + gamma) & MASK64
    assert outs == [6457827717110365317, 3203168211198807973, 9817491932198370423]


def _block_counts(dims, block):
    m = [d // b for d, b in zip(dims, block)]
    area = [block[1] * block[2], block[0] * block[2], block[0] * block[1]]
    NL, E = 0, 0
    for a in range(3):
        cnt = (m[a] - 1) * int(np.prod([m[b] for b in range(3) if b != a]))
        NL += cnt
        E += cnt * area[a]
    return NL, E


@pytest.mark.parametrize("dims,block", [((64, 64, 1), (16, 16, 1)), ((16, 16, 16), (8, 8, 8)),
                                        ((12, 8, 6), (4, 4, 3)), ((9, 6, 4), (3, 2, 4))])
def test_block_partition_interface_counts(dims, block):
    nx, ny, nz = dims
    n = nx * ny * nz
    faces = Faces.from_dict(cartesian_faces(nx, ny, nz, [(0, 0, 0.0)]))
    A, _ = assemble(faces, np.ones(n), n)
    part, m = partition_blocks(dims, block)
    st = build_structure(A, part)
    NL, E = _block_counts(dims, block)
    assert st.n_iface == NL and st.n_edges == E
    assert m == int(np.prod([d // b for d, b in zip(dims, block)]))
    assert np.array_equal(np.bincount(part), np.full(m, int(np.prod(block))))


def test_block_partition_formula():
    part, m = partition_blocks((8, 4, 2), (4, 2, 1))
    # cell (i, j, k) -> i//4 + 2*(j//2 + 2*k)
    for k in range(2):
        for j in range(4):
            for i in range(8):
                assert part[i + 8 * (j + 4 * k)] == i // 4 + 2 * (j // 2 + 2 * k)
    assert m == 8


def test_structure_invariants():
    P = make_config("c1")
    part, m = partition_blocks(P.dims, (16, 16, 1))
    st = build_structure(P.A, part)
    # permutation: stable sort by (part, index)
    assert np.all(np.diff(part[st.perm]) >= 0)
    for i in range(m):
        om = st.omega(i)
        assert np.all(np.diff(om) > 0) and np.all(part[om] == i)
    assert st.sub_ptr[-1] == P.n
    # every stored coupling is interior or in exactly one E_ij (as (k,l) or (l,k))
    rows = np.repeat(np.arange(P.n), np.diff(P.A.row_ptr))
    cols = P.A.col
    cross = (part[rows] != part[cols])
    pairs = set(zip(st.edge_k.tolist(), st.edge_l.tolist()))
    assert len(pairs) == st.n_edges
    for k, l in zip(rows[cross], cols[cross]):
        assert ((k, l) in pairs) != ((l, k) in pairs)
    assert 2 * st.n_edges == int(cross.sum())
    # ordering by (part k, part l, k, l) and interface numbering
    key = np.stack([part[st.edge_k], part[st.edge_l], st.edge_k, st.edge_l], 1)
    assert all(tuple(key[e]) < tuple(key[e + 1]) for e in range(len(key) - 1))
    ij = [tuple(x) for x in st.iface_ij]
    assert ij == sorted(ij) and len(set(ij)) == len(ij)
    for nidx, (i, j) in enumerate(st.iface_ij):
        e0, e1 = st.iface_ptr[nidx], st.iface_ptr[nidx + 1]
        assert np.all(part[st.edge_k[e0:e1]] == i) and np.all(part[st.edge_l[e0:e1]] == j)
        assert nidx in st.I[i] and nidx in st.I[j]


def _path_csr(n):
    faces = Faces.from_dict(cartesian_faces(n, 1, 1, []))
    A, _ = assemble(faces, np.ones(n), n)
    return A


def _expected_path_parts(n, lo, hi, seed):
    """On a path graph the double BFS orders a set by descending index (u is
    the far end, key = d_u - d_v decreases with the index), so every split
    sends the ``cut`` highest indices left."""
    out = []

    def rec(lo_i, hi_i, node):  # interval [lo_i, hi_i)
        size = hi_i - lo_i
        if size <= hi:
            out.append((lo_i, hi_i))
            return
        rho = 40 + splitmix64(seed ^ node) % 21
        cut = min(max(size * rho // 100, lo), size - lo)
        rec(hi_i - cut, hi_i, 2 * node)
        rec(lo_i, hi_i - cut, 2 * node + 1)

    rec(0, n, 1)
    part = np.empty(n, dtype=np.int32)
    for p, (a, b) in enumerate(out):
        part[a:b] = p
    return part, len(out)


@pytest.mark.parametrize("n,seed", [(2000, 0), (3333, 7), (801, 3)])
def test_bisect_path_graph_closed_form(n, seed):
    A = _path_csr(n)
    part, m = partition_bisect(A.row_ptr, A.col, A.val, n, 200, 800, seed)
    exp, me = _expected_path_parts(n, 200, 800, seed)
    assert m == me and np.array_equal(part, exp)


def test_bisect_grid_sizes_and_determinism():
    nx, ny, nz = 24, 20, 10
    n = nx * ny * nz
    faces = Faces.from_dict(cartesian_faces(nx, ny, nz, []))
    A, _ = assemble(faces, np.ones(n), n)
    p1, m1 = partition_bisect(A.row_ptr, A.col, A.val, n, 200, 800, 5)
    p2, m2 = partition_bisect(A.row_ptr, A.col, A.val, n, 200, 800, 5)
    assert m1 == m2 and np.array_equal(p1, p2)
    sizes = np.bincount(p1)
    assert sizes.sum() == n and sizes.min() >= 200 and sizes.max() <= 800
    p3, _ = partition_bisect(A.row_ptr, A.col, A.val, n, 200, 800, 6)
    assert not np.array_equal(p1, p3)


def test_bisect_disconnected_components_go_right():
    # two disjoint paths of 700 cells: the set (1400 > 800) is split with the
    # component of vertex 0 first (keys d_u - d_v) and the other component last
    n = 1400
    faces = Faces.from_dict(cartesian_faces(700, 1, 1, []))
    A1, _ = assemble(faces, np.ones(700), 700)
    import scipy.sparse as sp
    A = sp.block_diag([A1.to_scipy(), A1.to_scipy()]).tocsr()
    A.sort_indices()
    part, m = partition_bisect(A.indptr.astype(np.int64), A.indices, A.data, n, 200, 800, 1)
    rho = 40 + splitmix64(1 ^ 1) % 21
    cut = min(max(n * rho // 100, 200), n - 200)
    # left = the first `cut` cells in (key, id) order: descending ids of the
    # first path, then the second path in ascending id order
    order = list(range(699, -1, -1)) + list(range(700, 1400))
    left = np.sort(order[:cut])
    assert np.all(part[left] == part[left[0]])
    assert part[left[0]] == 0
