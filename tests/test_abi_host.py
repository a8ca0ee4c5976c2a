"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, its host partitioners and interface structure equal the oracle's bit
for bit, and argument validation rejects bad inputs before any device work."""
import hashlib
import json
import os
import re

import numpy as np
import pytest

import paper_2607_22905_amd as am
from paper_2607_22905_amd import AlgMortarError
from oracle import partition_blocks, partition_bisect, build_structure
from workloads import make_config
from workloads.grids import cartesian_faces, distorted_hex_faces
from workloads.tpfa import Faces, assemble, CSR
from tests._problems import random_mmatrix, dense_csr, random_3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = am.load()
    hdr = open(os.path.join(ROOT, "include", "algmortar.h")).read()
    names = re.findall(r"^(?:am_status|const char\*)\s+(\w+)\(", hdr, flags=re.M)
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("dims,block", [((64, 64, 1), (16, 16, 1)), ((12, 8, 6), (4, 4, 3)),
                                        ((16, 16, 16), (8, 8, 8)), ((5, 7, 3), (5, 7, 1))])
def test_partition_blocks_bit_exact(dims, block):
    a, ma = am.partition_blocks(dims, block)
    b, mb = partition_blocks(dims, block)
    assert ma == mb and np.array_equal(a, b)


def _grid(nx, ny, nz, distorted=False, seed=0):
    n = nx * ny * nz
    f = distorted_hex_faces(nx, ny, nz, 0.3, seed, [(0, 0, 0.0)]) if distorted else \
        cartesian_faces(nx, ny, nz, [(0, 0, 0.0)])
    A, _ = assemble(Faces.from_dict(f), np.exp(np.random.default_rng(seed).normal(size=n)), n)
    return A


@pytest.mark.parametrize("shape,seed", [((24, 20, 10), 5), ((40, 30, 8), 1), ((2000, 1, 1), 0)])
def test_partition_bisect_bit_exact(shape, seed):
    A = _grid(*shape, distorted=shape[2] > 1, seed=seed)
    a, ma = am.partition_bisect(A, 200, 800, seed)
    b, mb = partition_bisect(A.row_ptr, A.col, A.val, A.n, 200, 800, seed)
    assert ma == mb and np.array_equal(a, b)


def test_partition_bisect_full_c3_matches_golden():
    with open(os.path.join(ROOT, "tests", "golden", "structure.json")) as f:
        gold = json.load(f)["c3"]
    P = make_config("c3")
    part, m = am.partition_bisect(P.A, 200, 800, 3)
    assert m == gold["nparts"]
    assert hashlib.sha256(part.astype(np.int32).tobytes()).hexdigest() == gold["part"]
    s = am.structure(P.A, part, m)
    assert hashlib.sha256(s["iface_ij"].astype(np.int32).tobytes()).hexdigest() == gold["iface_ij"]
    assert hashlib.sha256(s["edge_k"].tobytes()).hexdigest() == gold["edge_k"]


def _check_structure(A, part, m, mortar="interface"):
    s = am.structure(A, part, m, mortar)
    st = build_structure(A, part, mortar)
    for k in ("perm", "sub_ptr", "iface_ptr", "edge_k", "edge_l"):
        assert np.array_equal(s[k], getattr(st, k)), k
    assert np.array_equal(s["iface_ij"], st.iface_ij)


def test_structure_bit_exact_blocks():
    for name in ("c1", "c2"):
        P = make_config(name)
        part, m = partition_blocks(P.dims, P.partition[1])
        _check_structure(P.A, part, m)


def test_structure_bit_exact_per_edge_and_bisect():
    P = random_3d(6, 6, 4, 1.0, 1, block=(3, 3, 2))
    part, m = partition_blocks(P.dims, P.partition[1])
    _check_structure(P.A, part, m, "edge")
    A = _grid(30, 20, 6, distorted=True, seed=3)
    part, m = partition_bisect(A.row_ptr, A.col, A.val, A.n, 200, 800, 2)
    _check_structure(A, part, m)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_structure_bit_exact_random_mmatrix(seed):
    Ad = random_mmatrix(60, 0.1, seed)
    Ad[3, 7] = Ad[7, 3] = 0.0  # explicit zeros are stored but are not couplings
    A = dense_csr(Ad)
    rp, ci, v = A.row_ptr.copy(), list(A.col), list(A.val)
    part = np.random.default_rng(seed).integers(0, 6, size=60).astype(np.int32)
    part[:6] = np.arange(6)
    _check_structure(A, part, 6)


def test_structure_independent_of_host_threads(monkeypatch):
    """The host structure (validation, interface edges) runs on several host
    threads; its output is the same for any thread count."""
    A = _grid(48, 36, 12, distorted=True, seed=5)
    part, m = partition_bisect(A.row_ptr, A.col, A.val, A.n, 200, 800, 3)
    outs = []
    for t in ("1", "8", "3"):
        monkeypatch.setenv("ALGMORTAR_HOST_THREADS", t)
        outs.append(am.structure(A, part, m))
    for o in outs[1:]:
        for k, v in outs[0].items():
            assert np.array_equal(o[k], v), k
    # the lowest failing row is named whatever the thread count
    bad = CSR(n=A.n, row_ptr=A.row_ptr, col=A.col, val=A.val.copy())
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    offd = np.nonzero(A.col != rows)[0]
    bad.val[offd[[2000, 9000]]] *= 2.0  # two asymmetric pairs
    msgs = set()
    for t in ("1", "8"):
        monkeypatch.setenv("ALGMORTAR_HOST_THREADS", t)
        with pytest.raises(AlgMortarError) as e:
            am.structure(bad, part, m)
        assert e.value.status_name == "AM_ERR_NOT_SYMMETRIC"
        msgs.add(str(e.value))
    assert len(msgs) == 1, msgs


def _small():
    P = random_3d(4, 4, 2, 1.0, 0, block=(2, 2, 2))
    part, m = partition_blocks(P.dims, P.partition[1])
    return P.A, part, m


def _expect(status_name, fn):
    with pytest.raises(AlgMortarError) as ei:
        fn()
    assert ei.value.status_name == status_name, str(ei.value)


def test_validation_positive_coupling():
    A, part, m = _small()
    val = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = np.flatnonzero(rows != A.col)[0]
    k, l = rows[off], A.col[off]
    val[off] = 0.5
    # keep symmetry
    j = np.flatnonzero((rows == l) & (A.col == k))[0]
    val[j] = 0.5
    B = CSR(A.n, A.row_ptr, A.col, val)
    _expect("AM_ERR_POSITIVE_COUPLING", lambda: am.structure(B, part, m))


def test_validation_asymmetric_nan_and_diagonal():
    A, part, m = _small()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = np.flatnonzero(rows != A.col)[0]
    val = A.val.copy()
    val[off] *= 1.0000001
    _expect("AM_ERR_NOT_SYMMETRIC", lambda: am.structure(CSR(A.n, A.row_ptr, A.col, val), part, m))
    val = A.val.copy()
    val[off + 1] = np.nan
    _expect("AM_ERR_ARG", lambda: am.structure(CSR(A.n, A.row_ptr, A.col, val), part, m))
    val = A.val.copy()
    val[rows == A.col] *= -1
    _expect("AM_ERR_NOT_SPD", lambda: am.structure(CSR(A.n, A.row_ptr, A.col, val), part, m))


def test_validation_partition_and_pattern():
    A, part, m = _small()
    bad = part.copy()
    bad[0] = m
    _expect("AM_ERR_ARG", lambda: am.structure(A, bad, m))
    _expect("AM_ERR_ARG", lambda: am.structure(A, part, m + 1))  # empty subdomain
    col = A.col.copy()
    col[[0, 1]] = col[[1, 0]]  # unsorted row
    _expect("AM_ERR_ARG", lambda: am.structure(CSR(A.n, A.row_ptr, col, A.val), part, m))
    _expect("AM_ERR_ARG", lambda: am.partition_blocks((10, 10, 1), (3, 5, 1)))
    _expect("AM_ERR_ARG", lambda: am.partition_bisect(A, 200, 300, 0))


def test_setup_rejects_before_device_work():
    """Invalid inputs to algmortar_setup fail in host validation, so this
    runs without a GPU."""
    A, part, m = _small()
    val = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = np.flatnonzero(rows != A.col)[0]
    val[off] *= 2.0
    _expect("AM_ERR_NOT_SYMMETRIC", lambda: am.AlgMortar(CSR(A.n, A.row_ptr, A.col, val), part, m, stream=False))
    _expect("AM_ERR_ARG", lambda: am.AlgMortar(A, part, m, max_nrhs=17, stream=False))
    _expect("AM_ERR_ARG", lambda: am.AlgMortar(A, part, m + 3, stream=False))


def _nd_check(A, part, m, max_nrhs):
    """The library's nested-dissection order of the interface system against
    the oracle's interface structure: a permutation of the basis functions;
    blocks mutually uncoupled (no two basis functions in different blocks
    share a subdomain, so S has no entry between them, eq.
    interface-problem-alg); a block within the kernels' size limit."""
    st = build_structure(A, part)
    order, blk, ntop = am.interface_nd(A, part, m, max_nrhs)
    NL = st.n_iface
    assert sorted(order.tolist()) == list(range(NL))
    nrows = int(blk[-1])
    assert nrows + ntop == NL and blk[0] == 0 and (np.diff(blk) > 0).all()
    blk_of = np.full(NL, -1)
    for b in range(len(blk) - 1):
        blk_of[order[blk[b]:blk[b + 1]]] = b
    # every subdomain: the basis functions it touches lie in at most one block
    sub_blk = {}
    for n in range(NL):
        if blk_of[n] < 0:
            continue
        for s in st.iface_ij[n]:
            assert sub_blk.setdefault(int(s), blk_of[n]) == blk_of[n], (n, s)
    cap = min(4096, 7936 // max_nrhs)
    assert np.diff(blk).max() <= cap
    return order, blk, ntop, st


def test_interface_nd_128cube_planes():
    """128^3 in 8^3 blocks (a 16^3 box of subdomains): the cuts are the axis
    planes of the box (separators of 256, 2 x 128, 4 x 64, 8 x 64, 16 x 32
    basis functions; the depth taken keeps the blocks' padding within 15%),
    32 blocks of 304, reading 73 MB per solve instead of 1.06 GB."""
    P = make_config("c4")
    part, m = partition_blocks(P.dims, P.partition[1])
    order, blk, ntop, st = _nd_check(P.A, part, m, 1)
    assert ntop == 256 + 256 + 256 + 512 + 512
    assert len(blk) - 1 == 32 and (np.diff(blk) == 304).all()


@pytest.mark.parametrize("max_nrhs", [1, 16])
def test_interface_nd_bisection_grid(max_nrhs):
    A = _grid(40, 30, 12, distorted=True, seed=3)
    part, m = partition_bisect(A.row_ptr, A.col, A.val, A.n, 30, 120, 5)
    order, blk, ntop, st = _nd_check(A, part, m, max_nrhs)
    assert ntop < st.n_iface


def test_interface_nd_small_and_2d():
    P = make_config("c1")
    part, m = partition_blocks(P.dims, P.partition[1])
    _nd_check(P.A, part, m, 1)
    A = _grid(12, 8, 6)
    part, m = partition_blocks((12, 8, 6), (4, 4, 3))
    _nd_check(A, part, m, 4)
