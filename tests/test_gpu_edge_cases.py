"""Edge cases of the HIP path against the FP64 oracle, through the C-ABI:
zero right-hand sides (alone and as one column of a block), the smallest
non-trivial problem (two cells, two subdomains), one-cell subdomains
everywhere, a subdomain touching 100 mortar basis functions (accepted with
one right-hand side, refused with eight), the set-up limits (130 basis
functions on one subdomain, a subdomain whose bandwidth no ordering brings
to 128) and a right-hand-side count beyond the handle's maximum."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from paper_2607_22905_amd import AlgMortarError  # noqa: E402
from oracle import AlgMortarCPU, partition_blocks, pcg  # noqa: E402
from tests._problems import random_2d, random_3d  # noqa: E402

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _ragged():
    P = random_3d(18, 15, 8, 1.5, 11, block=(6, 5, 4))
    part, m = partition_blocks(P.dims, P.partition[1])
    return P, part, m


def test_zero_rhs_alone():
    P, part, m = _ragged()
    h = am.AlgMortar(P.A, part, m)
    z = cpu(h.apply(gpu(np.zeros(P.n))))
    assert np.array_equal(z, np.zeros(P.n))
    x, info, _ = h.pcg(gpu(np.zeros(P.n)), 1e-10)
    assert np.array_equal(cpu(x), np.zeros(P.n))
    assert info[0]["converged"] == 1 and info[0]["iterations"] == 0
    assert info[0]["rel_res"] == 0.0 and info[0]["true_rel_res"] == 0.0
    h.close()


def test_zero_column_in_a_block():
    """Column 1 of three is zero: it stops at iteration 0 with x = 0 while
    the other two follow their own oracle solves."""
    P, part, m = _ragged()
    ora = AlgMortarCPU(P.A, part)
    B = np.zeros((3, P.n))
    B[0] = P.b
    B[2] = np.random.default_rng(7).standard_normal(P.n)
    h = am.AlgMortar(P.A, part, m, max_nrhs=4)
    X, info, _ = h.pcg(gpu(B), 1e-10)
    X = cpu(X)
    assert np.array_equal(X[1], np.zeros(P.n))
    assert info[1]["converged"] == 1 and info[1]["iterations"] == 0
    for k in (0, 2):
        res = pcg(lambda v: ora.As @ v, B[k], ora.apply, 1e-10)
        assert info[k]["converged"] == 1
        assert abs(info[k]["iterations"] - res.iterations) <= 1
        assert rel(X[k], res.x) <= 1e-8
    h.close()


def test_two_cells_two_subdomains():
    """2 x 1 grid, one cell per subdomain, one interface of one edge."""
    P = random_2d(nx=2, ny=1, sigma=0.0, block=(1, 1, 1))
    part, m = partition_blocks(P.dims, (1, 1, 1))
    assert m == 2
    ora = AlgMortarCPU(P.A, part)
    h = am.AlgMortar(P.A, part, m)
    r = np.array([0.7, -1.3])
    assert rel(cpu(h.apply(gpu(r))), ora.apply(r)) <= 1e-12
    x, info, _ = h.pcg(gpu(r), 1e-12)
    xd = np.linalg.solve(ora.As.toarray(), r)
    assert info[0]["converged"] == 1 and rel(cpu(x), xd) <= 1e-12
    h.close()


def test_one_cell_subdomains():
    """4 x 4 x 3 grid, every cell its own subdomain (48 subdomains, 104
    interfaces of one edge each)."""
    P = random_3d(4, 4, 3, 1.0, 5, block=(1, 1, 1))
    part, m = partition_blocks(P.dims, (1, 1, 1))
    assert m == P.n
    ora = AlgMortarCPU(P.A, part)
    h = am.AlgMortar(P.A, part, m, max_nrhs=2)
    R = np.random.default_rng(8).standard_normal((2, P.n))
    Z = cpu(h.apply(gpu(R)))
    for k in range(2):
        assert rel(Z[k], ora.apply(R[k])) <= 1e-12
    x, info, _ = h.pcg(gpu(P.b), 1e-10)
    res = pcg(lambda v: ora.As @ v, P.b, ora.apply, 1e-10)
    assert info[0]["converged"] == 1
    assert abs(info[0]["iterations"] - res.iterations) <= 1
    assert rel(cpu(x), res.x) <= 1e-8
    h.close()


def _comb(nx):
    """nx x 2 grid: row 0 is one subdomain (a chain of nx cells), every cell
    of row 1 is a subdomain of its own, so subdomain 0 touches nx mortar
    basis functions (2 nx - 1 interfaces in all)."""
    P = random_2d(nx=nx, ny=2, sigma=1.0, seed=3, block=(1, 1, 1))
    k = np.arange(P.n)
    x, y = k % nx, k // nx
    part = np.where(y == 0, 0, 1 + x).astype(np.int32)
    return P, part, nx + 1


def test_subdomain_with_100_basis_functions():
    P, part, m = _comb(100)
    ora = AlgMortarCPU(P.A, part)
    assert ora.st.n_iface == 199
    assert int((np.asarray(ora.st.iface_ij) == 0).any(axis=1).sum()) == 100
    h = am.AlgMortar(P.A, part, m)
    rng = np.random.default_rng(9)
    for _ in range(2):
        r = rng.standard_normal(P.n)
        assert rel(cpu(h.apply(gpu(r))), ora.apply(r)) <= 1e-12
    b = rng.standard_normal(P.n)
    x, info, _ = h.pcg(gpu(b), 1e-10)
    res = pcg(lambda v: ora.As @ v, b, ora.apply, 1e-10)
    assert info[0]["converged"] == 1
    assert abs(info[0]["iterations"] - res.iterations) <= 1
    assert rel(cpu(x), res.x) <= 1e-8
    h.close()
    with pytest.raises(AlgMortarError) as e:
        am.AlgMortar(P.A, part, m, max_nrhs=8)
    assert e.value.status_name == "AM_ERR_UNSUPPORTED"


@pytest.mark.parametrize("nrhs,separate", [(8, False), (16, True)])
def test_subdomain_with_48_basis_functions_many_columns(nrhs, separate):
    """One subdomain touching 48 basis functions (more than the 32 interface
    slots the 8/16-column update keeps in registers, and than the 32 the
    matrix-core reconstruction fetches ahead) with 8 and 16 columns: applies
    of every column within 1e-12 of the oracle, PCG within 1e-8 of the oracle
    with the iteration count within one."""
    P, part, m = _comb(48)
    ora = AlgMortarCPU(P.A, part)
    assert int((np.asarray(ora.st.iface_ij) == 0).any(axis=1).sum()) == 48
    h = am.AlgMortar(P.A, part, m, max_nrhs=nrhs, separate_iface=separate)
    rng = np.random.default_rng(48)
    R = rng.standard_normal((nrhs, P.n))
    Z = cpu(h.apply(gpu(R)))
    for c in range(nrhs):
        assert rel(Z[c], ora.apply(R[c])) <= 1e-12, c
    X, infos, _ = h.pcg(gpu(R), 1e-10)
    X = cpu(X)
    for c in (0, nrhs - 1):
        res = pcg(lambda v: ora.As @ v, R[c], ora.apply, 1e-10)
        assert infos[c]["converged"] == 1
        assert abs(infos[c]["iterations"] - res.iterations) <= 1
        assert rel(X[c], res.x) <= 1e-8
    h.close()


def test_setup_limits():
    P, part, m = _comb(130)
    with pytest.raises(AlgMortarError) as e:
        am.AlgMortar(P.A, part, m)
    assert e.value.status_name == "AM_ERR_UNSUPPORTED"
    # a 20^3 block: every ordering leaves a bandwidth far above 128
    Q = random_3d(20, 20, 20, 0.5, 2, block=(20, 20, 20))
    part, m = partition_blocks(Q.dims, (20, 20, 20))
    with pytest.raises(AlgMortarError) as e:
        am.AlgMortar(Q.A, part, m)
    assert e.value.status_name == "AM_ERR_UNSUPPORTED"


def test_more_rhs_than_the_handle_allows():
    P, part, m = _ragged()
    h = am.AlgMortar(P.A, part, m, max_nrhs=2)
    R = gpu(np.ones((3, P.n)))
    with pytest.raises(AlgMortarError) as e:
        h.apply(R)
    assert e.value.status_name == "AM_ERR_ARG"
    with pytest.raises(AlgMortarError) as e:
        h.pcg(R, 1e-8)
    assert e.value.status_name == "AM_ERR_ARG"
    # the handle still works afterwards
    r = np.random.default_rng(1).standard_normal(P.n)
    ora = AlgMortarCPU(P.A, part)
    assert rel(cpu(h.apply(gpu(r))), ora.apply(r)) <= 1e-12
    h.close()


def test_setup_independent_of_host_threads(monkeypatch):
    """The host part of set-up (orderings, layout, boundary weights) runs on
    several threads; handles set up with 1 and with 16 give the same S^-1 and
    (with one pinned local-kernel layout) the same applies, bit for bit, on
    a bisection partition with RCM local orderings."""
    from oracle import partition_bisect
    from workloads.grids import distorted_hex_faces
    from workloads.tpfa import Faces, assemble
    nx, ny, nz = 30, 24, 10
    n = nx * ny * nz
    f = Faces.from_dict(distorted_hex_faces(nx, ny, nz, 0.3, 4, [(0, 0, 0.0)]))
    A, b = assemble(f, np.exp(np.random.default_rng(2).normal(size=n)), n)
    part, m = partition_bisect(A.row_ptr, A.col, A.val, n, 200, 800, 4)
    monkeypatch.setenv("ALGMORTAR_TILE", "0")
    r = gpu(np.random.default_rng(3).standard_normal(n))
    out = []
    for t in ("1", "16"):
        monkeypatch.setenv("ALGMORTAR_HOST_THREADS", t)
        h = am.AlgMortar(A, part, m)
        out.append((h.export_interface("Sinv"), cpu(h.apply(r))))
        h.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
