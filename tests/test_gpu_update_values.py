"""New values on an existing handle (algmortar_update_values), through the
C-ABI: the refreshed handle against one set up from scratch on the same
values (identical arithmetic, so bit for bit: applies, PCG solutions and
iteration counts, S^-1), for host and device values, on a Cartesian block
partition, a bisection partition with RCM local orderings and the 2-D case;
the refreshed handle against the FP64 oracle; the checks (the handle keeps
its values when one fails); a failed factorization blocks solves until a
good update; and the differentiation model reusing one handle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from paper_2607_22905_amd import AlgMortarError  # noqa: E402
from oracle import AlgMortarCPU, partition_blocks, partition_bisect  # noqa: E402
from workloads.fields import grf  # noqa: E402
from workloads.grids import cartesian_faces, distorted_hex_faces  # noqa: E402
from workloads.tpfa import Faces, assemble, CSR  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _pinned_layout(monkeypatch):
    # the same local-kernel wave layout on every handle (the autotuner's
    # choice decides the order in which partial vectors are added)
    monkeypatch.setenv("ALGMORTAR_TILE", "0")


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _family(name):
    """(faces, n, part, m, [A for three permeability fields]) on one grid."""
    if name == "blocks":
        nx, ny, nz = 24, 20, 16
        f = Faces.from_dict(cartesian_faces(nx, ny, nz, [(0, 0, 1.0), (0, 1, 0.0)]))
        part, m = partition_blocks((nx, ny, nz), (6, 5, 4))
        shape = (nz, ny, nx)
    elif name == "bisect":
        nx, ny, nz = 30, 24, 10
        f = Faces.from_dict(distorted_hex_faces(nx, ny, nz, 0.3, 4, [(0, 0, 0.0)]))
        shape = (nz, ny, nx)
        part = m = None
    else:  # 2-D
        nx, ny = 48, 40
        f = Faces.from_dict(cartesian_faces(nx, ny, 1, [(0, 0, 0.0)]))
        part, m = partition_blocks((nx, ny, 1), (12, 10, 1))
        shape = (ny, nx)
    n = int(np.prod(shape))
    mats = []
    for seed in (1, 2, 3):
        g = grf(shape, 3.0, 1.5, seed).ravel()
        A, _ = assemble(f, np.exp(g), n)
        mats.append(A)
    if part is None:
        part, m = partition_bisect(mats[0].row_ptr, mats[0].col, mats[0].val, n, 200, 800, 4)
    return f, n, part, m, mats


def with_values(A, val):
    return CSR(n=A.n, row_ptr=A.row_ptr, col=A.col, val=val)


@pytest.mark.parametrize("name", ["blocks", "bisect", "2d"])
def test_update_equals_fresh_setup(name):
    f, n, part, m, (A1, A2, A3) = _family(name)
    assert np.array_equal(A1.col, A2.col) and np.array_equal(A1.row_ptr, A2.row_ptr)
    h = am.AlgMortar(A1, part, m, max_nrhs=2)
    rng = np.random.default_rng(5)
    r = gpu(rng.standard_normal(n))
    R = gpu(rng.standard_normal((2, n)))
    b = gpu(rng.standard_normal(n))
    # host values, then device values
    for A, dev in ((A2, False), (A3, True)):
        h.update_values(with_values(A, gpu(A.val)) if dev else A)
        fresh = am.AlgMortar(A, part, m, max_nrhs=2)
        assert np.array_equal(cpu(h.apply(r)), cpu(fresh.apply(r)))
        assert np.array_equal(cpu(h.apply(R)), cpu(fresh.apply(R)))
        x1, i1, _ = h.pcg(b, 1e-10)
        x2, i2, _ = fresh.pcg(b, 1e-10)
        assert i1[0]["iterations"] == i2[0]["iterations"]
        assert np.array_equal(cpu(x1), cpu(x2))
        assert np.array_equal(h.export_interface("Sinv"), fresh.export_interface("Sinv"))
        fresh.close()
    # and against the oracle on the last values
    ora = AlgMortarCPU(A3, part)
    rr = rng.standard_normal(n)
    assert rel(cpu(h.apply(gpu(rr))), ora.apply(rr)) <= 1e-12
    h.close()


def test_update_checks_keep_the_handle():
    f, n, part, m, (A1, A2, _) = _family("blocks")
    h = am.AlgMortar(A1, part, m)
    r = gpu(np.random.default_rng(6).standard_normal(n))
    z0 = cpu(h.apply(r))
    rp, col = A2.row_ptr, A2.col
    row = np.repeat(np.arange(n), np.diff(rp))
    off = np.nonzero(col != row)[0]
    cross = off[part[row[off]] != part[col[off]]]
    inner = off[part[row[off]] == part[col[off]]]

    def expect(val, status):
        with pytest.raises(AlgMortarError) as e:
            h.update_values(with_values(A2, val))
        assert e.value.status_name == status, e.value
        assert np.array_equal(cpu(h.apply(r)), z0)  # previous values kept

    v = A2.val.copy()
    v[inner[3]] *= 1.5  # its transpose unchanged
    expect(v, "AM_ERR_NOT_SYMMETRIC")
    v = A2.val.copy()
    p = inner[7]
    q = np.nonzero((row == col[p]) & (col == row[p]))[0][0]
    v[p] = v[q] = 0.5
    expect(v, "AM_ERR_POSITIVE_COUPLING")
    v = A2.val.copy()
    v[np.nonzero(col == row)[0][4]] = np.nan  # on the diagonal: no transpose to disagree
    expect(v, "AM_ERR_ARG")
    v = A2.val.copy()
    p = cross[0]
    q = np.nonzero((row == col[p]) & (col == row[p]))[0][0]
    v[p] = v[q] = 0.0  # an interface coupling dropped
    expect(v, "AM_ERR_ARG")
    v = A2.val.copy()
    d = np.nonzero(col == row)[0][5]
    v[d] = -1.0
    expect(v, "AM_ERR_NOT_SPD")
    # a different pattern
    with pytest.raises(AlgMortarError) as e:
        h.update_values(CSR(n=n, row_ptr=rp, col=np.roll(col, 1), val=A2.val))
    assert e.value.status_name == "AM_ERR_ARG"
    # a smoother blocks updates until it is removed
    blocks, nb = partition_blocks((24, 20, 16), (12, 10, 16))
    h.set_smoother(blocks, nb, 1)
    with pytest.raises(AlgMortarError) as e:
        h.update_values(A2)
    assert e.value.status_name == "AM_ERR_UNSUPPORTED"
    h.set_smoother(blocks, nb, 0)
    h.update_values(A2)
    fresh = am.AlgMortar(A2, part, m)
    assert np.array_equal(cpu(h.apply(r)), cpu(fresh.apply(r)))
    fresh.close()
    h.close()


def test_failed_factorization_blocks_solves():
    """Diagonals scaled far down (still positive, so the checks pass) make the
    local operators indefinite: the update reports AM_ERR_NOT_SPD, solves
    refuse until a good update, which then matches a fresh set-up."""
    f, n, part, m, (A1, A2, _) = _family("blocks")
    h = am.AlgMortar(A1, part, m)
    row = np.repeat(np.arange(n), np.diff(A2.row_ptr))
    v = A2.val.copy()
    dg = A2.col == row
    v[dg] *= 1e-3
    with pytest.raises(AlgMortarError) as e:
        h.update_values(with_values(A2, v))
    assert e.value.status_name == "AM_ERR_NOT_SPD"
    r = gpu(np.random.default_rng(7).standard_normal(n))
    with pytest.raises(AlgMortarError) as e:
        h.apply(r)
    assert e.value.status_name == "AM_ERR_NOT_SPD"
    with pytest.raises(AlgMortarError):
        h.pcg(r, 1e-8)
    h.update_values(A2)
    fresh = am.AlgMortar(A2, part, m)
    assert np.array_equal(cpu(h.apply(r)), cpu(fresh.apply(r)))
    fresh.close()
    h.close()


def test_darcy_model_reusing_its_handle():
    """Gradients through the differentiation form with one reused handle
    equal those with a handle set up per solve, for three permeabilities."""
    nx, ny, nz = 16, 16, 12
    faces = Faces.from_dict(cartesian_faces(nx, ny, nz, [(0, 0, 1.0), (0, 1, 0.0)]))
    n = nx * ny * nz
    part, m = partition_blocks((nx, ny, nz), (8, 8, 6))
    obs = torch.as_tensor(np.random.default_rng(3).choice(n, 200, replace=False), device=DEV)
    models = [am.DarcyModel(faces, n, part, m, reuse_handle=reuse) for reuse in (False, True)]
    for seed in (11, 12, 13):
        lk = gpu(grf((nz, ny, nx), 3.0, 1.0, seed).ravel())
        grads = []
        for model in models:
            x = lk.clone().requires_grad_(True)
            p = am.AlgMortarSolve.apply(x, model)
            (p[obs] ** 2).sum().backward()
            grads.append(cpu(x.grad))
        assert np.array_equal(grads[0], grads[1])
    for model in models:
        model.close()


def test_darcy_model_two_forwards_then_backward():
    """Two forward solves on a model that reuses its handle, then the first
    forward's backward: the handle holds the second permeability by then, so
    the backward must put the first one's values back.  The gradients equal
    those of a model with a handle per solve."""
    nx, ny, nz = 16, 16, 12
    faces = Faces.from_dict(cartesian_faces(nx, ny, nz, [(0, 0, 1.0), (0, 1, 0.0)]))
    n = nx * ny * nz
    part, m = partition_blocks((nx, ny, nz), (8, 8, 6))
    obs = torch.as_tensor(np.random.default_rng(4).choice(n, 200, replace=False), device=DEV)
    lks = [gpu(grf((nz, ny, nx), 3.0, 1.0, seed).ravel()) for seed in (21, 22)]
    grads = {}
    for reuse in (False, True):
        model = am.DarcyModel(faces, n, part, m, reuse_handle=reuse)
        xs = [lk.clone().requires_grad_(True) for lk in lks]
        ps = [am.AlgMortarSolve.apply(x, model) for x in xs]  # both forwards first
        (ps[0][obs] ** 2).sum().backward()                      # then the first backward
        (ps[1][obs] ** 2).sum().backward()
        grads[reuse] = [cpu(x.grad) for x in xs]
        model.close()
    for k in range(2):
        assert np.array_equal(grads[False][k], grads[True][k])
    # and the two permeabilities give different gradients (the test would not
    # see a handle that kept the wrong values otherwise)
    assert not np.allclose(grads[True][0], grads[True][1])
