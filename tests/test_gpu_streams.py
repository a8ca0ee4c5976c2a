"""Stream ordering at the C-ABI: the set-up, value update, PCG and adjoint
calls run on the library's own (non-blocking) stream, so they must first wait
for the caller's stream -- here torch's default stream, which the binding
passes as the null stream -- or they would read inputs that queued kernels
are still writing.  Each test queues a long chain of products on the default
stream that the input depends on, calls the library at once, and compares
with the same call made after an explicit synchronization."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from oracle import partition_blocks  # noqa: E402
from tests._problems import random_3d  # noqa: E402
from workloads.fields import grf  # noqa: E402
from workloads.grids import cartesian_faces  # noqa: E402
from workloads.tpfa import Faces  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _pinned_layout(monkeypatch):
    monkeypatch.setenv("ALGMORTAR_TILE", "0")


def _late(x):
    """x, written on the default stream behind some 20 ms of queued work (a
    fresh buffer that holds zeros until then)."""
    assert torch.cuda.current_stream().cuda_stream == 0
    big = torch.rand(4096, 4096, device=DEV) / 4096.0
    torch.cuda.synchronize()
    y = big
    for _ in range(24):
        y = torch.tanh(y @ big)  # bounded: 0 * y stays 0
    out = torch.zeros_like(x)
    out.copy_(x + 0.0 * y[0, 0].double())
    return out  # no synchronization: the copy is still queued


def test_pcg_waits_for_the_default_stream():
    P = random_3d(16, 16, 12, sigma=1.5, seed=5, block=(8, 8, 6))
    part, m = partition_blocks(P.dims, P.partition[1])
    h = am.AlgMortar(P.A, part, m)
    b = torch.as_tensor(P.b, dtype=torch.float64, device=DEV)
    x_ref, info_ref, _ = h.pcg(b, 1e-10)
    torch.cuda.synchronize()
    x, info, _ = h.pcg(_late(b), 1e-10)
    torch.cuda.synchronize()
    assert info[0]["iterations"] == info_ref[0]["iterations"] > 0
    assert torch.equal(x, x_ref)
    h.close()


def test_setup_and_update_wait_for_the_default_stream():
    P = random_3d(16, 16, 12, sigma=1.5, seed=6, block=(8, 8, 6))
    part, m = partition_blocks(P.dims, P.partition[1])
    r = torch.as_tensor(np.random.default_rng(1).standard_normal(P.n), device=DEV)
    href = am.AlgMortar(P.A, part, m)
    zref = href.apply(r)
    torch.cuda.synchronize()
    val = torch.as_tensor(P.A.val, dtype=torch.float64, device=DEV)

    class View:
        n, row_ptr, col = P.A.n, P.A.row_ptr, P.A.col

    View.val = _late(val)
    h = am.AlgMortar(View, part, m)  # device values still being written
    assert torch.equal(h.apply(r), zref)
    # new values on the handle, again still queued (twice the matrix: the
    # preconditioner of 2A applied to r is half that of A, exactly)
    View.val = _late(2.0 * val)
    h.update_values(View)
    z2 = h.apply(r)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(2.0 * z2 - zref) / torch.linalg.norm(zref)) <= 1e-12
    h.close()
    href.close()


def test_adjoint_waits_for_the_default_stream():
    nx, ny, nz = 16, 16, 12
    faces = Faces.from_dict(cartesian_faces(nx, ny, nz, [(0, 0, 1.0), (0, 1, 0.0)]))
    n = nx * ny * nz
    part, m = partition_blocks((nx, ny, nz), (8, 8, 6))
    lk = torch.as_tensor(grf((nz, ny, nx), 3.0, 1.0, 8).ravel(), device=DEV)
    model = am.DarcyModel(faces, n, part, m)
    p, h = model.forward_solve(lk)
    dJ = torch.as_tensor(np.random.default_rng(2).standard_normal(n), device=DEV)
    g_ref, _, _ = am.adjoint_grad(h, model.tpfa, lk, p, dJ, tol=1e-12)
    torch.cuda.synchronize()
    g, _, _ = am.adjoint_grad(h, model.tpfa, lk, p, _late(dJ), tol=1e-12)
    torch.cuda.synchronize()
    assert torch.equal(g, g_ref)
    h.close()
    model.close()
