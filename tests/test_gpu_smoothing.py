"""Block-Jacobi pre/post smoothing around AlgMortar (Sec. 5.4) on the GPU,
through the C-ABI, against the FP64 oracle: the smoothed apply to 1e-11
relative L2 (nu + 1 chained residual/solve steps on top of the apply's
1e-12), the smoothed PCG solution to 1e-8 at tolerance 1e-10 with the
iteration count within one, removal of the smoother, the one-block case that
reduces to a direct solve, several right-hand sides, and the error paths."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from paper_2607_22905_amd import AlgMortarError  # noqa: E402
from oracle import AlgMortarCPU, partition_blocks, pcg  # noqa: E402
from oracle.smoothing import SmoothedAlgMortarCPU  # noqa: E402
from workloads import make_config  # noqa: E402
from tests._problems import random_3d  # noqa: E402

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _case(name):
    """(A, b, AlgMortar partition, smoothing blocks) -- blocks are unions of
    subdomains whose bandwidth in ascending index order fits the band kernels:
    layered 32^3 with 8^3 subdomains and 8 x 8 x 32 blocks (2048 rows, window
    64); a ragged 18 x 15 x 8 grid with 6 x 5 x 4 subdomains and 6 x 15 x 8
    blocks (720 rows, window 128); the 64 x 64 2-D case with 16 x 16
    subdomains and 32 x 32 blocks."""
    if name == "layered":
        P = make_config("c2", nx=32, ny=32, nz=32)
        blk = (8, 8, 32)
    elif name == "ragged3d":
        P = random_3d(18, 15, 8, 1.5, 11, block=(6, 5, 4))
        blk = (6, 15, 8)
    elif name == "c1":
        P = make_config("c1")
        blk = (32, 32, 1)
    else:
        raise KeyError(name)
    part, m = partition_blocks(P.dims, P.partition[1])
    blocks, nb = partition_blocks(P.dims, blk)
    return P, part, m, blocks, nb


_cache = {}


def setup(name):
    if name not in _cache:
        P, part, m, blocks, nb = _case(name)
        _cache[name] = (P, part, m, blocks, nb, AlgMortarCPU(P.A, part))
    return _cache[name]


@pytest.mark.parametrize("name", ["layered", "ragged3d", "c1"])
@pytest.mark.parametrize("nu", [1, 3])
def test_smoothed_apply_matches_oracle(name, nu):
    P, part, m, blocks, nb, ora = setup(name)
    h = am.AlgMortar(P.A, part, m)
    h.set_smoother(blocks, nb, nu)
    r = np.random.default_rng(10 + nu).standard_normal(P.n)
    z = cpu(h.apply(gpu(r)))
    zo = SmoothedAlgMortarCPU(ora, blocks, nu).apply(r)
    assert rel(z, zo) <= 1e-11, rel(z, zo)
    h.close()


def test_smoothed_apply_several_rhs():
    P, part, m, blocks, nb, ora = setup("ragged3d")
    h = am.AlgMortar(P.A, part, m, max_nrhs=4)
    h.set_smoother(blocks, nb, 2)
    R = np.random.default_rng(3).standard_normal((3, P.n))  # rows = right-hand sides
    Z = cpu(h.apply(gpu(R)))
    so = SmoothedAlgMortarCPU(ora, blocks, 2)
    for k in range(3):
        zo = so.apply(R[k])
        assert rel(Z[k], zo) <= 1e-11
    h.close()


def test_zero_steps_removes_the_smoother():
    P, part, m, blocks, nb, ora = setup("layered")
    r = gpu(np.random.default_rng(4).standard_normal(P.n))
    h = am.AlgMortar(P.A, part, m)
    z0 = cpu(h.apply(r))
    h.set_smoother(blocks, nb, 2)
    z2 = cpu(h.apply(r))
    assert rel(z2, z0) > 1e-6  # the smoother changes the result
    h.set_smoother(blocks, nb, 0)
    assert np.array_equal(cpu(h.apply(r)), z0)
    h.close()


def test_one_block_is_a_direct_solve():
    """One block holding every unknown (64 x 64 grid, bandwidth 64): each
    smoothing step is an exact solve, so the apply returns A^{-1} r."""
    P, part, m, _, _, ora = setup("c1")
    h = am.AlgMortar(P.A, part, m)
    h.set_smoother(np.zeros(P.n, dtype=np.int32), 1, 1)
    r = np.random.default_rng(5).standard_normal(P.n)
    z = cpu(h.apply(gpu(r)))
    x = spla.spsolve(ora.As.tocsc(), r)
    assert rel(z, x) <= 1e-10
    h.close()


@pytest.mark.parametrize("name", ["layered", "ragged3d"])
def test_smoothed_pcg_matches_oracle(name):
    P, part, m, blocks, nb, ora = setup(name)
    nu = 2
    h = am.AlgMortar(P.A, part, m)
    h.set_smoother(blocks, nb, nu)
    x, info, _ = h.pcg(gpu(P.b), 1e-10)
    x = cpu(x)
    so = SmoothedAlgMortarCPU(ora, blocks, nu)
    As = ora.As
    res = pcg(lambda v: As @ v, P.b, so.apply, 1e-10)
    its0 = pcg(lambda v: As @ v, P.b, ora.apply, 1e-10).iterations
    assert info[0]["converged"] == 1
    assert abs(info[0]["iterations"] - res.iterations) <= 1
    assert res.iterations < its0
    assert info[0]["true_rel_res"] <= 1e-9
    assert rel(x, res.x) <= 1e-8
    h.close()


def test_smoothed_pcg_fp32_factors():
    P, part, m, blocks, nb, ora = setup("layered")
    h = am.AlgMortar(P.A, part, m, prec="fp32")
    h.set_smoother(blocks, nb, 2)
    x, info, _ = h.pcg(gpu(P.b), 1e-10)
    assert info[0]["converged"] == 1 and info[0]["true_rel_res"] <= 2e-10
    xo = pcg(lambda v: ora.As @ v, P.b, ora.apply, 1e-12).x
    assert rel(cpu(x), xo) <= 1e-8
    h.close()


def test_smoother_errors():
    P, part, m, blocks, nb, ora = setup("layered")
    h = am.AlgMortar(P.A, part, m)
    with pytest.raises(AlgMortarError) as e:
        h.set_smoother(blocks, nb, -1)
    assert e.value.status_name == "AM_ERR_ARG"
    bad = blocks.copy()
    bad[bad == 3] = 2  # block 3 left empty
    with pytest.raises(AlgMortarError) as e:
        h.set_smoother(bad, nb, 1)
    assert e.value.status_name == "AM_ERR_ARG"
    # one block over the whole 32^3 grid: bandwidth 1024 in index order
    with pytest.raises(AlgMortarError) as e:
        h.set_smoother(np.zeros(P.n, dtype=np.int32), 1, 1)
    assert e.value.status_name == "AM_ERR_UNSUPPORTED"
    # the handle still works without a smoother
    r = gpu(np.random.default_rng(6).standard_normal(P.n))
    assert rel(cpu(h.apply(r)), ora.apply(cpu(r))) <= 1e-12
    h.set_smoother(blocks, nb, 1)
    with pytest.raises(AlgMortarError) as e:
        h.pcg_profile(gpu(P.b), 1e-10)
    assert e.value.status_name == "AM_ERR_UNSUPPORTED"
    h.close()


def test_smoothed_pcg_several_rhs_and_replacement():
    """Smoothed PCG on 3 right-hand sides solved together (each column against
    its own oracle solve), after replacing a first smoother by another."""
    P, part, m, blocks, nb, ora = setup("ragged3d")
    h = am.AlgMortar(P.A, part, m, max_nrhs=4)
    other, no = partition_blocks(P.dims, (6, 15, 4))
    h.set_smoother(other, no, 1)
    h.set_smoother(blocks, nb, 2)
    rng = np.random.default_rng(9)
    B = rng.standard_normal((3, P.n))
    X, info, _ = h.pcg(gpu(B), 1e-10)
    X = cpu(X)
    so = SmoothedAlgMortarCPU(ora, blocks, 2)
    As = ora.As
    for k in range(3):
        res = pcg(lambda v: As @ v, B[k], so.apply, 1e-10)
        assert info[k]["converged"] == 1
        assert abs(info[k]["iterations"] - res.iterations) <= 1
        assert rel(X[k], res.x) <= 1e-8
    h.close()


def test_smoothed_cross_field_bf16_factors():
    """Smoothing on the cross-shaped kappa = 1e6 field with BF16 factors
    (flexible outer PCG): converges to the oracle's solution.  The field's
    contrast makes A ill conditioned (a 1e-10 residual leaves errors near
    3e-8), so both sides solve to 1e-12."""
    P = make_config("c6", nx=32, ny=32, nz=32)
    part, m = partition_blocks(P.dims, P.partition[1])
    blocks, nb = partition_blocks(P.dims, (8, 8, 16))
    h = am.AlgMortar(P.A, part, m, prec="bf16")
    h.set_smoother(blocks, nb, 1)
    x, info, _ = h.pcg(gpu(P.b), 1e-12)
    assert info[0]["converged"] == 1 and info[0]["true_rel_res"] <= 2e-12
    ora = AlgMortarCPU(P.A, part)
    xo = pcg(lambda v: ora.As @ v, P.b, ora.apply, 1e-12).x
    assert rel(cpu(x), xo) <= 1e-8
    h.close()
