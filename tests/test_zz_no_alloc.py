"""The allocation-free apply (algmortar_apply_static), through the C-ABI:
its result equals algmortar_apply's bit for bit (same kernels, work buffers
in the library's static device scratch instead of the handle's memory), on
two calls in a row of which the second has the smaller input, with a fused
and a separate interface solve and a padded right-hand-side block; a handle
and nrhs whose work buffers exceed the static scratch are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from paper_2607_22905_amd import AlgMortarError  # noqa: E402
from oracle import partition_blocks  # noqa: E402
from tests._problems import random_3d  # noqa: E402

DEV = "cuda:0"


def _handle(dims, block, seed, separate=False, max_nrhs=1):
    P = random_3d(*dims, sigma=1.5, seed=seed, block=block)
    part, m = partition_blocks(P.dims, P.partition[1])
    return P, am.AlgMortar(P.A, part, m, separate_iface=separate, max_nrhs=max_nrhs)


@pytest.mark.parametrize("separate", [False, True])
def test_static_apply_equals_apply_larger_then_smaller(separate):
    cases = [((32, 32, 24), (8, 8, 8), 31), ((16, 16, 8), (8, 8, 4), 32)]  # second smaller
    for dims, block, seed in cases:
        P, h = _handle(dims, block, seed, separate)
        r = torch.as_tensor(np.random.default_rng(seed).standard_normal(P.n), device=DEV)
        z_static = h.apply_static(r)
        z = h.apply(r)
        torch.cuda.synchronize()
        assert torch.equal(z_static, z), dims
        assert torch.isfinite(z).all()
        h.close()


def test_static_apply_padded_columns():
    """Three right-hand sides in a block of four: the padding column comes
    from the scratch and must not reach the outputs (and a second call with
    one column on a smaller handle follows)."""
    P, h = _handle((24, 24, 16), (8, 8, 8), 33, max_nrhs=4)
    R = torch.as_tensor(np.random.default_rng(5).standard_normal((3, P.n)), device=DEV)
    Zs = h.apply_static(R)
    Z = h.apply(R)
    torch.cuda.synchronize()
    assert torch.equal(Zs, Z)
    h.close()
    P2, h2 = _handle((16, 8, 8), (8, 8, 8), 34)
    r = torch.as_tensor(np.random.default_rng(6).standard_normal(P2.n), device=DEV)
    assert torch.equal(h2.apply_static(r), h2.apply(r))
    h2.close()


def test_static_apply_refuses_what_exceeds_the_scratch():
    P, h = _handle((64, 64, 64), (8, 8, 8), 35, max_nrhs=16)
    R = torch.zeros((16, P.n), dtype=torch.float64, device=DEV)
    with pytest.raises(AlgMortarError) as ei:
        h.apply_static(R)
    assert ei.value.status_name == "AM_ERR_ARG"
    # the handle still works, also through the static form with one column
    r = torch.as_tensor(np.random.default_rng(7).standard_normal(P.n), device=DEV)
    assert torch.equal(h.apply_static(r), h.apply(r))
    h.close()
