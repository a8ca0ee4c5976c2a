"""The second workload family on the GPU, through the C-ABI, against the FP64
oracle: the periodic high-contrast cross pattern (kappa = 1e6 channels, p
fixed on the y faces) and the contrast sweep K -> K^theta on the layered
field.  Bars as for the other workloads: apply within 1e-12 relative L2, PCG
at tolerance 1e-10 within 1e-8 with the iteration count within one."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from oracle import AlgMortarCPU, partition_blocks, pcg  # noqa: E402
from workloads import make_config  # noqa: E402

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = {
    "cross32": lambda: make_config("c6", nx=32, ny=32, nz=32),
    "cross24x40x16": lambda: make_config("c6", nx=24, ny=40, nz=16),
    "layered32_theta0.6": lambda: make_config("c2", nx=32, ny=32, nz=32, theta=0.6),
    "layered32_theta1.4": lambda: make_config("c2", nx=32, ny=32, nz=32, theta=1.4),
    "cross32_theta1.4": lambda: make_config("c6", nx=32, ny=32, nz=32, theta=1.4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_apply_and_pcg_match_oracle(name):
    P = CASES[name]()
    part, m = partition_blocks(P.dims, P.partition[1])
    ora = AlgMortarCPU(P.A, part)
    h = am.AlgMortar(P.A, part, m)
    r = np.random.default_rng(7).standard_normal(P.n)
    assert rel(cpu(h.apply(gpu(r))), ora.apply(r)) <= 1e-12
    x, info, _ = h.pcg(gpu(P.b), 1e-10)
    As = ora.As
    res = pcg(lambda v: As @ v, P.b, ora.apply, 1e-10)
    assert info[0]["converged"] == 1
    assert abs(info[0]["iterations"] - res.iterations) <= 1
    assert info[0]["true_rel_res"] <= 1e-9
    assert rel(cpu(x), res.x) <= 1e-8
    h.close()
