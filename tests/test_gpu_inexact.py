"""The inexact interface solve (AM_FLAG_INEXACT_IFACE: block-Jacobi PCG on S
to a relative tolerance, Sec. 6 and Sec. 7) through the C-ABI, against the
oracle's InexactAlgMortarCPU with the same blocks (64 consecutive basis
functions), tolerance and iteration cap.

* A fixed number of inner iterations (rtol 0): the inner PCG is then the same
  sequence of operations on both sides, so applies agree to 1e-12 (1, 3 and
  16 right-hand sides).
* rtol 1e-2, the paper's setting: the outer PCG with the flexible beta
  reaches tol 1e-10, its solution within 1e-8 of the oracle's (flexible PCG
  with the oracle's inexact preconditioner) and of the exact preconditioner's
  solution, with the outer iteration count within two of the oracle's (an
  inner stop can fall one iteration apart when a residual sits at the
  tolerance)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from paper_2607_22905_amd import AlgMortarError  # noqa: E402
from oracle import pcg  # noqa: E402
from oracle.inexact import InexactAlgMortarCPU  # noqa: E402
from tests.test_gpu_parity import rel, gpu, cpu, setup_case  # noqa: E402
from tests.test_gpu_interface_nd import _get  # noqa: E402


@pytest.mark.parametrize("name,maxit", [("c1", 3), ("layered", 5), ("bisect", 4), ("grf64", 6)])
def test_fixed_inner_iterations_apply(name, maxit):
    A, part, m, b, ora = _get(name)
    inx = InexactAlgMortarCPU(ora, rtol=0.0, maxit=maxit, block_rows=64)
    h = am.AlgMortar(A, part, m, inexact_iface=True, max_nrhs=16)
    h.set_inexact(0.0, maxit)
    rng = np.random.default_rng(maxit)
    r = rng.standard_normal(A.n)
    assert rel(cpu(h.apply(gpu(r))), inx.apply(r)) <= 1e-12
    for ncol in (3, 16):
        R = rng.standard_normal((ncol, A.n))
        Z = cpu(h.apply(gpu(R)))
        for k in sorted({0, ncol // 2, ncol - 1}):
            assert rel(Z[k], inx.apply(R[k])) <= 1e-12, (ncol, k)
    h.close()


@pytest.mark.parametrize("name", ["c1", "layered", "grf64"])
def test_tolerance_1e2_flexible_pcg(name):
    A, part, m, b, ora = _get(name)
    As = A.to_scipy()
    inx = InexactAlgMortarCPU(ora, rtol=1e-2, maxit=50, block_rows=64)
    ref = pcg(lambda v: As @ v, b, inx.apply, 1e-10, beta="pr")
    exact = pcg(lambda v: As @ v, b, ora.apply, 1e-10)
    h = am.AlgMortar(A, part, m, inexact_iface=True)
    x, info, _ = h.pcg(gpu(b), 1e-10)
    x = cpu(x)
    print(f"{name}: outer iterations {info[0]['iterations']} (oracle {ref.iterations}, exact "
          f"interface solve {exact.iterations})")
    assert info[0]["converged"] == 1
    assert abs(info[0]["iterations"] - ref.iterations) <= 2
    assert np.linalg.norm(b - As @ x) / np.linalg.norm(b) <= 2e-10
    assert rel(x, ref.x) <= 1e-8 and rel(x, exact.x) <= 1e-8
    h.close()


def test_set_inexact_checks():
    A, part, m, b, ora = setup_case("c1")
    h = am.AlgMortar(A, part, m)
    with pytest.raises(AlgMortarError):
        h.set_inexact(1e-2, 10)  # not an inexact handle
    h.close()
    h = am.AlgMortar(A, part, m, inexact_iface=True)
    for bad in ((1.5, 10), (-1.0, 10), (1e-2, 0), (1e-2, 5000)):
        with pytest.raises(AlgMortarError):
            h.set_inexact(*bad)
    with pytest.raises(AlgMortarError):
        h.apply_static(gpu(b))
    h.close()
