"""Pins for the oracle's inexact interface solve (Sec. 6 option: PCG with
block Jacobi on S, stopped at a relative residual; Sec. 7 uses 1e-2).

Checked against what the definitions fix, not against the oracle's own
arithmetic: a tiny tolerance reproduces the exact apply; one block holding
every basis function makes block Jacobi the exact inverse, so the inner PCG
stops after one iteration with the exact apply; one-row blocks are point
Jacobi (division by the diagonal of S); every inner solve meets its stopping
rule and the iteration before it does not; and the outer flexible PCG with
the inexact preconditioner reaches the direct solution of A x = b."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import AlgMortarCPU, partition_blocks, pcg
from oracle.inexact import BlockJacobiS, InexactAlgMortarCPU
from tests._problems import random_2d, random_3d
from workloads import make_config


def _case(k):
    if k == 0:
        P = make_config("c1")
    elif k == 1:
        P = random_3d(16, 16, 12, 1.5, 3, block=(4, 4, 4))
    else:
        P = make_config("c2", nx=24, ny=24, nz=16)
    part, _ = partition_blocks(P.dims, P.partition[1])
    return P, AlgMortarCPU(P.A, part)


@pytest.fixture(params=[0, 1, 2], scope="module")
def case(request):
    return _case(request.param)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_tiny_tolerance_is_the_exact_apply(case):
    P, ora = case
    inx = InexactAlgMortarCPU(ora, rtol=1e-14, maxit=2000, block_rows=16)
    r = np.random.default_rng(1).standard_normal(P.n)
    assert _rel(inx.apply(r), ora.apply(r)) <= 1e-11


def test_one_block_is_an_exact_inner_solve(case):
    P, ora = case
    inx = InexactAlgMortarCPU(ora, rtol=1e-2, maxit=50, block_rows=ora.S.shape[0])
    r = np.random.default_rng(2).standard_normal(P.n)
    z = inx.apply(r)
    assert inx.inner_iterations == [1]
    assert _rel(z, ora.apply(r)) <= 1e-12


def test_one_row_blocks_are_point_jacobi(case):
    P, ora = case
    bj = BlockJacobiS(ora.S, 1)
    v = np.random.default_rng(3).standard_normal(ora.S.shape[0])
    assert np.allclose(bj(v), v / ora.S.diagonal(), rtol=1e-15, atol=0)


def test_inner_solves_meet_their_stopping_rule(case):
    P, ora = case
    inx = InexactAlgMortarCPU(ora, rtol=1e-2, maxit=200, block_rows=16)
    r = np.random.default_rng(4).standard_normal(P.n)
    b = ora.interface_rhs(ora.local_solves(r))
    eta = inx.solve_S(b)
    k = inx.inner_iterations[-1]
    assert k >= 1
    assert np.linalg.norm(b - ora.S @ eta) <= 1.001e-2 * np.linalg.norm(b)
    # the iteration before does not meet it (a stop by the rule, not by maxit)
    prev = InexactAlgMortarCPU(ora, rtol=0.0, maxit=k - 1, block_rows=16)
    eta_prev = prev.solve_S(b) if k > 1 else np.zeros_like(b)
    assert np.linalg.norm(b - ora.S @ eta_prev) > 0.999e-2 * np.linalg.norm(b)


def test_flexible_pcg_reaches_the_direct_solution(case):
    P, ora = case
    inx = InexactAlgMortarCPU(ora, rtol=1e-2, maxit=200, block_rows=16)
    As = P.A.to_scipy().tocsc()
    xd = spla.spsolve(As, P.b)
    res = pcg(lambda v: As @ v, P.b, inx.apply, 1e-10, beta="pr")
    assert res.converged
    assert _rel(res.x, xd) <= 1e-7
    assert res.true_rel_res <= 2e-10
