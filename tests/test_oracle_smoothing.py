"""Pins for the oracle's block-Jacobi smoothing around AlgMortar (Sec. 5.4).

Checked against what the definitions and linear algebra fix, not against the
oracle's own arithmetic: zero steps give AlgMortar itself; one block holding
every unknown makes each smoothing step an exact solve (a direct solve of A);
one-cell blocks are point Jacobi (division by the diagonal); blocks solved by
a dense library solve; the composition with equal pre- and post-steps is
symmetric and positive definite, while unequal counts are not symmetric; and
since AlgMortar's spectrum relative to A lies in (0, 1] (Sec. 5.2) and block
Jacobi is an A-norm contraction for a diagonally dominant M-matrix, the
smoothed spectrum lies in (0, 1] with a smallest eigenvalue no lower than
AlgMortar's.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import AlgMortarCPU, partition_blocks, pcg
from oracle.smoothing import BlockJacobi, SmoothedAlgMortarCPU, smoothed_apply
from tests._problems import random_2d, random_3d


def _case(k):
    if k == 0:
        P = random_3d(8, 8, 4, 1.5, 5, block=(4, 4, 2))
        blocks, _ = partition_blocks(P.dims, (8, 4, 2))
    elif k == 1:
        P = random_2d(12, 12, 2.0, 6, block=(4, 4, 1))
        blocks, _ = partition_blocks(P.dims, (12, 4, 1))
    else:
        P = random_3d(6, 6, 6, 1.0, 7, block=(3, 3, 3))
        blocks, _ = partition_blocks(P.dims, (6, 3, 6))
    part, _ = partition_blocks(P.dims, P.partition[1])
    return P, AlgMortarCPU(P.A, part), blocks


@pytest.fixture(params=[0, 1, 2])
def case(request):
    return _case(request.param)


def _dense_inv(op, n):
    return np.stack([op(e) for e in np.eye(n)], axis=1)


def test_zero_steps_is_algmortar(case):
    P, am, blocks = case
    r = np.random.default_rng(1).standard_normal(P.n)
    sm = SmoothedAlgMortarCPU(am, blocks, 0)
    assert np.array_equal(sm.apply(r), am.apply(r))


@pytest.mark.parametrize("nu", [1, 3])
def test_one_block_is_a_direct_solve(case, nu):
    P, am, _ = case
    r = np.random.default_rng(2).standard_normal(P.n)
    z = SmoothedAlgMortarCPU(am, np.zeros(P.n, dtype=np.int64), nu).apply(r)
    x = spla.spsolve(am.As.tocsc(), r)
    assert np.linalg.norm(z - x) <= 1e-10 * np.linalg.norm(x)


def test_point_blocks_are_jacobi(case):
    P, am, _ = case
    r = np.random.default_rng(3).standard_normal(P.n)
    bj = BlockJacobi(am.As, np.arange(P.n))
    d = am.As.diagonal()
    assert np.allclose(bj.solve(r), r / d, rtol=1e-15, atol=0)


def test_block_solves_match_dense_solves(case):
    P, am, blocks = case
    r = np.random.default_rng(4).standard_normal(P.n)
    x = BlockJacobi(am.As, blocks).solve(r)
    Ad = am.As.toarray()
    for b in np.unique(blocks):
        ix = np.flatnonzero(blocks == b)
        xb = np.linalg.solve(Ad[np.ix_(ix, ix)], r[ix])
        assert np.allclose(x[ix], xb, rtol=1e-12, atol=1e-14 * abs(xb).max())


@pytest.mark.parametrize("nu", [1, 2])
def test_symmetric_and_linear(case, nu):
    P, am, blocks = case
    sm = SmoothedAlgMortarCPU(am, blocks, nu)
    rng = np.random.default_rng(5)
    u, v = rng.standard_normal(P.n), rng.standard_normal(P.n)
    Mu, Mv = sm.apply(u), sm.apply(v)
    assert abs(u @ Mv - v @ Mu) <= 1e-12 * abs(u @ Mv)
    assert np.allclose(sm.apply(2.0 * u - 3.0 * v), 2.0 * Mu - 3.0 * Mv, rtol=1e-12,
                       atol=1e-12 * abs(Mu).max())
    # unequal pre- and post-steps break the symmetry the pin relies on
    def lopsided(r):
        z = np.zeros_like(r)
        z = z + sm.bj.solve(r - am.As @ z)
        return z + am.apply(r - am.As @ z)
    a, b = u @ lopsided(v), v @ lopsided(u)
    assert abs(a - b) > 1e-6 * abs(a)


@pytest.mark.parametrize("nu", [1, 2])
def test_spectrum_in_unit_interval(case, nu):
    P, am, blocks = case
    n = P.n
    Ad = am.As.toarray()
    Ms = _dense_inv(SmoothedAlgMortarCPU(am, blocks, nu).apply, n)
    Mam = _dense_inv(am.apply, n)
    assert np.allclose(Ms, Ms.T, atol=1e-11 * abs(Ms).max())
    assert sla.eigh(0.5 * (Ms + Ms.T), eigvals_only=True)[0] > 0
    th_s = np.sort(np.linalg.eigvals(Ms @ Ad).real)
    th_a = np.sort(np.linalg.eigvals(Mam @ Ad).real)
    assert th_s.max() <= 1.0 + 1e-9
    assert th_s.min() > 0
    assert th_s.min() >= th_a.min() - 1e-10


def test_smoothing_reduces_pcg_iterations():
    P, am, blocks = _case(0)
    A = am.As
    its0 = pcg(lambda v: A @ v, P.b, am.apply, 1e-10).iterations
    sm = SmoothedAlgMortarCPU(am, blocks, 2)
    res = pcg(lambda v: A @ v, P.b, sm.apply, 1e-10)
    assert res.converged and res.true_rel_res <= 1e-9
    assert res.iterations < its0


def test_multi_column_apply_is_columnwise(case):
    P, am, blocks = case
    sm = SmoothedAlgMortarCPU(am, blocks, 1)
    R = np.random.default_rng(6).standard_normal((P.n, 3))
    Z = sm.apply(R)
    for k in range(3):
        assert np.array_equal(Z[:, k], sm.apply(R[:, k]))
