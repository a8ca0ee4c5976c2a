"""Pins for the oracle's PCG and adjoint gradient."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import AlgMortarCPU, partition_blocks, pcg, adjoint, dense
from workloads import make_config
from workloads.tpfa import assemble
from tests._problems import random_2d, random_3d


def test_pcg_matches_direct_solve_c1():
    P = make_config("c1")
    part, _ = partition_blocks(P.dims, P.partition[1])
    pre = AlgMortarCPU(P.A, part)
    As = P.A.to_scipy()
    res = pcg(lambda v: As @ v, P.b, pre.apply, 1e-10)
    xd = spla.spsolve(As.tocsc(), P.b)
    assert res.converged and res.true_rel_res < 1e-9
    assert np.linalg.norm(res.x - xd) <= 1e-8 * np.linalg.norm(xd)
    # AlgMortar beats Jacobi by a wide margin on this problem
    jac = pcg(lambda v: As @ v, P.b, lambda r: r / As.diagonal(), 1e-10)
    assert res.iterations * 4 < jac.iterations


def test_pcg_exact_preconditioner_one_iteration():
    P = random_3d(6, 6, 4, 1.0, 1, block=(3, 3, 2))
    part, _ = partition_blocks(P.dims, P.partition[1])
    As = P.A.to_scipy()
    for mortar, p in (("edge", part), ("interface", np.zeros(P.n, dtype=np.int32))):
        pre = AlgMortarCPU(P.A, p, mortar)
        res = pcg(lambda v: As @ v, P.b, pre.apply, 1e-10)
        assert res.iterations == 1


def test_pcg_plain_cg_identity():
    """With the identity preconditioner PCG is CG; compare with a dense solve
    (an SPD system of 48 unknowns converges within 48 steps in exact
    arithmetic)."""
    P = random_3d(4, 4, 3, 0.5, 2, block=(2, 2, 3))
    As = P.A.to_scipy()
    res = pcg(lambda v: As @ v, P.b, lambda r: r.copy(), 1e-12, maxit=500)
    assert res.converged
    assert np.allclose(res.x, np.linalg.solve(dense.to_dense(P.A), P.b), rtol=1e-9)


def test_pcg_polak_ribiere_matches_fletcher_reeves_for_symmetric_precond():
    P = random_2d(16, 16, 1.0, 3, block=(4, 4, 1))
    part, _ = partition_blocks(P.dims, P.partition[1])
    pre = AlgMortarCPU(P.A, part)
    As = P.A.to_scipy()
    a = pcg(lambda v: As @ v, P.b, pre.apply, 1e-10)
    b = pcg(lambda v: As @ v, P.b, pre.apply, 1e-10, beta="pr")
    assert abs(a.iterations - b.iterations) <= 1
    assert np.allclose(a.x, b.x, rtol=1e-8)


def _solve(A, b):
    return spla.spsolve(A.to_scipy().tocsc(), b)


@pytest.mark.parametrize("mk", [lambda: random_2d(10, 8, 1.0, 4, block=(5, 4, 1)),
                                lambda: random_3d(6, 5, 4, 1.5, 5, block=(3, 5, 2))])
def test_adjoint_gradient_matches_central_differences(mk):
    P = mk()
    rng = np.random.default_rng(12)
    obs = np.sort(rng.choice(P.n, size=P.n // 3, replace=False))
    pobs = rng.standard_normal(obs.size) * 0.1

    def J(logK):
        A, f = assemble(P.faces, np.exp(logK), P.n)
        return adjoint.loss(_solve(A, f), obs, pobs)

    A, f = assemble(P.faces, np.exp(P.logK), P.n)
    p = _solve(A, f)
    lam = _solve(A, adjoint.dloss_dp(p, obs, pobs))
    g = adjoint.gradient(P.faces, P.logK, p, lam)
    h = 1e-5
    for c in rng.choice(P.n, size=8, replace=False):
        e = np.zeros(P.n)
        e[c] = h
        fd = (J(P.logK + e) - J(P.logK - e)) / (2 * h)
        assert abs(fd - g[c]) <= 1e-6 * max(abs(g).max(), 1e-30)


def test_adjoint_gradient_matches_dense_derivative():
    """``dJ/dtheta_c = -lambda^T (dA/dtheta_c p - df/dtheta_c)`` with the
    derivatives of A and f taken by complex-step on the assembly."""
    P = random_2d(6, 5, 1.0, 6, block=(3, 5, 1))
    A, f = assemble(P.faces, np.exp(P.logK), P.n)
    p = _solve(A, f)
    lam = np.random.default_rng(13).standard_normal(P.n)
    g = adjoint.gradient(P.faces, P.logK, p, lam)
    for c in range(0, P.n, 7):
        h = 1e-30
        th = P.logK.astype(complex)
        th[c] += 1j * h
        K = np.exp(th)
        # complex-step through the TPFA formulas (same face list)
        tk = K[P.faces.k] * P.faces.gk
        interior = P.faces.l >= 0
        tl = np.zeros_like(tk)
        tl[interior] = K[P.faces.l[interior]] * P.faces.gl[interior]
        T = np.zeros_like(tk)
        T[interior] = tk[interior] * tl[interior] / (tk[interior] + tl[interior])
        dA = np.zeros((P.n, P.n))
        df = np.zeros(P.n)
        for fidx in range(P.faces.n_faces):
            k, l = P.faces.k[fidx], P.faces.l[fidx]
            if l >= 0:
                d = T[fidx].imag / h
                dA[k, k] += d; dA[l, l] += d; dA[k, l] -= d; dA[l, k] -= d
            else:
                d = tk[fidx].imag / h
                dA[k, k] += d
                df[k] += d * P.faces.pD[fidx]
        assert np.isclose(g[c], -lam @ (dA @ p - df), rtol=1e-10, atol=1e-14)
