"""Pins for the oracle's AlgMortar set-up and apply.

Each check is fixed by the paper or by linear algebra, independently of the
oracle's own arithmetic: identities of Sec. 3.2-3.3 and 4, the closed-form
reduced preconditioner (Sec. 5.1), exactness special cases (single subdomain,
per-edge mortar space, chains, two cells), the interface-only residual
(Sec. 5.3), weak flux continuity (Sec. 3.3 remark), the spectral bound
(Sec. 5.2) and M-matrix properties of the basis functions and of ``S``.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import AlgMortarCPU, NotSPDError, partition_blocks, partition_bisect, dense
from workloads.grids import cartesian_faces
from workloads.tpfa import Faces, assemble
from tests._problems import random_2d, random_3d, chain, dense_csr, random_mmatrix


def _pre(P, mortar="interface"):
    part, _ = partition_blocks(P.dims, P.partition[1])
    return AlgMortarCPU(P.A, part, mortar)


CASES = [
    lambda: random_2d(8, 8, 1.0, 0, block=(4, 4, 1)),
    lambda: random_2d(9, 6, 2.0, 1, block=(3, 3, 1)),
    lambda: random_3d(6, 6, 4, 1.5, 2, block=(3, 3, 2)),
    lambda: random_3d(4, 4, 4, 0.0, 3, block=(2, 2, 2)),
]


@pytest.fixture(params=range(len(CASES)))
def case(request):
    P = CASES[request.param]()
    return P, _pre(P)


def test_B_transpose_is_4WM(case):
    P, pre = case
    ops = dense.operators(pre)
    assert np.allclose(ops["B"].T, 4.0 * ops["W"] @ ops["M"], rtol=0, atol=1e-14 * abs(ops["W"]).max())


def test_trace_identities(case):
    P, pre = case
    ops = dense.operators(pre)
    st = pre.st
    p = np.random.default_rng(1).standard_normal(P.n)
    W, L, U = ops["W"], ops["L"], ops["U"]
    a, k, l = st.edge_a, st.edge_k, st.edge_l
    assert np.isclose(p @ U.T @ W @ L @ p, np.sum(a * p[k] * p[l]))
    assert np.isclose(p @ L.T @ W @ L @ p, np.sum(a * p[k] ** 2))
    assert np.isclose(p @ U.T @ W @ U @ p, np.sum(a * p[l] ** 2))


def test_local_rewrite_is_exact(case):
    """``Ahat p + B M p = A p`` (eq. local-system-rewrite with lambda = M p)."""
    P, pre = case
    ops = dense.operators(pre)
    Ad = dense.to_dense(P.A)
    assert np.allclose(ops["Ahat"] + ops["B"] @ ops["M"], Ad, rtol=0, atol=1e-13 * abs(Ad).max())
    # and the energy identity p^T Ahat p = p^T A p - 4 (Mp)^T W (Mp)
    p = np.random.default_rng(2).standard_normal(P.n)
    Mp = ops["M"] @ p
    assert np.isclose(p @ ops["Ahat"] @ p, p @ Ad @ p - 4.0 * Mp @ ops["W"] @ Mp)


def test_Q_is_spd_and_equivalent(case):
    P, pre = case
    ops = dense.operators(pre)
    Q = dense.Q_matrix(ops)
    assert np.allclose(Q, Q.T, atol=1e-13 * abs(Q).max())
    assert sla.eigh(Q, eigvals_only=True)[0] > 0
    # eliminating eta from Q gives the reduced preconditioner (scaled by 1/4)
    n = P.n
    S = Q[:n, :n] - Q[:n, n:] @ np.linalg.solve(Q[n:, n:], Q[n:, :n])
    assert np.allclose(4.0 * S, dense.reduced_preconditioner(ops), atol=1e-12 * abs(S).max())


def test_apply_matches_reduced_preconditioner(case):
    P, pre = case
    Mc = dense.reduced_preconditioner(dense.operators(pre))
    r = np.random.default_rng(3).standard_normal((P.n, 3))
    z = pre.apply(r)
    zd = np.linalg.solve(Mc, r)
    assert np.linalg.norm(z - zd) <= 1e-12 * np.linalg.norm(zd)


def test_spectrum_bound(case):
    """Eigenvalues of Mcal^{-1} A lie in [1/(1+K_Lambda), 1] (Sec. 5.2)."""
    P, pre = case
    ops = dense.operators(pre)
    Ad = dense.to_dense(P.A)
    Mc = dense.reduced_preconditioner(ops)
    Mc = 0.5 * (Mc + Mc.T)
    th = sla.eigh(Ad, Mc, eigvals_only=True)
    KL = dense.K_lambda(ops, Ad)
    assert th.max() <= 1.0 + 1e-10
    assert th.min() >= 1.0 / (1.0 + KL) - 1e-10
    assert th.min() > 0


def test_interface_only_residual(case):
    """``r - A z`` vanishes on cells with no interface edge (Sec. 5.3)."""
    P, pre = case
    r = np.random.default_rng(4).standard_normal(P.n)
    z = pre.apply(r)
    res = r - P.A.matvec(z)
    touch = np.zeros(P.n, dtype=bool)
    touch[pre.st.edge_k] = True
    touch[pre.st.edge_l] = True
    assert np.abs(res[~touch]).max() <= 1e-12 * np.abs(r).max()
    assert np.abs(res[touch]).max() > 1e-8


def test_weak_flux_continuity(case):
    """``eta_n`` is the a-weighted mean of ``(z_k + z_l)/2`` over ``E_n``
    (eq. local-system-lm-b with a piecewise constant mortar)."""
    P, pre = case
    st = pre.st
    r = np.random.default_rng(5).standard_normal(P.n)
    z, parts = pre.apply(r, return_parts=True)
    for nidx in range(st.n_iface):
        e = slice(st.iface_ptr[nidx], st.iface_ptr[nidx + 1])
        a = st.edge_a[e]
        avg = 0.5 * (z[st.edge_k[e]] + z[st.edge_l[e]])
        assert np.isclose(parts["eta"][nidx], np.sum(a * avg) / np.sum(a), rtol=1e-11, atol=1e-13)


def test_S_and_mbf_mmatrix_properties(case):
    P, pre = case
    S = pre.S.toarray()
    assert sla.eigh(S, eigvals_only=True)[0] > 0
    off = S - np.diag(np.diag(S))
    assert off.max() <= 1e-14 * abs(S).max()
    # MBFs in [0, 1]; they sum to one on subdomains without Dirichlet rows
    rowsum = P.A.matvec(np.ones(P.n))
    st = pre.st
    total = np.zeros(P.n)
    for midx in range(st.n_iface):
        for s, vals in pre.phat[midx].items():
            assert vals.min() >= -1e-14 and vals.max() <= 1 + 1e-12
            total[st.omega(s)] += vals
    for i in range(pre.m):
        om = st.omega(i)
        if np.all(np.abs(rowsum[om]) < 1e-12 * abs(P.A.val).max()):
            assert np.allclose(total[om], 1.0, atol=1e-12)


def test_unit_permeability_local_operator_is_local_dirichlet():
    """Remark: for K = I on a uniform grid, ``A_i`` is the local TPFA
    operator with Dirichlet faces (half-transmissibility 2) on the subdomain
    boundary."""
    P = random_3d(6, 4, 4, 0.0, 0, block=(3, 2, 2), dirichlet=((0, 0, 0.0),))
    pre = _pre(P)
    for i in range(pre.m):
        om = pre.st.omega(i)
        # subdomain geometry: block (bi, bj, bk) of 3x2x2 cells
        ci = om[0]
        x0, y0, z0 = ci % 6, (ci // 6) % 4, ci // 24
        dirichlet = []
        if x0 > 0:
            dirichlet.append((0, 0, 0.0))
        if x0 + 3 < 6:
            dirichlet.append((0, 1, 0.0))
        if y0 > 0:
            dirichlet.append((1, 0, 0.0))
        if y0 + 2 < 4:
            dirichlet.append((1, 1, 0.0))
        if z0 > 0:
            dirichlet.append((2, 0, 0.0))
        if z0 + 2 < 4:
            dirichlet.append((2, 1, 0.0))
        if x0 == 0:
            dirichlet.append((0, 0, 0.0))  # the global Dirichlet face
        f = Faces.from_dict(cartesian_faces(3, 2, 2, dirichlet))
        Aloc, _ = assemble(f, np.ones(12), 12)
        assert np.allclose(pre.Ai[i], dense.to_dense(Aloc), rtol=0, atol=1e-14)


def test_single_subdomain_is_direct_solve():
    P = random_3d(4, 4, 3, 1.0, 6, block=(4, 4, 3))
    pre = _pre(P)
    assert pre.st.n_iface == 0
    r = np.random.default_rng(6).standard_normal(P.n)
    z = pre.apply(r)
    assert np.allclose(z, np.linalg.solve(dense.to_dense(P.A), r), rtol=1e-12, atol=0)


@pytest.mark.parametrize("mk", [lambda: random_2d(8, 8, 1.0, 7, block=(4, 4, 1)),
                                lambda: random_3d(6, 6, 4, 1.0, 8, block=(3, 3, 2))])
def test_per_edge_mortar_is_direct_solve(mk):
    """With Lambda = R^E the method reproduces A (Sec. 3.3)."""
    P = mk()
    pre = _pre(P, mortar="edge")
    r = np.random.default_rng(9).standard_normal(P.n)
    z = pre.apply(r)
    zd = np.linalg.solve(dense.to_dense(P.A), r)
    assert np.linalg.norm(z - zd) <= 1e-11 * np.linalg.norm(zd)


def test_chain_with_single_edge_interfaces_is_exact():
    """Every E_ij of a 1-D chain is one edge, so the piecewise constant space
    equals R^E and the preconditioner is A^{-1}."""
    A, faces, g = chain(24, 1)
    part = np.repeat(np.arange(6), 4).astype(np.int32)
    pre = AlgMortarCPU(A, part)
    r = np.random.default_rng(10).standard_normal(24)
    assert np.allclose(pre.apply(r), np.linalg.solve(dense.to_dense(A), r), rtol=1e-12)


def test_two_cell_closed_form():
    """A = [[t+T, -T], [-T, t+T]], parts {0}, {1}: closed forms of A_i, the MBF,
    S, b, eta and z = A^{-1} r."""
    t, T = 1.7, 0.45
    Ad = np.array([[t + T, -T], [-T, t + T]])
    A = dense_csr(Ad)
    pre = AlgMortarCPU(A, np.array([0, 1], dtype=np.int32))
    assert np.allclose(pre.Ai[0], [[t + 2 * T]]) and np.allclose(pre.Ai[1], [[t + 2 * T]])
    assert np.isclose(pre.phat[0][0][0], 2 * T / (t + 2 * T))
    assert np.isclose(pre.S.toarray()[0, 0], T * t / (t + 2 * T))
    r = np.array([0.3, -1.1])
    z, parts = pre.apply(r, return_parts=True)
    assert np.isclose(parts["b"][0], T * (r[0] + r[1]) / (2 * (t + 2 * T)))
    assert np.isclose(parts["eta"][0], (r[0] + r[1]) / (2 * t))
    assert np.isclose(z[0], ((t + T) * r[0] + T * r[1]) / (t * (t + 2 * T)))
    assert np.allclose(z, np.linalg.solve(Ad, r))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_mmatrix_irregular_partition(seed):
    """General SPD M-matrices with irregular parts: apply equals the dense
    reduced preconditioner, and the spectrum bound holds."""
    Ad = random_mmatrix(40, 0.08, seed)
    A = dense_csr(Ad)
    part = np.random.default_rng(seed).integers(0, 5, size=40).astype(np.int32)
    part[:5] = np.arange(5)
    pre = AlgMortarCPU(A, part)
    ops = dense.operators(pre)
    Mc = dense.reduced_preconditioner(ops)
    r = np.random.default_rng(11).standard_normal(40)
    assert np.allclose(pre.apply(r), np.linalg.solve(Mc, r), rtol=1e-11)
    th = sla.eigh(Ad, 0.5 * (Mc + Mc.T), eigvals_only=True)
    assert 0 < th.min() and th.max() <= 1 + 1e-10


def test_not_spd_detected():
    Ad = np.array([[1.0, -2.0, 0], [-2.0, 1.0, -0.5], [0, -0.5, 2.0]])
    with pytest.raises(NotSPDError):
        AlgMortarCPU(dense_csr(Ad), np.array([0, 0, 1], dtype=np.int32))


def test_mutation_dropped_factor_two_is_caught():
    """A plausible mistake (the factor 2 of B_ij dropped) breaks the dense
    reduced-preconditioner pin: guards the pin's sensitivity."""
    P = random_2d(8, 8, 1.0, 0, block=(4, 4, 1))
    pre = _pre(P)
    Mc = dense.reduced_preconditioner(dense.operators(pre))
    r = np.random.default_rng(3).standard_normal(P.n)
    good = pre.apply(r)

    class Broken(AlgMortarCPU):
        def B_local(self, s, nidx):
            return 0.5 * super().B_local(s, nidx)

    part, _ = partition_blocks(P.dims, P.partition[1])
    bad = Broken(P.A, part).apply(r)
    zd = np.linalg.solve(Mc, r)
    assert np.linalg.norm(good - zd) < 1e-12 * np.linalg.norm(zd)
    assert np.linalg.norm(bad - zd) > 1e-3 * np.linalg.norm(zd)
