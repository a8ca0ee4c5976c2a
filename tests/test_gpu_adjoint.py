"""Differentiation form on the GPU: device TPFA assembly, the face-scatter
gradient kernel, the adjoint solve on the forward handle and the autograd
Function, against the FP64 oracle and against central finite differences
(h = 1e-6; the perturbed solves start from p and solve for the correction to
1e-10 relative to its right-hand side).  All calls go through the C-ABI."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from oracle import AlgMortarCPU, adjoint, partition_blocks, pcg  # noqa: E402
from workloads import make_config  # noqa: E402
from workloads.fields import grf  # noqa: E402
from workloads.grids import cartesian_faces, distorted_hex_faces  # noqa: E402
from workloads.tpfa import Faces, assemble  # noqa: E402

DEV = "cuda:0"
HERE = os.path.dirname(os.path.abspath(__file__))


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def small_problem():
    """24 x 24 x 16 cells, ln K a field with sigma 2 and ell (12, 12, 4),
    p = 1 at x = 0 and p = 0 at x = 24, 8^3 blocks (18 subdomains), 60
    observation cells."""
    nx, ny, nz = 24, 24, 16
    n = nx * ny * nz
    g = grf((nz, ny, nx), (4.0, 12.0, 12.0), 2.0, 21).ravel()
    gp = g + 0.1 * grf((nz, ny, nx), (4.0, 12.0, 12.0), 2.0, 22).ravel()
    faces = Faces.from_dict(cartesian_faces(nx, ny, nz, [(0, 0, 1.0), (0, 1, 0.0)]))
    part, m = partition_blocks((nx, ny, nz), (8, 8, 8))
    obs = np.sort(np.random.default_rng(23).choice(n, size=60, replace=False))
    return dict(n=n, logK=g, logK_pert=gp, faces=faces, part=part, m=m, obs=obs)


def oracle_gradient(faces, logK, n, part, obs, pobs, tol=1e-12):
    A, f = assemble(faces, np.exp(logK), n)
    As = A.to_scipy()
    pre = AlgMortarCPU(A, part)
    p = pcg(lambda v: As @ v, f, pre.apply, tol).x
    lam = pcg(lambda v: As @ v, adjoint.dloss_dp(p, obs, pobs), pre.apply, tol).x
    return p, lam, adjoint.gradient(faces, logK, p, lam)


def perturbation_rhs(faces, logK, c, dh, p0):
    """Right-hand side of the correction d for ln K_c -> ln K_c + dh:
    (A + dA)(p0 + d) = f + df gives (A + dA) d = df - dA p0 + (f - A p0).
    The last term is the same for +dh and -dh and drops out of d+ - d-, so
    only the perturbation is formed, face by face: an interior face (k, l)
    adds -dT (p0_k - p0_l) to row k and +dT (p0_k - p0_l) to row l; a
    Dirichlet face of c adds dt (pD - p0_c).  Forming f - A p0 instead
    subtracts numbers of size |T p| to leave one of size h |T dp|."""
    from workloads.tpfa import transmissibilities
    sel = np.flatnonzero((faces.k == c) | (faces.l == c))
    sub = Faces(k=faces.k[sel], l=faces.l[sel], gk=faces.gk[sel], gl=faces.gl[sel],
                pD=faces.pD[sel])
    K0 = np.exp(logK)
    K1 = K0.copy()
    K1[c] = np.exp(logK[c] + dh)
    tk0, _, T0 = transmissibilities(sub, K0)
    tk1, _, T1 = transmissibilities(sub, K1)
    r = np.zeros(logK.size)
    inner = sub.l >= 0
    k, l = sub.k[inner], sub.l[inner]
    flux = (T1[inner] - T0[inner]) * (p0[k] - p0[l])
    np.add.at(r, k, -flux)
    np.add.at(r, l, flux)
    kb = sub.k[~inner]
    np.add.at(r, kb, (tk1[~inner] - tk0[~inner]) * (sub.pD[~inner] - p0[kb]))
    return r


def fd_gradient(model, faces, logK, p0, obs, pobs, cells, h=1e-6, tol=1e-10):
    """Central differences of J on the GPU path: each perturbed system is set
    up on the device and solved for the correction d from p0 (PCG to ``tol``
    relative to its right-hand side), and J(p0 + d+) - J(p0 + d-) is
    evaluated as 1/2 sum_obs (d+ - d-)(2 (p0 - pobs) + d+ + d-), the same
    number without the cancellation of subtracting two nearly equal losses."""
    p0h = cpu(p0)
    th0 = cpu(logK)
    e0 = p0h[obs] - pobs
    out = []
    for c in cells:
        ds = []
        for sgn in (1.0, -1.0):
            th = logK.clone()
            th[c] += sgn * h
            A, _ = model.assemble(th)
            r = perturbation_rhs(faces, th0, c, sgn * h, p0h)
            hd = am.AlgMortar(A, model.part, model.nparts)
            d, info, _ = hd.pcg(gpu(r), tol)
            assert info[0]["converged"] == 1
            hd.close()
            ds.append(cpu(d)[obs])
        dJ = 0.5 * float(np.sum((ds[0] - ds[1]) * (2.0 * e0 + ds[0] + ds[1])))
        out.append(dJ / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("grid", ["cartesian", "hex"])
def test_tpfa_assembly_matches_host(grid):
    nx, ny, nz = 10, 9, 7
    n = nx * ny * nz
    if grid == "cartesian":
        faces = Faces.from_dict(cartesian_faces(nx, ny, nz, [(0, 0, 1.0), (0, 1, 0.5)]))
    else:
        faces = Faces.from_dict(distorted_hex_faces(nx, ny, nz, 0.3, 6, [(0, 0, 0.25)]))
    logK = np.random.default_rng(3).normal(size=n) * 2.0
    A, f = assemble(faces, np.exp(logK), n)
    t = am.Tpfa(faces, n)
    assert np.array_equal(t.row_ptr, A.row_ptr) and np.array_equal(t.col, A.col)
    val, fd = t.assemble(gpu(logK))
    val, fd = cpu(val), cpu(fd)
    assert np.all(np.abs(val - A.val) <= 1e-13 * np.abs(A.val))
    assert np.all(np.abs(fd - f) <= 1e-13 * np.abs(f))
    t.close()


def test_face_gradient_matches_oracle():
    nx, ny, nz = 12, 10, 9
    n = nx * ny * nz
    faces = Faces.from_dict(distorted_hex_faces(nx, ny, nz, 0.3, 8, [(0, 0, 1.0), (0, 1, 0.0)]))
    rng = np.random.default_rng(9)
    logK, p, lam = rng.normal(size=n), rng.normal(size=n), rng.normal(size=n)
    ref = adjoint.gradient(faces, logK, p, lam)
    t = am.Tpfa(faces, n)
    g = cpu(t.face_grad(gpu(logK), gpu(p), gpu(lam)))
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()
    t.close()


def test_adjoint_gradient_small_grid():
    """Adjoint gradient vs the oracle's (whole field) and vs central finite
    differences on 6 cells; the autograd Function gives the same gradient."""
    P = small_problem()
    n = P["n"]
    model = am.DarcyModel(P["faces"], n, P["part"], P["m"], tol=1e-10, adjoint_tol=1e-12)
    pp, hp = model.forward_solve(gpu(P["logK_pert"]))
    hp.close()
    pobs = cpu(pp)[P["obs"]]
    p_o, lam_o, g_o = oracle_gradient(P["faces"], P["logK"], n, P["part"], P["obs"], pobs)

    logK = gpu(P["logK"])
    p, h = model.forward_solve(logK)
    assert np.linalg.norm(cpu(p) - p_o) <= 1e-8 * np.linalg.norm(p_o)
    dJdp = gpu(adjoint.dloss_dp(cpu(p), P["obs"], pobs))
    g, lam, info = am.adjoint_grad(h, model.tpfa, logK, p, dJdp, tol=1e-12)
    assert info["converged"] == 1
    g = cpu(g)
    assert np.linalg.norm(g - g_o) <= 1e-7 * np.linalg.norm(g_o)
    h.close()

    # autograd
    th = logK.clone().requires_grad_(True)
    pa = am.AlgMortarSolve.apply(th, model)
    J = 0.5 * ((pa[torch.as_tensor(P["obs"], device=DEV)] - gpu(pobs)) ** 2).sum()
    J.backward()
    ga = cpu(th.grad)
    assert np.abs(ga - g).max() <= 1e-12 * np.abs(g).max()

    gmax = np.abs(g_o).max()
    cand = np.flatnonzero(np.abs(g_o) >= 1e-3 * gmax)
    cells = np.sort(np.random.default_rng(24).choice(cand, size=6, replace=False))
    fd = fd_gradient(model, P["faces"], logK, p, P["obs"], pobs, cells)
    relerr = np.abs(g[cells] - fd) / np.abs(fd)
    assert relerr.max() <= 1e-5, relerr
    model.close()


def test_adjoint_gradient_96cube():
    """The 96^3 differentiation workload (1728 subdomains): loss and sampled
    gradient against the oracle's stored record, and the 20 finite-difference
    cells to 1e-5 relative (state and adjoint solved to 1e-12)."""
    gold = json.load(open(os.path.join(HERE, "golden", "c5_adjoint.json")))
    P = make_config("c5")
    part, m = partition_blocks(P.dims, P.partition[1])
    obs = P.extra["obs"]
    # the state is solved as tightly as the adjoint: finite differences
    # differentiate the exact solution map, and a 1e-10 state shifts the
    # adjoint gradient by ~1e-8 of its maximum (1e-5 relative on the
    # smallest finite-difference cells)
    model = am.DarcyModel(P.faces, P.n, part, m, tol=P.extra["adjoint_tol"],
                          adjoint_tol=P.extra["adjoint_tol"])
    pp, hp = model.forward_solve(gpu(P.extra["logK_pert"]))
    hp.close()
    pobs_full = cpu(pp)
    pobs = pobs_full[obs]
    logK = gpu(P.logK)
    p, h = model.forward_solve(logK)
    ph = cpu(p)
    idx = np.array(gold["sample_idx"])
    assert np.abs(ph[idx] - np.array(gold["p_sample"])).max() <= 1e-7
    assert np.abs(pobs_full[idx] - np.array(gold["pobs_sample"])).max() <= 1e-7
    J = adjoint.loss(ph, obs, pobs)
    assert abs(J - gold["J"]) <= 1e-5 * gold["J"]
    dJdp = gpu(adjoint.dloss_dp(ph, obs, pobs))
    g, lam, info = am.adjoint_grad(h, model.tpfa, logK, p, dJdp, tol=P.extra["adjoint_tol"])
    assert info["converged"] == 1
    h.close()
    g = cpu(g)
    gmax = gold["grad_max"]
    assert np.abs(g[idx] - np.array(gold["grad_sample"])).max() <= 1e-6 * gmax
    cells = np.array(gold["fd_cells"])
    assert np.abs(g[cells] - np.array(gold["grad_fd_cells"])).max() <= 1e-6 * gmax
    fd = fd_gradient(model, P.faces, logK, p, obs, pobs, cells, h=P.extra["fd_h"])
    relerr = np.abs(g[cells] - fd) / np.abs(fd)
    print("c5 FD relative errors: max %.3e median %.3e" % (relerr.max(), np.median(relerr)))
    assert relerr.max() <= 1e-5, relerr
    model.close()
