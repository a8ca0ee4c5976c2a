"""The nested-dissection interface solve (the default where eta = S^{-1} b is
its own launches) through the C-ABI: explicit inverses of the mutually
uncoupled diagonal blocks of S in a nested-dissection order of the basis
functions and of the Schur complement on the separators above them (block
elimination; Sec. 4: S is SPD).  Against the FP64 oracle (which solves with
S directly), against the dense explicit S^{-1} product of the same handle
type, and against the fused form, on cases with and without separator rows,
one to sixteen right-hand sides, in applies and in PCG."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from oracle import AlgMortarCPU, partition_blocks, pcg  # noqa: E402
from workloads import make_config  # noqa: E402
from tests.test_gpu_parity import rel, gpu, cpu, setup_case  # noqa: E402

_cache = {}


def _big(name):
    """cases whose dissection has separator rows: a 64^3 GRF grid (16 blocks,
    320 separator rows) and a 40 x 40 x 24 layered grid with 5 x 4 x 4
    subdomains (1252 basis functions, 308 separator rows)"""
    if name not in _cache:
        if name == "grf64":
            P = make_config("c4", nx=64, ny=64, nz=64)
            part, m = partition_blocks(P.dims, P.partition[1])
        else:
            P = make_config("c2", nx=40, ny=40, nz=24)
            part, m = partition_blocks(P.dims, (5, 4, 4))
        _cache[name] = (P.A, part, m, P.b, AlgMortarCPU(P.A, part))
    return _cache[name]


def _get(name):
    return _big(name) if name in ("grf64", "tiles") else setup_case(name)


@pytest.mark.parametrize("name", ["c1", "layered", "bisect", "grf64", "tiles"])
def test_nd_apply_against_oracle_and_dense(name):
    A, part, m, b, ora = _get(name)
    order, blk, ntop = am.interface_nd(A, part, m, 1)
    hn = am.AlgMortar(A, part, m, separate_iface=True)
    hd = am.AlgMortar(A, part, m, separate_iface=True, dense_iface=True)
    hf = am.AlgMortar(A, part, m)
    rng = np.random.default_rng(21)
    for r in (b, rng.standard_normal(A.n), rng.standard_normal(A.n)):
        zr = ora.apply(r)
        zn = cpu(hn.apply(gpu(r)))
        assert rel(zn, zr) <= 1e-12, (name, ntop, rel(zn, zr))
        assert rel(zn, cpu(hd.apply(gpu(r)))) <= 1e-12
        assert rel(zn, cpu(hf.apply(gpu(r)))) <= 1e-12
    # the reordered inverse, exported in the original order, equals the dense one
    Sn, Sd = hn.export_interface("Sinv"), hd.export_interface("Sinv")
    assert np.linalg.norm(Sn - Sd) <= 1e-11 * np.linalg.norm(Sd)
    for h in (hn, hd, hf):
        h.close()


@pytest.mark.parametrize("name,max_nrhs,ncol", [("grf64", 16, 16), ("tiles", 4, 3),
                                                ("grf64", 2, 2), ("bisect", 8, 5)])
def test_nd_several_columns_apply_and_pcg(name, max_nrhs, ncol):
    A, part, m, b, ora = _get(name)
    h = am.AlgMortar(A, part, m, separate_iface=True, max_nrhs=max_nrhs)
    R = np.random.default_rng(ncol).standard_normal((ncol, A.n))
    Z = cpu(h.apply(gpu(R)))
    for k in range(ncol):
        assert rel(Z[k], ora.apply(R[k])) <= 1e-12, k
    X, info, _ = h.pcg(gpu(R), 1e-10)
    X = cpu(X)
    As = A.to_scipy()
    for k in sorted({0, ncol // 2, ncol - 1}):
        ref = pcg(lambda v: As @ v, R[k], ora.apply, 1e-10)
        assert info[k]["converged"] == 1
        assert abs(info[k]["iterations"] - ref.iterations) <= 1
        assert rel(X[k], ref.x) <= 1e-8, k
    h.close()


def test_nd_pcg_graph_and_plain_launches_agree():
    """The dissection launches inside captured PCG chunks and as plain
    launches give the same iterate bit for bit (same kernels, same order)."""
    A, part, m, b, ora = _get("grf64")
    hg = am.AlgMortar(A, part, m, separate_iface=True)
    hp = am.AlgMortar(A, part, m, separate_iface=True, graph=False)
    xg, ig, _ = hg.pcg(gpu(b), 1e-10)
    xp, ip, _ = hp.pcg(gpu(b), 1e-10)
    assert ig[0]["iterations"] == ip[0]["iterations"]
    assert torch.equal(xg, xp)
    As = A.to_scipy()
    ref = pcg(lambda v: As @ v, b, ora.apply, 1e-10)
    assert abs(ig[0]["iterations"] - ref.iterations) <= 1 and rel(cpu(xg), ref.x) <= 1e-8
    hg.close()
    hp.close()


def test_nd_update_values_equals_fresh_setup(monkeypatch):
    """New values on a handle in the dissection form redo its blocks and
    C^{-1}: applies equal those of a fresh set-up bit for bit."""
    monkeypatch.setenv("ALGMORTAR_TILE", "0")
    P = make_config("c4", nx=64, ny=64, nz=64)
    part, m = partition_blocks(P.dims, P.partition[1])
    h = am.AlgMortar(P.A, part, m, separate_iface=True)
    P2 = make_config("c4", seed=9, nx=64, ny=64, nz=64)
    h.update_values(P2.A)
    fresh = am.AlgMortar(P2.A, part, m, separate_iface=True)
    r = gpu(np.random.default_rng(2).standard_normal(P.n))
    assert torch.equal(h.apply(r), fresh.apply(r))
    h.close()
    fresh.close()
