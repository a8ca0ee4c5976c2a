"""The three large workloads at full size, in the launch configurations the
benchmark times, against stored oracle results (tests/golden/full_*.npz,
written by tests/golden/make_golden.py from oracle/ only, sampled at 4096
seeded cells with the full vectors' norms):

* 64^3 layered (contrast 1e6), 512 subdomains, 1 right-hand side;
* 128^3 GRF, 4096 subdomains, 1 right-hand side (the benchmark workload);
* 128 x 128 x 64 distorted hexahedra, bisection into 1,922 subdomains,
  16 right-hand sides solved together (columns 0, 5 and 15 kept).

Bars: applies (Algorithm 2) relative L2 <= 1e-12 on the sample, every sampled
entry within 1e-12 of the vector's largest magnitude, the norm within 1e-12;
and, on every cell of the full vector, the residual r - A z vanishes on cells
with no coupling to another subdomain (local solves are exact there; Sec. 5.3).
PCG at tol 1e-10: iterations within one of the oracle's, the true residual
recomputed on the host within 2e-10, and the solution within relative L2 1e-8
of the oracle's (on the sample).  On the 64^3 layered workload the oracle's
own tol-1e-10 solution is 1.3e-8 from its tol-1e-13 reference, so when the
direct comparison misses 1e-8, both solutions are measured against that
reference instead and the GPU's distance must not exceed the oracle's by
more than 1e-9 (the reading of the parity metric for that workload)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2607_22905_amd as am  # noqa: E402
from workloads import make_config  # noqa: E402

DEV = "cuda:0"
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.load(os.path.join(GOLD, f"full_{name}.npz"), allow_pickle=False)


def _setup(name):
    P = make_config(name)
    if P.partition[0] == "blocks":
        part, m = am.partition_blocks(P.dims, P.partition[1])
    else:
        _, lo, hi, seed = P.partition
        part, m = am.partition_bisect(P.A, lo, hi, seed)
    return P, part, m


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _apply_vectors(P, g):
    vecs = []
    for lab in g["apply_labels"]:
        lab = str(lab)
        if lab.startswith("normal"):
            vecs.append(np.random.default_rng(int(lab[6:])).standard_normal(P.n))
        elif lab == "b":
            vecs.append(P.b)
        else:
            vecs.append(P.b[:, int(lab[1:])])
    return vecs


def _check_apply(P, g, r, z, t, As, interior):
    idx = g["sample_idx"]
    zs = g["apply_sample"][t]
    assert _rel(z[idx], zs) <= 1e-12, (t, _rel(z[idx], zs))
    assert np.abs(z[idx] - zs).max() <= 1e-12 * g["apply_maxabs"][t]
    assert abs(np.linalg.norm(z) - g["apply_norm"][t]) <= 1e-12 * g["apply_norm"][t]
    # full vector: A z = r on cells with no coupling outside their subdomain
    res = np.abs(r - As @ z)[interior]
    scale = (abs(As) @ np.abs(z) + np.abs(r))[interior]
    assert (res <= 1e-12 * scale).all(), float((res / scale).max())


def _interior(P, part):
    A = P.A
    rows = np.repeat(np.arange(P.n), np.diff(A.row_ptr))
    cross = part[rows] != part[A.col]
    touch = np.zeros(P.n, dtype=bool)
    touch[rows[cross]] = True
    return ~touch


def _check_x(name, P, g, x, info, c, As, b):
    idx = g["sample_idx"]
    assert info["converged"] == 1
    assert abs(info["iterations"] - int(g["iterations"][c])) <= 1, (info["iterations"], g["iterations"][c])
    tr = np.linalg.norm(b - As @ x) / np.linalg.norm(b)
    assert tr <= 2e-10, tr
    err = _rel(x[idx], g["x_sample"][c])
    print(f"{name} column {c}: iterations {info['iterations']} (oracle {int(g['iterations'][c])}), "
          f"solution vs oracle rel L2 {err:.3e}, true residual {tr:.2e}")
    if err <= 1e-8:
        return
    assert "ref_x_sample" in g.files, err
    ref = g["ref_x_sample"][c]
    e_gpu, e_or = _rel(x[idx], ref), _rel(g["x_sample"][c], ref)
    print(f"{name}: against the tol-1e-13 reference: GPU {e_gpu:.3e}, oracle {e_or:.3e}")
    assert e_gpu <= e_or + 1e-9


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_fullsize_single_rhs(name):
    g = _load(name)
    P, part, m = _setup(name)
    As = P.A.to_scipy().tocsr()
    interior = _interior(P, part)
    h = am.AlgMortar(P.A, part, m)
    for t, r in enumerate(_apply_vectors(P, g)):
        z = h.apply(torch.as_tensor(r, device=DEV)).cpu().numpy()
        _check_apply(P, g, r, z, t, As, interior)
    x, info, _ = h.pcg(torch.as_tensor(P.b, device=DEV), 1e-10)
    _check_x(name, P, g, x.cpu().numpy(), info[0], 0, As, P.b)
    h.close()


def test_fullsize_batched_16_rhs():
    name = "c3"
    g = _load(name)
    P, part, m = _setup(name)
    As = P.A.to_scipy().tocsr()
    interior = _interior(P, part)
    h = am.AlgMortar(P.A, part, m, max_nrhs=16)
    B = np.ascontiguousarray(P.b.T)  # rows = right-hand sides
    cols = [int(c) for c in g["rhs_columns"]]
    Z = h.apply(torch.as_tensor(B, device=DEV)).cpu().numpy()  # all 16 together
    labels = [str(l) for l in g["apply_labels"]]
    for t, lab in enumerate(labels):
        if lab.startswith("b"):
            c = int(lab[1:])
            _check_apply(P, g, B[c], Z[c], t, As, interior)
        else:
            r = np.random.default_rng(int(lab[6:])).standard_normal(P.n)
            z = h.apply(torch.as_tensor(r, device=DEV)).cpu().numpy()
            _check_apply(P, g, r, z, t, As, interior)
    X, info, _ = h.pcg(torch.as_tensor(B, device=DEV), 1e-10)
    X = X.cpu().numpy()
    for t, c in enumerate(cols):
        _check_x(name, P, g, X[c], info[c], t, As, B[c])
    h.close()
