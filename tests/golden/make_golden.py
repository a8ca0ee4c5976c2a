"""Write the stored expected values under tests/golden/ (calls only oracle/ and
the shared input generators).

    python tests/golden/make_golden.py

* ``structure.json``: SHA-256 of the partition map, permutation, interface edge
  arrays and interface pairs of every workload (the index sets are integer
  results, so later runs and the host library must reproduce them bit for
  bit), plus their sizes.
* ``c1_pcg.json``: iteration count and solution norms of the oracle's
  AlgMortar-PCG on the 2-D workload (tol 1e-10).
* ``c2_pcg.json``: the 64^3 layered workload (the benchmark's): the oracle's
  apply of a seeded N(0,1) vector and its PCG solution at the workload's
  tolerance (1e-8), as norms plus values at 256 seeded cells.
* ``c4_pcg.json``: the 128^3 precision workload: the oracle's PCG solution at
  tol 1e-8 and at 1e-12 (the reference the reduced-precision forms are
  measured against), values at 256 seeded cells, norms, iteration counts.
* ``c5_adjoint.json``: the 96^3 differentiation workload: the oracle's loss
  J = 1/2 sum_obs (p - pobs)^2 (pobs from the perturbed-field forward solve),
  its adjoint gradient dJ/dlog K at 256 seeded cells and at the 20
  finite-difference cells (drawn among cells with |g| >= 1e-3 max|g|), and
  the gradient's norm and maximum.  All oracle solves at tol 1e-12.

* ``full_c2.npz``, ``full_c4.npz``, ``full_c3.npz``: the three large
  workloads at full size, at 4096 seeded cells (sample seed 17) with the
  full vectors' L2 norms and maximum magnitudes.  Applies of the workload's
  right-hand side(s) and seeded N(0,1) vectors; PCG solutions at tol 1e-10
  with their iteration counts; for the 64^3 layered workload (contrast 1e6)
  also a reference solve at tol 1e-13.  The 16-RHS irregular workload keeps
  columns 0, 5 and 15 (its oracle solves one column at a time).

    python tests/golden/make_golden.py [structure|c2|c5|c4|full_c2|full_c4|full_c3]
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import make_config  # noqa: E402
from oracle import partition_blocks, partition_bisect, build_structure, AlgMortarCPU, pcg  # noqa: E402


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def structure_record(P):
    if P.partition[0] == "blocks":
        part, m = partition_blocks(P.dims, P.partition[1])
    else:
        _, lo, hi, seed = P.partition
        part, m = partition_bisect(P.A.row_ptr, P.A.col, P.A.val, P.n, lo, hi, seed)
    st = build_structure(P.A, part)
    return dict(n=P.n, nnz=P.A.nnz, nparts=int(m), n_iface=int(st.n_iface),
                n_edges=int(st.n_edges), max_iface_per_sub=int(max(len(x) for x in st.I)),
                part=sha(part.astype(np.int32)), perm=sha(st.perm.astype(np.int32)),
                edge_k=sha(st.edge_k.astype(np.int32)), edge_l=sha(st.edge_l.astype(np.int32)),
                iface_ptr=sha(st.iface_ptr.astype(np.int64)),
                iface_ij=sha(st.iface_ij.astype(np.int32)))


def main():
    out = {}
    for name in ("c1", "c2", "c3", "c4", "c5"):
        P = make_config(name)
        out[name] = structure_record(P)
        print(name, out[name]["nparts"], out[name]["n_iface"], flush=True)
    with open(os.path.join(HERE, "structure.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    P = make_config("c1")
    part, _ = partition_blocks(P.dims, P.partition[1])
    pre = AlgMortarCPU(P.A, part)
    As = P.A.to_scipy()
    res = pcg(lambda v: As @ v, P.b, pre.apply, P.tol)
    rec = dict(iterations=res.iterations, x_norm2=float(np.linalg.norm(res.x)),
               x_sum=float(res.x.sum()), true_rel_res=res.true_rel_res)
    with open(os.path.join(HERE, "c1_pcg.json"), "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(rec)


def c2_record():
    P = make_config("c2")
    part, _ = partition_blocks(P.dims, P.partition[1])
    pre = AlgMortarCPU(P.A, part)
    idx = np.sort(np.random.default_rng(7).choice(P.n, size=256, replace=False))
    r = np.random.default_rng(11).standard_normal(P.n)
    z = pre.apply(r)
    As = P.A.to_scipy()
    res = pcg(lambda v: As @ v, P.b, pre.apply, P.tol)
    rec = dict(apply_seed=11, sample_idx=idx.tolist(), apply_sample=z[idx].tolist(),
               apply_norm=float(np.linalg.norm(z)), iterations=res.iterations,
               x_sample=res.x[idx].tolist(), x_norm2=float(np.linalg.norm(res.x)),
               true_rel_res=res.true_rel_res, tol=P.tol)
    with open(os.path.join(HERE, "c2_pcg.json"), "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print("c2", res.iterations, res.true_rel_res)


def c5_record():
    from oracle import adjoint
    P = make_config("c5")
    part, _ = partition_blocks(P.dims, P.partition[1])
    As = P.A.to_scipy()
    pre = AlgMortarCPU(P.A, part)
    tol = 1e-12
    res = pcg(lambda v: As @ v, P.b, pre.apply, tol)
    p = res.x
    # observed pressures: forward solve with the perturbed field (own operator)
    from workloads.tpfa import assemble
    Ap, fp = assemble(P.faces, np.exp(P.extra["logK_pert"]), P.n, None)
    Aps = Ap.to_scipy()
    pre_p = AlgMortarCPU(Ap, part)
    pobs_full = pcg(lambda v: Aps @ v, fp, pre_p.apply, tol).x
    obs = P.extra["obs"]
    pobs = pobs_full[obs]
    J = adjoint.loss(p, obs, pobs)
    lam_res = pcg(lambda v: As @ v, adjoint.dloss_dp(p, obs, pobs), pre.apply, tol)
    g = adjoint.gradient(P.faces, P.logK, p, lam_res.x)
    gmax = float(np.abs(g).max())
    cand = np.flatnonzero(np.abs(g) >= 1e-3 * gmax)
    fd_cells = np.sort(np.random.default_rng(P.extra["fd_seed"]).choice(cand, size=P.extra["n_fd"],
                                                                       replace=False))
    idx = np.sort(np.random.default_rng(7).choice(P.n, size=256, replace=False))
    rec = dict(J=J, grad_norm=float(np.linalg.norm(g)), grad_max=gmax, fd_cells=fd_cells.tolist(),
               grad_fd_cells=g[fd_cells].tolist(), sample_idx=idx.tolist(), grad_sample=g[idx].tolist(),
               p_sample=p[idx].tolist(), pobs_sample=pobs_full[idx].tolist(),
               iterations=dict(p=res.iterations, pobs=None, lam=lam_res.iterations), tol=tol)
    with open(os.path.join(HERE, "c5_adjoint.json"), "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print("c5", J, res.iterations, lam_res.iterations, gmax)


def c4_record():
    """128^3 precision workload: the oracle's PCG solution at the workload's
    tolerance (1e-8) and a tight reference (1e-12), as norms and values at
    256 seeded cells, with the iteration counts."""
    P = make_config("c4")
    part, _ = partition_blocks(P.dims, P.partition[1])
    pre = AlgMortarCPU(P.A, part)
    As = P.A.to_scipy()
    idx = np.sort(np.random.default_rng(7).choice(P.n, size=256, replace=False))
    res = pcg(lambda v: As @ v, P.b, pre.apply, P.tol)
    tight = pcg(lambda v: As @ v, P.b, pre.apply, 1e-12)
    rec = dict(sample_idx=idx.tolist(), iterations=res.iterations, x_sample=res.x[idx].tolist(),
               x_norm2=float(np.linalg.norm(res.x)), true_rel_res=res.true_rel_res, tol=P.tol,
               tight_iterations=tight.iterations, tight_x_sample=tight.x[idx].tolist(),
               tight_x_norm2=float(np.linalg.norm(tight.x)),
               err_vs_tight=float(np.linalg.norm(res.x - tight.x) / np.linalg.norm(tight.x)))
    with open(os.path.join(HERE, "c4_pcg.json"), "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print("c4", res.iterations, tight.iterations, rec["err_vs_tight"])


FULL_SAMPLE_SEED = 17
FULL_SAMPLE = 4096
FULL_APPLY_SEEDS = (101, 102, 103)
FULL_C3_COLUMNS = (0, 5, 15)


def full_record(name):
    """Oracle applies and tol-1e-10 PCG solutions of a large workload at full
    size, sampled at FULL_SAMPLE seeded cells (see the module docstring)."""
    import time
    P = make_config(name)
    if P.partition[0] == "blocks":
        part, _ = partition_blocks(P.dims, P.partition[1])
    else:
        _, lo, hi, seed = P.partition
        part, _ = partition_bisect(P.A.row_ptr, P.A.col, P.A.val, P.n, lo, hi, seed)
    t0 = time.time()
    pre = AlgMortarCPU(P.A, part)
    print(name, "oracle set-up", round(time.time() - t0), "s", flush=True)
    As = P.A.to_scipy()
    idx = np.sort(np.random.default_rng(FULL_SAMPLE_SEED).choice(P.n, size=FULL_SAMPLE, replace=False))
    cols = FULL_C3_COLUMNS if P.b.ndim == 2 else (None,)
    rhs = [P.b if c is None else P.b[:, c] for c in cols]
    vecs, labels = list(rhs), [f"b{'' if c is None else c}" for c in cols]
    for sd in (FULL_APPLY_SEEDS if P.b.ndim == 1 else FULL_APPLY_SEEDS[:1]):
        vecs.append(np.random.default_rng(sd).standard_normal(P.n))
        labels.append(f"normal{sd}")
    out = dict(sample_idx=idx.astype(np.int64), apply_labels=np.array(labels),
               rhs_columns=np.array([-1 if c is None else c for c in cols], dtype=np.int64))
    za = []
    for v in vecs:
        z = pre.apply(v)
        za.append((z[idx], np.linalg.norm(z), np.abs(z).max()))
    out["apply_sample"] = np.array([a[0] for a in za])
    out["apply_norm"] = np.array([a[1] for a in za])
    out["apply_maxabs"] = np.array([a[2] for a in za])
    print(name, "applies done", flush=True)
    xs, its, nrm, mx, trr = [], [], [], [], []
    for b in rhs:
        t0 = time.time()
        res = pcg(lambda v: As @ v, b, pre.apply, 1e-10)
        print(name, "pcg 1e-10", res.iterations, res.true_rel_res, round(time.time() - t0), "s", flush=True)
        xs.append(res.x[idx])
        its.append(res.iterations)
        nrm.append(np.linalg.norm(res.x))
        mx.append(np.abs(res.x).max())
        trr.append(res.true_rel_res)
    out.update(x_sample=np.array(xs), iterations=np.array(its, dtype=np.int64),
               x_norm=np.array(nrm), x_maxabs=np.array(mx), true_rel_res=np.array(trr),
               tol=np.float64(1e-10))
    if name == "c2":
        ref = pcg(lambda v: As @ v, rhs[0], pre.apply, 1e-13)
        print(name, "pcg 1e-13", ref.iterations, ref.true_rel_res, flush=True)
        out.update(ref_x_sample=ref.x[idx][None, :], ref_iterations=np.array([ref.iterations]),
                   ref_x_norm=np.array([np.linalg.norm(ref.x)]), ref_tol=np.float64(1e-13))
    np.savez(os.path.join(HERE, f"full_{name}.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["structure", "c2", "c5", "c4"]
    for name in ("c2", "c4", "c3"):
        if f"full_{name}" in which:
            full_record(name)
    if "structure" in which:
        main()
    if "c2" in which:
        c2_record()
    if "c5" in which:
        c5_record()
    if "c4" in which:
        c4_record()
