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


if __name__ == "__main__":
    main()
    c2_record()
