"""The oracle reproduces the stored index structure (tests/golden/structure.json,
written by tests/golden/make_golden.py) and the stored 2-D PCG record."""
import json
import os

import numpy as np
import pytest

from workloads import make_config
from oracle import partition_blocks, AlgMortarCPU, pcg

HERE = os.path.dirname(os.path.abspath(__file__))
import importlib.util

_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
make_golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(make_golden)


with open(os.path.join(HERE, "golden", "structure.json")) as f:
    GOLD = json.load(f)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_structure_hashes(name):
    rec = make_golden.structure_record(make_config(name))
    assert rec == GOLD[name]


def test_c1_pcg_record():
    with open(os.path.join(HERE, "golden", "c1_pcg.json")) as f:
        gold = json.load(f)
    P = make_config("c1")
    part, _ = partition_blocks(P.dims, P.partition[1])
    pre = AlgMortarCPU(P.A, part)
    As = P.A.to_scipy()
    res = pcg(lambda v: As @ v, P.b, pre.apply, P.tol)
    assert res.iterations == gold["iterations"]
    assert np.isclose(np.linalg.norm(res.x), gold["x_norm2"], rtol=1e-12)
