"""The autotuner's persisted choices (ALGMORTAR_AUTOTUNE_CACHE): two fresh
processes solve the same 8-column system on the bisection grid (three
candidate wave layouts of the vector-unit tile kernel; 16 columns run the
matrix-core kernels, which have one layout); the first times the layouts and
records its choice,
the second reads it and times nothing; their solutions are equal bit for
bit (the layouts differ in the order partial vectors are added, so without
the record two processes could differ in the last bits)."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import sys, json
sys.path.insert(0, {root!r})
import numpy as np, torch
import paper_2607_22905_amd as am
from tests.test_gpu_parity import _case
A, part, m, b = _case("bisect")
h = am.AlgMortar(A, part, m, max_nrhs=8)
R = np.random.default_rng(5).standard_normal((8, A.n))
X, info, _ = h.pcg(torch.as_tensor(R, device="cuda:0"), 1e-10)
ch, us = h.tile_choice(8)
np.save({out!r}, X.cpu().numpy())
print(json.dumps({{"choice": ch, "us": us}}))
h.close()
'''


def _run(tmp_path, tag, cache):
    out = str(tmp_path / f"x_{tag}.npy")
    env = dict(os.environ, ALGMORTAR_AUTOTUNE_CACHE=cache)
    env.pop("ALGMORTAR_TILE", None)
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, out=out)], env=env,
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    import json
    return np.load(out), json.loads(r.stdout.strip().splitlines()[-1])


def test_two_processes_bitwise_equal(tmp_path):
    cache = str(tmp_path / "autotune.txt")
    x1, i1 = _run(tmp_path, "first", cache)
    lines = open(cache).read().split()
    assert len(lines) >= 2 and int(lines[1]) == i1["choice"]
    assert any(u > 0 for u in i1["us"])  # the first process timed the layouts
    x2, i2 = _run(tmp_path, "second", cache)
    assert i2["choice"] == i1["choice"] and all(u == 0 for u in i2["us"])
    assert np.array_equal(x1, x2)


def test_sixteen_columns_one_layout():
    """16 columns with the interface solve as its own launches run the
    matrix-core kernels in both window buckets: one layout, nothing timed."""
    import torch  # noqa: F401
    sys.path.insert(0, ROOT)
    import paper_2607_22905_amd as am
    from tests.test_gpu_parity import _case
    A, part, m, b = _case("bisect")
    h = am.AlgMortar(A, part, m, max_nrhs=16, separate_iface=True)
    ch, us = h.tile_choice(16)
    assert ch == 0 and us == [0.0]
    h.close()


def test_one_column_bf16_products_one_layout():
    """One column under BF16 x BF16 products, every subdomain in window 64
    and the interface solve as its own launches: the matrix-core kernel, one
    layout, nothing timed; without the flag the layouts are timed."""
    import torch  # noqa: F401
    sys.path.insert(0, ROOT)
    import paper_2607_22905_amd as am
    from tests.test_gpu_parity import _case
    A, part, m, b = _case("layered")
    h = am.AlgMortar(A, part, m, prec="bf16", separate_iface=True, bf16_products=True)
    ch, us = h.tile_choice(1)
    assert ch == 0 and us == [0.0]
    h.close()
    h = am.AlgMortar(A, part, m, prec="bf16", separate_iface=True)
    ch, us = h.tile_choice(1)
    assert len(us) > 1 and all(u > 0.0 for u in us)
    h.close()
