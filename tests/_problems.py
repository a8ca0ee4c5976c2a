"""Small seeded problems shared by the tests (built from ``workloads`` only)."""
import numpy as np

from workloads.configs import cartesian_problem
from workloads.fields import grf
from workloads.grids import cartesian_faces
from workloads.tpfa import Faces, assemble, CSR


def random_2d(nx=8, ny=8, sigma=1.0, seed=0, dirichlet=((0, 0, 0.0),), block=(4, 4, 1)):
    g = grf((ny, nx), 2.0, sigma, seed) if sigma > 0 else np.zeros((ny, nx))
    return cartesian_problem("t2d", nx, ny, 1, g, list(dirichlet), None, block, 1e-12)


def random_3d(nx=6, ny=6, nz=4, sigma=1.0, seed=0, block=(3, 3, 2),
              dirichlet=((0, 0, 1.0), (0, 1, 0.0))):
    g = grf((nz, ny, nx), 2.0, sigma, seed) if sigma > 0 else np.zeros((nz, ny, nx))
    return cartesian_problem("t3d", nx, ny, nz, g, list(dirichlet), None, block, 1e-12)


def chain(n=12, seed=0, dirichlet_left=True):
    """1-D chain of cells (a 1 x n grid) with random K."""
    g = np.random.default_rng(seed).normal(size=n)
    faces = Faces.from_dict(cartesian_faces(n, 1, 1, [(0, 0, 0.0)] if dirichlet_left else []))
    A, f = assemble(faces, np.exp(g), n)
    return A, faces, g


def dense_csr(Ad):
    """CSR of a dense symmetric matrix (exact zeros dropped)."""
    n = Ad.shape[0]
    rows, cols = np.nonzero(Ad)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return CSR(n=n, row_ptr=row_ptr, col=cols.astype(np.int32), val=Ad[rows, cols].astype(np.float64))


def random_mmatrix(n, density, seed):
    """Random SPD M-matrix: random graph, negative couplings, diagonal
    = row sum of |couplings| + positive shift on a few rows."""
    rng = np.random.default_rng(seed)
    Ad = np.zeros((n, n))
    for k in range(n):
        for l in range(k + 1, n):
            if rng.random() < density or l == k + 1:
                w = rng.uniform(0.1, 10.0)
                Ad[k, l] = Ad[l, k] = -w
    d = -Ad.sum(axis=1)
    d[rng.choice(n, size=max(1, n // 5), replace=False)] += rng.uniform(0.5, 2.0)
    Ad[np.arange(n), np.arange(n)] = d
    return Ad
