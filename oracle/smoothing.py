"""Block-Jacobi pre- and post-smoothing around the AlgMortar correction
(Sec. 5.4) -- TEST INFRASTRUCTURE ONLY (part of the FP64 CPU oracle).

Sec. 5.4 observes that the residual left by an AlgMortar correction lives on
cells next to the partition interface only, and damps it with block-Jacobi
steps, the same number before and after the correction so that the
preconditioner stays symmetric.  Readings where the paper is silent:

* the smoother is textbook block Jacobi: ``B = blockdiag(A[K, K])`` over a
  partition of the unknowns into blocks ``K`` (typically unions of several
  AlgMortar subdomains), each block solved exactly (the paper runs PETSc's
  block Jacobi with its default settings and sets only the number of blocks);
* one smoothing step is ``z <- z + B^{-1} (r - A z)``;
* the smoothed preconditioner applied to ``r`` starts from ``z = 0``, takes
  ``nu`` steps, the correction ``z <- z + Mcal^{-1} (r - A z)`` and ``nu``
  more steps (multiplicative composition).
"""
import numpy as np
import scipy.sparse.linalg as spla


class BlockJacobi:
    """``B^{-1}`` for ``B = blockdiag(A[K, K])``, every block factored by a
    sparse direct solver.  ``As``: scipy sparse matrix; ``blocks``: block id
    of every unknown, ids ``0 .. nblocks-1``, none empty."""

    def __init__(self, As, blocks):
        self.As = As.tocsr()
        self.blocks = np.asarray(blocks, dtype=np.int64)
        nb = int(self.blocks.max()) + 1
        self.idx = [np.flatnonzero(self.blocks == b) for b in range(nb)]
        if any(ix.size == 0 for ix in self.idx):
            raise ValueError("empty smoothing block")
        self.lu = [spla.splu(self.As[ix][:, ix].tocsc()) for ix in self.idx]

    def solve(self, r):
        r = np.asarray(r, dtype=np.float64)
        out = np.zeros_like(r)
        for ix, lu in zip(self.idx, self.lu):
            out[ix] = lu.solve(np.ascontiguousarray(r[ix]))
        return out


def smoothed_apply(As, bj, correction, nu, r):
    """``z = M^{-1} r`` of the symmetric multiplicative composition: ``nu``
    block-Jacobi steps, the correction ``correction`` (a function, e.g.
    ``AlgMortarCPU.apply``), ``nu`` block-Jacobi steps, from ``z = 0``.
    ``r`` may hold several columns (shape (n, k))."""
    r = np.asarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    for _ in range(nu):
        z = z + bj.solve(r - As @ z)
    z = z + correction(r - As @ z)
    for _ in range(nu):
        z = z + bj.solve(r - As @ z)
    return z


class SmoothedAlgMortarCPU:
    """AlgMortar with ``nu`` block-Jacobi steps before and after it."""

    def __init__(self, am, blocks, nu):
        self.am = am
        self.As = am.As
        self.bj = BlockJacobi(am.As, blocks)
        self.nu = int(nu)

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        if r.ndim == 2:
            return np.stack([self.apply(r[:, k]) for k in range(r.shape[1])], axis=1)
        return smoothed_apply(self.As, self.bj, self.am.apply, self.nu, r)
