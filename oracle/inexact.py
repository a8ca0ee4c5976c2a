"""AlgMortar with an inexact interface solve (test infrastructure, FP64).

Sec. 6 offers two ways to solve the interface system of Algorithm 2: a
direct factorization, or PCG with a block-Jacobi preconditioner stopped at a
loose relative residual; Sec. 7 uses the latter with relative tolerance 1e-2
throughout.  This module is the plain form of that option:

* ``eta`` solves ``S eta = b`` approximately by PCG (``oracle.pcg``: zero
  initial guess, Fletcher-Reeves beta, stop when the recursive residual
  satisfies ``||r||_2 <= rtol ||b||_2``, at most ``maxit`` iterations);
* the preconditioner is block Jacobi on S: the basis functions, in their
  lexicographic ``(i, j)`` numbering, are cut into contiguous blocks, and
  each diagonal block ``S[K, K]`` is solved exactly (dense Cholesky);
* everything else is the exact apply of ``AlgMortarCPU`` (local solves,
  interface right-hand side, reconstruction).

Readings (the paper states neither): blocks of ``block_rows`` consecutive
basis functions (the last one shorter); the outer PCG around this
preconditioner uses the flexible Polak-Ribiere beta (``pcg(..., beta="pr")``),
because an inner solve stopped by a tolerance makes the preconditioner
depend on its argument.
"""
import numpy as np
import scipy.linalg as sla

from .pcg import pcg


class BlockJacobiS:
    """``z = blockdiag(S[K, K])^{-1} r`` over contiguous blocks of rows."""

    def __init__(self, S, block_rows):
        S = S.tocsr()
        n = S.shape[0]
        self.bounds = [(a, min(n, a + block_rows)) for a in range(0, n, block_rows)]
        self.factors = []
        for a, e in self.bounds:
            blk = S[a:e][:, a:e].toarray()
            self.factors.append(sla.cho_factor(blk, lower=True))

    def __call__(self, r):
        z = np.empty_like(r)
        for (a, e), f in zip(self.bounds, self.factors):
            z[a:e] = sla.cho_solve(f, r[a:e])
        return z


class InexactAlgMortarCPU:
    """AlgMortar apply with ``eta`` from block-Jacobi PCG on S (see module
    docstring).  ``base``: a set-up ``AlgMortarCPU``; ``rtol``: inner relative
    tolerance (0 runs exactly ``maxit`` inner iterations unless the residual
    vanishes); ``block_rows``: rows per block-Jacobi block."""

    def __init__(self, base, rtol=1e-2, maxit=50, block_rows=64):
        self.base = base
        self.rtol = float(rtol)
        self.maxit = int(maxit)
        self.S = base.S.tocsr()
        self.bj = BlockJacobiS(self.S, block_rows)
        self.inner_iterations = []

    def solve_S(self, b):
        if not np.any(b):
            self.inner_iterations.append(0)
            return np.zeros_like(b)
        tol = self.rtol if self.rtol > 0 else 1e-300
        res = pcg(lambda v: self.S @ v, b, self.bj, tol, maxit=self.maxit)
        self.inner_iterations.append(res.iterations)
        return res.x

    def apply(self, r):
        base = self.base
        r = np.asarray(r, dtype=np.float64)
        pbar = base.local_solves(r)
        b = base.interface_rhs(pbar)
        eta = self.solve_S(b)
        return base.reconstruct(pbar, eta)
