"""Preconditioned conjugate gradients (paper Sec. 5: AlgMortar is used as the
PCG preconditioner; Sec. 7: zero initial guess, stop on the relative residual
in the Euclidean norm).

The paper does not state its beta formula or iteration cap.  Readings:
Fletcher-Reeves ``beta = (r_new, z_new) / (r, z)`` (the textbook choice for an
exactly symmetric preconditioner), the Polak-Ribiere variant
``beta = (r_new - r, z_new) / (r, z)`` when ``beta="pr"``, a stop when the
recursive residual satisfies ``||r||_2 <= tol * ||b||_2``, and ``maxit``
10000.
"""
from dataclasses import dataclass

import numpy as np


class BreakdownError(RuntimeError):
    pass


@dataclass
class PCGResult:
    x: np.ndarray
    iterations: int
    rel_res: float          # recursive residual / ||b||
    true_rel_res: float     # ||b - A x|| / ||b||
    converged: bool
    history: list


def pcg(matvec, b, precond, tol, maxit=10000, beta="fr", x0=None):
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = np.array(x0, dtype=np.float64)
        r = b - matvec(x)
    hist = [float(np.linalg.norm(r))]
    if bnorm == 0.0:
        return PCGResult(x, 0, 0.0, 0.0, True, hist)
    if hist[0] <= tol * bnorm:
        return PCGResult(x, 0, hist[0] / bnorm, hist[0] / bnorm, True, hist)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    if not rz > 0:
        raise BreakdownError("(r, z) <= 0")
    its = 0
    converged = False
    for it in range(1, maxit + 1):
        q = matvec(p)
        pq = float(p @ q)
        if not pq > 0:
            raise BreakdownError("(p, Ap) <= 0")
        alpha = rz / pq
        x += alpha * p
        r_old = r
        r = r - alpha * q
        its = it
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= tol * bnorm:
            converged = True
            break
        z = precond(r)
        rz_new = float(r @ z)
        if beta == "fr":
            bt = rz_new / rz
        else:
            bt = (rz_new - float(r_old @ z)) / rz
        if not rz_new > 0:
            raise BreakdownError("(r, z) <= 0")
        p = z + bt * p
        rz = rz_new
    true_res = float(np.linalg.norm(b - matvec(x))) / bnorm
    return PCGResult(x, its, hist[-1] / bnorm, true_res, converged, hist)
