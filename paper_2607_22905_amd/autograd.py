"""Differentiation form: a TPFA Darcy solve ``A(theta) p = f(theta) + q``,
``theta = ln K``, with AlgMortar-PCG forward and a hand-written adjoint
backward, exposed as a ``torch.autograd.Function``.

Forward: the device assembles ``A(theta)`` and the Dirichlet part of ``f``
(``am_tpfa_assemble``), sets up AlgMortar on it (Algorithm 1) and solves with
PCG (Sec. 5).  Backward: the adjoint system ``A lambda = dJ/dp`` is solved
with the same handle (``A`` is symmetric), and a per-cell face gather turns
``p`` and ``lambda`` into ``dJ/dtheta`` (``algmortar_adjoint_grad``).  Only
argument marshalling happens here; every step runs in the HIP library.
"""
import numpy as np

from .solver import AlgMortar, Tpfa, adjoint_grad

__all__ = ["DarcyModel", "AlgMortarSolve"]


class DarcyModel:
    """Fixed grid, partition and sources; the permeability is the input.

    faces: face list with arrays ``k, l, gk, gl, pD`` (``l = -1`` marks a
    Dirichlet face); n: cells; part/nparts: the partition; source: host
    float64[n] or None (``q``); tol / adjoint_tol: PCG tolerances of the
    forward and adjoint solves; reuse_handle: keep one AlgMortar handle and
    give it each new permeability's values (``update_values``: the numeric
    set-up only) instead of setting up a new handle per solve."""

    def __init__(self, faces, n, part, nparts, source=None, tol=1e-10, adjoint_tol=1e-12,
                 prec="fp64", maxit=10000, device=0, reuse_handle=False):
        import torch
        self.n = int(n)
        self.part = np.ascontiguousarray(part, dtype=np.int32)
        self.nparts = int(nparts)
        self.tol = float(tol)
        self.adjoint_tol = float(adjoint_tol)
        self.prec = prec
        self.maxit = int(maxit)
        self.device = torch.device("cuda", device)
        self.tpfa = Tpfa(faces, self.n, device)
        self.source = None
        if source is not None:
            self.source = torch.as_tensor(np.ascontiguousarray(source, dtype=np.float64),
                                          device=self.device)
        self.last_info = None
        self.reuse_handle = bool(reuse_handle)
        self._h = None
        # which forward's values the shared handle holds: a forward stamps
        # its solve with a new token; a backward whose token differs puts its
        # own values back first (several forwards before one backward)
        self._h_token = None
        self._next_token = 0

    def assemble(self, logK):
        """(matrix view for AlgMortar, right-hand side f + q) on the device."""
        val, f = self.tpfa.assemble(logK)
        if self.source is not None:
            f = f + self.source
        return self.tpfa.matrix(val), f

    def forward_solve(self, logK):
        """(p, handle): the handle keeps the factored preconditioner for the
        adjoint solve; the caller closes it, unless the model reuses its
        handle (then ``close`` of the model does)."""
        A, f = self.assemble(logK)
        if self.reuse_handle and self._h is not None:
            self._h.update_values(A)
            h = self._h
        else:
            h = AlgMortar(A, self.part, self.nparts, prec=self.prec)
            if self.reuse_handle:
                self._h = h
        if self.reuse_handle:
            self._next_token += 1
            self._h_token = self._next_token
        p, info, _ = h.pcg(f, self.tol, maxit=self.maxit)
        self.last_info = info[0]
        return p, h

    def handle_for(self, logK, token):
        """The handle holding the values of the forward stamped ``token``
        (on a shared handle: put back with ``update_values`` if a later
        forward replaced them)."""
        if self.reuse_handle and self._h_token != token:
            A, _ = self.assemble(logK)
            self._h.update_values(A)
            self._h_token = token
        return self._h

    def close(self):
        if self._h is not None:
            self._h.close()
            self._h = None
        self.tpfa.close()


class AlgMortarSolve:
    """``p = AlgMortarSolve.apply(logK, model)``: differentiable in ``logK``
    (a float64 CUDA tensor of shape (n,))."""

    _fn = None

    @classmethod
    def apply(cls, logK, model):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(logK, model)


def _make_function():
    import torch

    class _Solve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, logK, model):
            logK = logK.detach().contiguous()
            p, h = model.forward_solve(logK)
            ctx.save_for_backward(logK, p)
            ctx.model = model
            ctx.handle = h
            ctx.token = model._h_token
            return p

        @staticmethod
        def backward(ctx, grad_p):
            logK, p = ctx.saved_tensors
            model, h = ctx.model, ctx.handle
            if model.reuse_handle:
                # a later forward may have given the shared handle its values
                h = model.handle_for(logK, ctx.token)
            try:
                g, lam, info = adjoint_grad(h, model.tpfa, logK, p, grad_p.contiguous(),
                                            tol=model.adjoint_tol, maxit=model.maxit)
                model.last_adjoint_info = info
            finally:
                if not model.reuse_handle:
                    h.close()
                ctx.handle = None
            return g, None

    return _Solve
