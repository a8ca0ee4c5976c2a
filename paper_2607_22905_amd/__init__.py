"""MI355X (gfx950) AlgMortar-PCG: the algebraic multiscale mortar preconditioner
inside a conjugate gradient solve, as hand-written HIP kernels behind a C-ABI
(include/algmortar.h).  This package is the thin Python binding.

The library must be built first (``python -m paper_2607_22905_amd.build``);
nothing here falls back to CPU code.
"""
from .solver import (AlgMortar, Tpfa, adjoint_grad, interface_nd, partition_blocks,
                     partition_bisect, structure, structure_sizes)
from ._lib import AlgMortarError, load
from .autograd import AlgMortarSolve, DarcyModel

__all__ = ["AlgMortar", "Tpfa", "adjoint_grad", "interface_nd", "partition_blocks", "partition_bisect",
           "structure", "structure_sizes", "AlgMortarError", "load", "AlgMortarSolve",
           "DarcyModel"]
