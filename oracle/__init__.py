"""FP64 CPU oracle for AlgMortar-PCG -- TEST INFRASTRUCTURE ONLY.

A plain, slow, deliberately unoptimised implementation of what the GPU
library computes, written from the paper (AlgMortar: a fully algebraic
multiscale mortar preconditioner), used to check the HIP path.  Only the test
suite, the package's smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does.  It shares no code with the HIP
library; both take their inputs from ``workloads``.

Modules
-------
partition  graph partition (block and recursive-bisection rules) -- Sec. 3.1
structure  permutation, interface edge sets E_ij, interface numbering -- Sec. 3.1-3.2
algmortar  local operators A_i, Cholesky, MBFs, interface matrix S, apply
           -- Sec. 3.3-3.4, Algorithms 1 and 2
pcg        preconditioned conjugate gradients -- Sec. 5, Sec. 7 set-up
smoothing  block-Jacobi pre/post smoothing around AlgMortar -- Sec. 5.4
adjoint    adjoint gradient dJ/dlog K of a least-squares loss (no paper analogue)
dense      dense matrices of the operators for small-case identities -- Sec. 3-5

Pins: every function is checked in ``tests/test_oracle_*.py`` against what the
paper and the mathematics fix (identities, closed forms, special cases that
reduce to a direct solve, spectral bounds, finite differences).
"""
from .partition import partition_blocks, partition_bisect, splitmix64
from .structure import build_structure, Structure
from .algmortar import AlgMortarCPU, NotSPDError
from .pcg import pcg, PCGResult
from . import adjoint, dense

__all__ = [
    "partition_blocks", "partition_bisect", "splitmix64", "build_structure",
    "Structure", "AlgMortarCPU", "NotSPDError", "pcg", "PCGResult", "adjoint",
    "dense",
]
