"""Seeded synthetic inputs for the AlgMortar-PCG path.

This package builds the *inputs* of the method only: permeability fields,
grid geometry, the TPFA face list, the assembled sparse matrix ``A`` and
right-hand sides.  It contains none of the preconditioner's arithmetic
(partition, interfaces, local operators, basis functions, interface system,
Krylov iteration); those live independently in ``oracle/`` (CPU checker) and
in the HIP library.  Both sides draw their inputs from here.

The paper states its problem as ``A p = f`` with ``A`` SPD and nonpositive
off-diagonals (Sec. 3, eq. linear-system); the workloads below are
cell-centred TPFA discretizations of single-phase Darcy flow (Sec. 2 and the
experiments of Sec. 7), with synthetic fields standing in for the paper's
datasets.
"""
from .fields import grf, layered_log10k
from .grids import cartesian_faces, distorted_hex_faces, cell_index
from .tpfa import Faces, assemble, CSR
from .configs import Problem, make_config, CONFIG_NAMES

__all__ = [
    "grf", "layered_log10k", "cartesian_faces", "distorted_hex_faces",
    "cell_index", "Faces", "assemble", "CSR", "Problem", "make_config",
    "CONFIG_NAMES",
]
