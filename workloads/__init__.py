"""Seeded synthetic atomistic block-sparse operators and dense multi-vectors.

This package only *generates inputs*: atom positions, species, neighbour
graphs, block values and random multi-vectors.  It performs none of the
operator arithmetic (no products, no transposes, no moments); that lives in
the device library and, independently, in ``oracle/``.  Both sides consume
what is generated here.

Block convention (the reading used throughout): atom ``i`` carries ``b_i``
orbitals, so the coupling of atoms ``i`` and ``j`` is a dense ``b_i x b_j``
block (the paper's block model, section 2.1).  Blocks are stored in graph
(CSR) order, each block row-major, columns sorted ascending inside a row.

Every operator is symmetric (``A_ji = A_ij^T``, self blocks symmetric).  The
random draw order is fixed: positions -> species permutation -> block values
(upper blocks ``i <= j`` in ascending ``(i, j)``, a self block drawing only its
upper triangle row by row) -> multi-vectors.
"""
from .core import (Operator, random_cube, sc_lattice, zincblende_sphere,
                   random_pattern, multivector, inf_norm_scale)
from .configs import make_config, CONFIG_NAMES

__all__ = ["Operator", "random_cube", "sc_lattice", "zincblende_sphere",
           "random_pattern", "multivector", "inf_norm_scale", "make_config",
           "CONFIG_NAMES"]
