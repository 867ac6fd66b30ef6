"""Named synthetic workloads shaped like the paper's operators.

The paper benchmarks periodic atom-centred graphs built with a finite
interaction cutoff (section 4, setup) and InP nanoparticles (section 5); its
inputs are not public, so these seeded stand-ins replace them:

* ``C1``  1,000 atoms, periodic cube, density 0.05/A^3, b in {4, 9} (500/500),
  cutoff 6 A (strict, self included), values U[-1,1]*exp(-r/2), nrhs 16.
* ``C2``  periodic 32^3 simple-cubic lattice, b = 13, self + 6 + 12 neighbours,
  values U[-1,1]*exp(-r), nrhs 1 and 32.
* ``C3``  zincblende sphere (a = 5.87 A, radius 104 A) with b = 13 cations,
  b = 9 anions, b = 1 passivating atoms, couplings closer than 5.37 A
  (through the third shell), values U[-1,1]*exp(-r), nrhs 64.
* ``C4``  the C2 operator divided by 1.01*||A||_inf, random block R (nrhs 64,
  seed 4): input of the degree-64 Chebyshev recurrence.
* ``C5``  100,000 atoms, density 0.05, b in {1, 4, 9} (20k/40k/40k), cutoff
  5 A, values as C1 rounded to FP32, nrhs 32, X and G drawn N(0,1).
* ``FD50`` 50 atoms in a 10 A periodic cube, b in {1, 4, 9} (10/20/20),
  cutoff 5 A, nrhs 32: the finite-difference instance.
* ``P8``  the paper's fixed-block (BSR) domain: 38,400 atoms, density 0.05,
  every b = 8, cutoff 5 A, values as C1 (about 510 MiB of FP64 values).
* ``G1``  the block-product (SpGEMM) operand: 11,520 atoms, density 0.05,
  b uniform over 9..20 (960 atoms each, the paper's variable-block range),
  cutoff 5 A, values as C1 (about 500 MiB of FP64 values, the storage the
  paper's kernel benchmarks target); the product is A A.

``scale`` < 1 shrinks an operator (atom count or lattice size) so the CPU
oracle finishes in seconds; the construction and draw order are unchanged.
"""
from __future__ import annotations

import numpy as np

from .core import (random_cube, sc_lattice, zincblende_sphere, multivector,
                   inf_norm_scale, scaled)

CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5", "FD50", "G1", "P8")
DEFAULT_NRHS = {"C1": 16, "C2": 32, "C3": 64, "C4": 64, "C5": 32, "FD50": 32, "G1": 16, "P8": 16}


def _round_counts(total, fracs):
    c = [int(round(total * f)) for f in fracs]
    c[-1] = total - sum(c[:-1])
    return c


def make_operator(name: str, scale: float = 1.0):
    """The operator of a named workload (``scale`` shrinks it)."""
    if name == "C1":
        n = max(8, int(round(1000 * scale)))
        return random_cube(n, 0.05, list(zip((4, 9), _round_counts(n, (0.5, 0.5)))),
                           6.0, 2.0, seed=1, name="C1")
    if name in ("C2", "C4"):
        m = 32 if scale >= 1.0 else max(3, int(round(32 * scale ** (1 / 3))))
        return sc_lattice(m, 13, seed=2, decay=1.0, name="C2")
    if name == "C3":
        radius = 104.0 * (scale ** (1 / 3) if scale < 1.0 else 1.0)
        return zincblende_sphere(radius, 5.87, 13, 9, 5.37, seed=3, name="C3")
    if name == "C5":
        n = max(30, int(round(100_000 * scale)))
        return random_cube(n, 0.05, list(zip((1, 4, 9), _round_counts(n, (0.2, 0.4, 0.4)))),
                           5.0, 2.0, seed=5, name="C5")
    if name == "FD50":
        # 50 atoms in a 10 A box: density 0.05
        return random_cube(50, 0.05, [(1, 10), (4, 20), (9, 20)], 5.0, 2.0,
                           seed=55, name="FD50", box=10.0)
    if name == "P8":
        n = max(60, int(round(38_400 * scale)))
        return random_cube(n, 0.05, [(8, n)], 5.0, 2.0, seed=8, name="P8")
    if name == "G1":
        n = max(60, int(round(11_520 * scale)) // 12 * 12)
        return random_cube(n, 0.05, [(bb, n // 12) for bb in range(9, 21)], 5.0, 2.0,
                           seed=7, name="G1")
    raise KeyError(name)


def make_config(name: str, scale: float = 1.0, nrhs: int | None = None):
    """Return ``(op, vectors)`` for a named workload.

    ``vectors`` holds ``X`` (and ``G`` for C5 and FD50, ``R`` for C4), FP64,
    row-major ``N x nrhs``, drawn after the operator's values in the fixed
    order.  C4 returns the already scaled operator; its R comes from seed 4.
    """
    nrhs = DEFAULT_NRHS[name] if nrhs is None else nrhs
    op = make_operator(name, scale)
    if name == "C4":
        s = inf_norm_scale(op)
        op = scaled(op, s, name="C4")
        R = np.random.default_rng(4).standard_normal((op.N, nrhs))
        return op, {"R": R}
    vec = {"X": multivector(op, nrhs)}
    if name in ("C5", "FD50"):
        vec["G"] = multivector(op, nrhs)
    return op, vec
