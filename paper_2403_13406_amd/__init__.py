"""eslb: fourth-order entropy-stable lattice Boltzmann time loop on MI355X (gfx950).

Method: Bellotti, Helluy, Navoret, "Fourth-order entropy-stable lattice
Boltzmann schemes for hyperbolic systems" (arXiv 2403.13406).  The compute path
is libeslb.so (hand-written HIP, C ABI in include/eslb.h); this package only
marshals arguments.  Importing it does not load the library; the first Solver
does, and raises if the library is missing (there is no CPU fallback).
"""
from .batch import Batch  # noqa: F401
from .solver import EslbError, Solver, make_problem  # noqa: F401
