"""Plain FP64 CPU oracle of the hybrid-PIC step (Morris, Robinson & Ridgers,
arXiv 2107.01723).  TEST INFRASTRUCTURE ONLY.

This package is the checker, not the product.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the HIP path: it has its own constants, its own Philox generator,
its own cross-section tables and its own physics, written in SI units and
FP64 with NumPy, processing particles in id order.  Each function cites the
passage of the paper it restates.

Parts whose absolute values no closed form, printed number or invariant can
fix are marked "parity unpinned" in their docstrings: the ionisation state
Z* (More's Thomas-Fermi fit, cited but not given by the paper), the Coulomb
logarithm (Lee-More, cited but not given) and therefore the absolute
resistivity.  Their invariants (limits, monotonicity, Spitzer scaling) are
still pinned.
"""
from . import constants, philox, tables, solid, fields, particles, run  # noqa: F401
from .run import OracleRun  # noqa: F401
