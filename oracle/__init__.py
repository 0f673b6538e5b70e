"""FP64 CPU oracle for CoNCPD-APG / lraCoNCPD-APG (test infrastructure only).

Only tests, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  Parity status of each function is recorded in the
module docstrings; every function here is pinned by the CPU test-suite
(``pytest -m "not gpu"``) against brute force, closed forms or invariants.
"""
from . import apg, tucker  # noqa: F401
