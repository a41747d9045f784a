"""Plain CPU FP64 reference (the oracle) for the H-LU path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the CPU-baseline leg of the benchmark may import anything from here; the
device library never calls it and never falls back to it.  It shares no code
with the device path: only the seeded input generators in ``hlu_inputs``
serve both.

Parity status of each function is stated in its docstring; functions without
an independent pin say "parity unpinned".
"""
from .hlu import *  # noqa: F401,F403
