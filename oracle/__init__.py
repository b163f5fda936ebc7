"""CPU FP64 oracle for the spinor polarizability path.  TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library and never imports it.
"""
from .gw_oracle import *  # noqa: F401,F403

from .closure import *  # noqa: F401,F403

from .symmetry import *  # noqa: F401,F403
