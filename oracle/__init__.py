"""CPU FP64 oracle for the unaligned RKHS-mode CP-HIFI subproblem.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package.  The
library (``paper_2603_25691_amd``) never imports or calls it, and this package
imports nothing from the library: the two sides share only the seeded input
generators in ``synth``.
"""

from .cphifi_oracle import *  # noqa: F401,F403
from .cphifi_als import *  # noqa: F401,F403
