"""FP64 CPU oracle of the eMAGPIE epoch: test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP product path never imports or calls it.
"""
from . import emagpie_oracle  # noqa: F401
