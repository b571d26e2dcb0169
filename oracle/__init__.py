"""FP64 CPU oracle for the ACE build — test infrastructure, not product code.

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package.  It imports nothing from the HIP package.
"""
from . import ace_oracle  # noqa: F401
from . import scdm_oracle  # noqa: F401
