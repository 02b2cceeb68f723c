"""Independent FP64 CPU oracle of the randomized GSVD (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package; the HIP library never does, and this
package imports nothing from the library.
"""
from . import philox, rgsvd, mlp  # noqa: F401
