"""FP64 CPU oracle of the pseudo-transient NPB solver (Wilson & Zhao).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import or run anything in
this package.  It shares no code with the HIP library and never imports it.
"""
from .npb import *  # noqa: F401,F403
