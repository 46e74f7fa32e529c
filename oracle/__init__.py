"""FP64 CPU oracle of the EMC iteration -- test infrastructure, not product code.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library.
"""
from .emc_oracle import *  # noqa: F401,F403
