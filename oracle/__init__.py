"""CPU FP64 oracle for the DPDE VV+SER step (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never uses it.
"""
from .oracle import *  # noqa: F401,F403
