"""CPU oracle of the hot-electron particle-in-cell step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  It wraps `pic_oracle.c` (plain FP64 C) through ctypes and never touches the
device library.
"""
from .oracle import build, run, philox, OracleResult, NCOUNTERS, COUNTER_NAMES  # noqa: F401
