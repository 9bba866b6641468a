"""CPU FP64 oracle (test infrastructure only: imported by tests, the smoke check and the CPU-baseline leg of the benchmark)."""

from . import wfq_oracle  # noqa: F401
from .wfq_oracle import Problem  # noqa: F401
