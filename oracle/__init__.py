"""FP64 CPU oracle for the Floquet-operator build.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, links or
executes this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do. It shares no code with the HIP path.
"""
from .floquet_oracle import *  # noqa: F401,F403
