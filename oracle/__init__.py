"""Plain, slow complex128 CPU oracle for the multi-RHS coarse operator and block CG.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only the tests, the smoke check of the entry module and the CPU-baseline leg
of the benchmark may call it. It shares no code with the HIP library; the two
meet only through the seeded input generators in ``workloads``.
"""
from .coarse_oracle import *  # noqa: F401,F403
