"""FP64 CPU oracle for BCFW on quadratic semi-relaxed OT (arXiv:2103.05857).

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU library never does.
"""
from .oracle import *  # noqa: F401,F403
