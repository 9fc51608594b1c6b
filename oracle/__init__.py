"""FP64 CPU oracle of AWG-preconditioned CG.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and
the benchmark's CPU-baseline leg; never by the GPU library.
"""
from .awg_oracle import *  # noqa: F401,F403
