"""FP64 CPU oracle for the matched-filter hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain definition of what
the HIP path computes, written from the paper (Chung et al., "Application of
GPUs to Search Pipeline for Gravitational Waves from Coalescing Binaries",
arXiv:0906.4175) and the literature it cites for the template.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.  The
product library never calls it and shares no code, constants or helpers with it.

Every function states the passage it follows.  Points where the paper is
silent or ambiguous take an explicit reading; the readings are listed in the
module docstring of :mod:`oracle.mf_oracle`.

Functions without an independent pin: none (the SPA coefficients are pinned
through the stationary-phase time/frequency relation against an independently
written chirp-time polynomial; see the test suite).
"""
from .mf_oracle import *  # noqa: F401,F403
