"""Plain FP64 CPU oracle for equispaced-Fourier GP regression (EFGP).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls,
links or executes anything under this directory: only the test suite, the
smoke check and the CPU-baseline leg of the benchmark do.  The oracle shares
no code with the GPU library.

Every function cites the passage of the paper (Greengard, Rachh, Barnett,
"Equispaced Fourier representations for efficient Gaussian process
regression from a billion data points", arXiv 2210.10210) that it follows.
Direct O(N*M) exponential sums live in ``efgp_direct.c``; the rest is numpy /
scipy in float64.
"""
from .efgp import *  # noqa: F401,F403
