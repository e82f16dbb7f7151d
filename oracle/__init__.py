"""Plain FP64 CPU oracle for polynomial preconditioned Arnoldi.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(``paper_1806_08020_amd``); the only common module is the seeded input
generator ``paper_1806_08020_amd.workloads``, which holds no part of the
method's arithmetic.

The oracle follows Embree, Loe & Morgan, "Polynomial Preconditioned Arnoldi"
(arXiv:1806.08020), step by step and in the paper's notation, using NumPy /
SciPy library routines (dense eig, solve, QR, CSR mat-vec) as single steps.
It is slow and obviously correct by construction; every function cites the
passage it follows.  See ``oracle/ppa_oracle.py``.
"""
from .ppa_oracle import *  # noqa: F401,F403
