"""MI355X-native polynomial preconditioned Arnoldi (arXiv:1806.08020).

The hot path runs in ``libppa.so`` (hand-written HIP for gfx950 behind a C
ABI, see ``include/ppa.h``); ``paper_1806_08020_amd.ppa`` is the thin ctypes
binding.  ``paper_1806_08020_amd.workloads`` builds seeded synthetic inputs.
Importing the package itself loads nothing.
"""
__version__ = "0.1.0"
