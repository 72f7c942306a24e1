"""MI355X-native BCCB LASSO solvers for single-snapshot 2D harmonic recovery.

The compute path lives in the HIP shared library built from ``csrc/`` and is
reached through the thin ctypes binding in :mod:`paper_2509_13592_amd.bccb`.
Importing this package does not load the library; importing ``bccb`` does,
and fails loudly when the library has not been built.
"""

__all__ = ["scenes"]
