"""SMASH (arXiv 1705.05443) H^2 / HSS construction and product on MI355X.

The compute path is the HIP library ``libsmash.so`` (built from ``csrc/``),
reached through its C ABI (``include/smash.h``).  ``api`` is a thin ctypes
binding: it marshals torch device tensors into pointers and nothing else.
Importing the package loads nothing; ``api`` loads the library on first use
and raises if it is missing.
"""

__all__ = ["api", "workloads"]
