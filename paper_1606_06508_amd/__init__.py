"""Floater-Hormann barycentric rational interpolation on MI355X (gfx950).

The compute path is the HIP library ``libfh.so`` behind the C ABI declared in
``include/fh.h``; ``paper_1606_06508_amd.fh`` is the thin ctypes binding to it
(argument marshalling only).  Importing this package loads nothing; the
library is opened on first use and a missing library is an error, never a
fallback.
"""
__all__ = ["fh", "inputs"]
