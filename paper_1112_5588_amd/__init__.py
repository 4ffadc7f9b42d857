"""pJDS sparse matrix-vector multiplication for AMD Instinct MI355X (gfx950).

Implements the padded jagged diagonals storage format and its GPU product from Kreutzer et
al., "Sparse matrix-vector multiplication on GPGPU clusters: a new storage format and a
scalable implementation" (arXiv:1112.5588), with ELLPACK-R and CSR products beside it.
All arithmetic runs in the HIP kernels of ``libpjds.so``; this package only marshals
arguments (``_lib``) and keeps device arrays (``matrix``).
"""
from . import _lib
from ._lib import PjdsError
from .matrix import CsrMatrix, EllrMatrix, PjdsBatch, PjdsMatrix

__all__ = ["PjdsMatrix", "PjdsBatch", "EllrMatrix", "CsrMatrix", "PjdsError", "_lib"]
