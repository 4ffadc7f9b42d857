"""Parity checks of a computed sparse product against the CPU oracle.

Two checks on the same seeded inputs:

* the relative L2 error of the whole result (1e-12 for binary64 arithmetic, 1e-5 for
  binary32), and
* a bound on every single row.  A sum of n products evaluated in floating point with unit
  roundoff u, in any order and with or without fused multiply-adds, differs from the exact
  sum by at most gamma_n * sum_k |a_k x_k|, gamma_n = n u / (1 - n u) (Higham, *Accuracy and
  Stability of Numerical Algorithms*, 2nd ed., Sect. 3.1, the dot-product bound and the
  remark that it holds for any order of evaluation).  The oracle's own binary64 result obeys
  the same bound with u = 2^-53, so the kernel's row i must lie within
  (gamma_{L_i}(u_kernel) + gamma_{L_i}(2^-53)) * sum_j |a_ij x_j| of it, L_i the number of
  stored entries of row i.  The sum of magnitudes is the oracle's product of |A| and |x|
  (rounded upwards by a factor 1 + 2 gamma to cover its own rounding).

A row that is off by more than its own bound fails even when the norm of the whole vector
hides it.  Rows may be sampled: ``rows`` lists the original rows whose results ``y`` holds.
"""
from __future__ import annotations

import numpy as np

import oracle
import synth

U64 = 2.0 ** -53
U32 = 2.0 ** -24
TOL = {8: 1e-12, 4: 1e-5}          # by the kernel's value size in bytes


def gamma(n, u: float) -> np.ndarray:
    n = np.asarray(n, dtype=np.float64)
    return n * u / (1.0 - n * u)


def sub_rows(A, rows) -> synth.CSR:
    """The rows ``rows`` of A (in that order) as a CSR matrix with A's columns."""
    rows = np.asarray(rows, dtype=np.int64)
    rp = np.asarray(A.row_ptr, np.int64)
    lens = rp[rows + 1] - rp[rows]
    new_rp = np.zeros(len(rows) + 1, np.int64)
    new_rp[1:] = np.cumsum(lens)
    idx = (np.repeat(rp[rows] - new_rp[:-1], lens) + np.arange(int(new_rp[-1]), dtype=np.int64)).astype(np.int64)
    return synth.CSR(len(rows), A.n_cols, new_rp, np.asarray(A.col)[idx], np.asarray(A.val)[idx])


def _abs(A) -> synth.CSR:
    return synth.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(np.asarray(A.val)))


def _unit(value_bytes: int) -> float:
    return U64 if value_bytes == 8 else U32


def assert_rows(y, A, x, value_bytes: int = 8, rows=None, tol: float | None = None, extra_terms: int = 0):
    """y (host array) against the oracle's A x, by relative L2 error and row by row.

    ``value_bytes`` is the size of the kernel's arithmetic type (8 or 4); x is the binary64
    copy of exactly the values the kernel read.  ``extra_terms`` widens each row's term count
    for results that add further rounded terms of the same row (e.g. a split into parts).
    Returns the relative error."""
    S = A if rows is None else sub_rows(A, rows)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64).ravel()
    ref = oracle.csr_spmv(S, x)
    mag = oracle.csr_spmv(_abs(S), np.abs(x))
    L = np.diff(np.asarray(S.row_ptr, np.int64)) + extra_terms
    bound = (gamma(L, _unit(value_bytes)) + gamma(L, U64)) * mag * (1.0 + 2.0 * gamma(L, U64))
    err = np.abs(y - ref)
    bad = np.flatnonzero(~(err <= bound))
    assert bad.size == 0, (f"{bad.size} rows outside the per-row bound; first: row "
                           f"{int(bad[0]) if rows is None else int(np.asarray(rows)[bad[0]])} "
                           f"|dy| = {err[bad[0]]:.3e} > {bound[bad[0]]:.3e}")
    rel = oracle.rel_l2(y, ref)
    assert rel <= (tol if tol is not None else TOL[value_bytes]), rel
    return rel


def assert_rows_mm(Y, A, X, rows=None, value_bytes: int = 8, tol: float | None = None):
    """The many-right-hand-side form: column v of Y against the oracle's A X[:, v], row by row."""
    S = A if rows is None else sub_rows(A, rows)
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64).reshape(S.n_rows, X.shape[1])
    ref = oracle.csr_spmmv(S, X)
    mag = oracle.csr_spmmv(_abs(S), np.abs(X))
    L = np.diff(np.asarray(S.row_ptr, np.int64))[:, None]
    bound = (gamma(L, _unit(value_bytes)) + gamma(L, U64)) * mag * (1.0 + 2.0 * gamma(L, U64))
    err = np.abs(Y - ref)
    bad = np.argwhere(~(err <= bound))
    assert bad.size == 0, f"{len(bad)} entries outside the per-row bound; first (row, vector) {tuple(bad[0])}"
    rel = oracle.rel_l2(Y, ref)
    assert rel <= (tol if tol is not None else TOL[value_bytes]), rel
    return rel


def assert_rows_axpby(y, A, x, a: float, b: float, z, value_bytes: int = 8, rows=None, tol: float | None = None):
    """y = a (A x) + b z, row by row: L_i + 2 rounded terms (the product's L_i, the scaling and
    the added b z_i), each bounded by its magnitude."""
    S = A if rows is None else sub_rows(A, rows)
    x = np.asarray(x, np.float64)
    z = np.asarray(z, np.float64).ravel()
    if rows is not None:
        z = z[np.asarray(rows)]
    y = np.asarray(y, np.float64).ravel()
    ref = a * oracle.csr_spmv(S, x) + b * z
    mag = abs(a) * oracle.csr_spmv(_abs(S), np.abs(x)) + abs(b) * np.abs(z)
    L = np.diff(np.asarray(S.row_ptr, np.int64)) + 2
    bound = (gamma(L, _unit(value_bytes)) + gamma(L, U64)) * mag * (1.0 + 2.0 * gamma(L, U64))
    err = np.abs(y - ref)
    bad = np.flatnonzero(~(err <= bound))
    assert bad.size == 0, f"{bad.size} rows outside the per-row bound; first {int(bad[0])}"
    rel = oracle.rel_l2(y, ref)
    assert rel <= (tol if tol is not None else TOL[value_bytes]), rel
    return rel


class RowReference:
    """The oracle's A x, sum of |a_ij x_j| and row lengths of one matrix and x, computed once and
    checked against several results (full-size matrices with many product forms)."""

    def __init__(self, A, x):
        self.A = A
        self.x = np.asarray(x, np.float64)
        self.ref = oracle.csr_spmv(A, self.x)
        self.mag = oracle.csr_spmv(_abs(A), np.abs(self.x))
        self.L = np.diff(np.asarray(A.row_ptr, np.int64))

    def check(self, y, value_bytes: int = 8, rows=None, extra_terms: int = 0, tol: float | None = None) -> float:
        """y holds rows ``rows`` of A x (all rows when None), in that order."""
        sel = slice(None) if rows is None else np.asarray(rows)
        ref, mag, L = self.ref[sel], self.mag[sel], self.L[sel] + extra_terms
        y = np.asarray(y, np.float64).ravel()
        bound = (gamma(L, _unit(value_bytes)) + gamma(L, U64)) * mag * (1.0 + 2.0 * gamma(L, U64))
        err = np.abs(y - ref)
        bad = np.flatnonzero(~(err <= bound))
        assert bad.size == 0, (f"{bad.size} rows outside the per-row bound; first: row "
                               f"{int(bad[0]) if rows is None else int(np.asarray(rows)[bad[0]])} "
                               f"|dy| = {err[bad[0]]:.3e} > {bound[bad[0]]:.3e}")
        rel = oracle.rel_l2(y, ref)
        assert rel <= (tol if tol is not None else TOL[value_bytes]), rel
        return rel
