"""CPU oracle for pJDS sparse matrix-vector multiplication -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The library under test never does, and the oracle imports nothing from it: the
two share only the seeded input generators in ``synth``.

What it computes (Kreutzer et al., arXiv:1112.5588):
* ``csr_spmv`` / ``csr_spmmv`` - y = A x from the plain definition, serial binary64 C code
  without contraction (``oracle.c``);
* ``pjds_build`` - the pJDS arrays by the "sort" and "pad" steps of Sect. 2.1 and the
  ``col_start`` addressing of Listing 2 (plus a per-block layout for sort windows);
* ``pjds_spmv`` - Listing 2 read literally on the oracle's own arrays;
* ``ellr_build`` - the ELLPACK-R arrays of Listing 1;
* ``mlp`` - a binary64 numpy forward/backward/Adam of the tuner network;
* ``features`` - the matrix features of the learned tuner, from their definitions.

Pins that tie each function to something other than itself live in ``tests/test_oracle*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)


_SO_T = os.path.join(_HERE, "liboracle_threads.so")
_SRC_T = os.path.join(_HERE, "csr_threads.c")


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc: -O2, no FP contraction, generic x86-64 code; and the
    all-core timing form ``csr_threads.c`` (-O3, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    if force or not os.path.exists(_SO_T):
        tmp = _SO_T + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fPIC", "-shared", _SRC_T, "-o", tmp])
        os.replace(tmp, _SO_T)
    return _SO


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        L.oracle_csr_spmv.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_csr_spmv_f32val.argtypes = [ctypes.c_int64, _i64p, _i32p, _f32p, _f64p, _f64p]
        L.oracle_csr_spmmv.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int32, _f64p, _f64p]
        L.oracle_pjds_sort.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int64, ctypes.c_int64, _i32p, _i32p]
        L.oracle_pjds_sort.restype = ctypes.c_int64
        L.oracle_pjds_block_max.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i64p]
        L.oracle_pjds_col_start.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, ctypes.c_int64, _i64p]
        L.oracle_pjds_block_start.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p, _i64p]
        L.oracle_pjds_fill.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       _i64p, _i32p, _f64p, _i32p, _i64p, ctypes.c_int64, _i32p, _f64p]
        L.oracle_pjds_spmv.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _i32p, _i64p,
                                       _i32p, _f64p, _f64p, _f64p]
        L.oracle_ellr_fill.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p, _i32p,
                                       _f64p, _i32p, _i32p, _f64p]
        _lib = L
    return _lib


_lib_t = None


def lib_threads() -> ctypes.CDLL:
    global _lib_t
    if _lib_t is None:
        if not os.path.exists(_SO_T):
            build(force=False)
        L = ctypes.CDLL(_SO_T)
        L.oracle_csr_spmv_threads.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_csr_spmv_f32val_threads.argtypes = [ctypes.c_int64, _i64p, _i32p, _f32p, _f64p, _f64p]
        _lib_t = L
    return _lib_t


def csr_spmv_threads(A, x: np.ndarray, y: np.ndarray | None = None) -> tuple[np.ndarray, int]:
    """The same product as ``csr_spmv`` with the rows shared among all OpenMP threads (bitwise
    the same result); for timing the CPU baseline on every core.  Returns (y, threads used)."""
    rp, col = _c(A.row_ptr, np.int64), _c(A.col, np.int32)
    x = _c(x, np.float64)
    if y is None:
        y = np.empty(A.n_rows, dtype=np.float64)
    if A.val.dtype == np.float32:
        used = lib_threads().oracle_csr_spmv_f32val_threads(A.n_rows, _p(rp, _i64p), _p(col, _i32p),
                                                            _p(_c(A.val, np.float32), _f32p), _p(x, _f64p),
                                                            _p(y, _f64p))
    else:
        used = lib_threads().oracle_csr_spmv_threads(A.n_rows, _p(rp, _i64p), _p(col, _i32p),
                                                     _p(_c(A.val, np.float64), _f64p), _p(x, _f64p), _p(y, _f64p))
    return y, int(used)


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def csr_spmv(A, x: np.ndarray) -> np.ndarray:
    """y = A x in binary64 (A's values widened exactly if they are float32)."""
    rp, col = _c(A.row_ptr, np.int64), _c(A.col, np.int32)
    x = _c(x, np.float64)
    y = np.empty(A.n_rows, dtype=np.float64)
    if A.val.dtype == np.float32:
        lib().oracle_csr_spmv_f32val(A.n_rows, _p(rp, _i64p), _p(col, _i32p),
                                     _p(_c(A.val, np.float32), _f32p), _p(x, _f64p), _p(y, _f64p))
    else:
        lib().oracle_csr_spmv(A.n_rows, _p(rp, _i64p), _p(col, _i32p),
                              _p(_c(A.val, np.float64), _f64p), _p(x, _f64p), _p(y, _f64p))
    return y


def csr_spmmv(A, X: np.ndarray) -> np.ndarray:
    """Y = A X for row-major X of shape (n_cols, k); returns (n_rows, k)."""
    X = _c(X, np.float64)
    k = X.shape[1]
    Y = np.empty((A.n_rows, k), dtype=np.float64)
    rp, col, val = _c(A.row_ptr, np.int64), _c(A.col, np.int32), _c(A.val, np.float64)
    lib().oracle_csr_spmmv(A.n_rows, _p(rp, _i64p), _p(col, _i32p), _p(val, _f64p), k,
                           _p(X, _f64p), _p(Y, _f64p))
    return Y


def pjds_build(A, b_r: int = 64, window: int | None = None, layout: str = "jd",
               symmetric: bool = False, lanes: int = 1) -> dict:
    """The pJDS arrays of A (see ``oracle.c`` for the construction and its citations).

    ``window`` None or >= n_rows is a global sort.  ``layout`` "jd" (Listing 2, requires a
    global sort) or "block"; ``lanes`` > 1 (block layout only) stores T = lanes consecutive
    slots per row and step.  Returns perm, row_len, block_max, offsets, col_p, val_p and
    the sizes n_pad, n_blocks, nnz_stored, max_row_len.
    """
    n = A.n_rows
    rp = _c(A.row_ptr, np.int64)
    w = 0 if window is None or window >= n else int(window)
    lay = {"jd": 0, "block": 1}[layout]
    if lay == 0 and w != 0:
        raise ValueError("JD layout needs a global sort")
    if lanes < 1 or (lanes > 1 and lay == 0):
        raise ValueError("lanes per row >= 1, and > 1 only with the block layout")
    if symmetric and A.n_rows != A.n_cols:
        raise ValueError("symmetric renumbering needs a square matrix")
    n_pad_guess = (n + b_r - 1) // b_r * b_r
    perm = np.zeros(max(n, 1), dtype=np.int32)
    row_len = np.zeros(max(n_pad_guess, 1), dtype=np.int32)
    n_pad = lib().oracle_pjds_sort(n, _p(rp, _i64p), b_r, w, _p(perm, _i32p), _p(row_len, _i32p))
    if n_pad < 0:
        raise ValueError("invalid block height or sort window")
    perm, row_len = perm[:n], row_len[:n_pad]
    n_blocks = n_pad // b_r
    block_max = np.zeros(max(n_blocks, 1), dtype=np.int64)
    lib().oracle_pjds_block_max(n_pad, b_r, _p(row_len, _i32p), _p(block_max, _i64p))
    block_max = block_max[:n_blocks]
    max_len = int(block_max.max()) if n_blocks else 0
    if lay == 0:
        offsets = np.zeros(max_len + 1, dtype=np.int64)
        bm = _c(block_max, np.int64) if n_blocks else np.zeros(1, np.int64)
        lib().oracle_pjds_col_start(n_blocks, b_r, _p(bm, _i64p), max_len, _p(offsets, _i64p))
    else:
        offsets = np.zeros(n_blocks + 1, dtype=np.int64)
        bm = _c(block_max, np.int64) if n_blocks else np.zeros(1, np.int64)
        lib().oracle_pjds_block_start(n_blocks, b_r, lanes, _p(bm, _i64p), _p(offsets, _i64p))
    nnz_stored = int(offsets[-1])
    col_p = np.zeros(max(nnz_stored, 1), dtype=np.int32)
    val_p = np.zeros(max(nnz_stored, 1), dtype=np.float64)
    col = _c(A.col, np.int32) if A.nnz else np.zeros(1, np.int32)
    val = _c(A.val, np.float64) if A.nnz else np.zeros(1, np.float64)
    perm_c = perm if n else np.zeros(1, np.int32)
    lib().oracle_pjds_fill(n, b_r, lanes, lay, int(bool(symmetric)), _p(rp, _i64p), _p(col, _i32p),
                           _p(val, _f64p), _p(perm_c, _i32p), _p(offsets, _i64p), nnz_stored,
                           _p(col_p, _i32p), _p(val_p, _f64p))
    col_p, val_p = col_p[:nnz_stored], val_p[:nnz_stored]
    if A.val.dtype == np.float32:
        val_p = val_p.astype(np.float32)          # exact: every value came from float32
    return dict(perm=perm, row_len=row_len, block_max=block_max, offsets=offsets, col_p=col_p,
                val_p=val_p, n_pad=int(n_pad), n_blocks=int(n_blocks), nnz_stored=nnz_stored,
                max_row_len=max_len, b_r=b_r, layout=layout, n_rows=n, symmetric=bool(symmetric),
                lanes=lanes)


def pjds_spmv(P: dict, x: np.ndarray) -> np.ndarray:
    """Listing 2 on the oracle's arrays: the product in the permuted row basis, y_perm[i] =
    (A x)[perm[i]] (with ``symmetric`` arrays, x must be in the permuted basis too)."""
    n = P["n_rows"]
    x = _c(x, np.float64) if len(x) else np.zeros(1)
    y = np.empty(max(n, 1), dtype=np.float64)
    col_p = P["col_p"] if P["nnz_stored"] else np.zeros(1, np.int32)
    val_p = _c(P["val_p"], np.float64) if P["nnz_stored"] else np.zeros(1)
    lib().oracle_pjds_spmv(n, P["b_r"], P.get("lanes", 1), {"jd": 0, "block": 1}[P["layout"]],
                           _p(_c(P["row_len"], np.int32), _i32p), _p(_c(P["offsets"], np.int64), _i64p),
                           _p(_c(col_p, np.int32), _i32p), _p(val_p, _f64p), _p(x, _f64p), _p(y, _f64p))
    return y[:n]


def ellr_build(A, pad_to: int = 64) -> dict:
    """The ELLPACK-R arrays of Listing 1: column-major n_pad x max_len, rowmax per row."""
    n = A.n_rows
    n_pad = (n + pad_to - 1) // pad_to * pad_to
    lens = np.diff(A.row_ptr)
    max_len = int(lens.max()) if n else 0
    rowmax = np.zeros(max(n_pad, 1), dtype=np.int32)
    col_e = np.zeros(max(n_pad * max_len, 1), dtype=np.int32)
    val_e = np.zeros(max(n_pad * max_len, 1), dtype=np.float64)
    col = _c(A.col, np.int32) if A.nnz else np.zeros(1, np.int32)
    val = _c(A.val, np.float64) if A.nnz else np.zeros(1)
    lib().oracle_ellr_fill(n, n_pad, max_len, _p(_c(A.row_ptr, np.int64), _i64p), _p(col, _i32p),
                           _p(val, _f64p), _p(rowmax, _i32p), _p(col_e, _i32p), _p(val_e, _f64p))
    val_e = val_e[:n_pad * max_len]
    if A.val.dtype == np.float32:
        val_e = val_e.astype(np.float32)
    return dict(rowmax=rowmax[:n_pad], col=col_e[:n_pad * max_len], val=val_e, n_pad=n_pad,
                max_len=max_len, n_rows=n)


def rel_l2(y: np.ndarray, y_ref: np.ndarray) -> float:
    """||y - y_ref||_2 / ||y_ref||_2 in binary64 (absolute error when y_ref is zero)."""
    y = np.asarray(y, dtype=np.float64).ravel()
    y_ref = np.asarray(y_ref, dtype=np.float64).ravel()
    d = float(np.linalg.norm(y - y_ref))
    r = float(np.linalg.norm(y_ref))
    return d / r if r > 0 else d


def split_columns(A, c0: int, c1: int):
    """The local/non-local split of Sect. 3.1 (vector mode), row by row from its definition:
    entries with column in [c0, c1) go to the local part, the others to the non-local part,
    each row keeping its order.  Returns ((row_ptr, col, val) local, (row_ptr, col, val) rest)."""
    parts = ([0], [], []), ([0], [], [])
    for i in range(A.n_rows):
        for k in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            p = parts[0] if c0 <= int(A.col[k]) < c1 else parts[1]
            p[1].append(int(A.col[k]))
            p[2].append(A.val[k])
        for p in parts:
            p[0].append(len(p[1]))
    return tuple((np.array(rp, np.int64), np.array(c, np.int32), np.array(v, dtype=np.asarray(A.val).dtype))
                 for rp, c, v in parts)
