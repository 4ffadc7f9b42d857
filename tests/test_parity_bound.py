"""The per-row error bound used by the GPU parity tests, checked on the CPU: results computed
in binary32 or in another summation order pass, and a planted mistake in one row fails."""
import numpy as np
import pytest

import oracle
import synth
from parity import assert_rows, assert_rows_axpby, assert_rows_mm, sub_rows


def f32_rows_reversed(A, x):
    """A x with binary32 products and sums, each row summed from its last entry to its first."""
    y = np.zeros(A.n_rows, np.float32)
    for i in range(A.n_rows):
        acc = np.float32(0)
        for k in range(A.row_ptr[i + 1] - 1, A.row_ptr[i] - 1, -1):
            acc = np.float32(acc + np.float32(np.float32(A.val[k]) * np.float32(x[A.col[k]])))
        y[i] = acc
    return y.astype(np.float64)


def test_sub_rows_picks_rows_in_order():
    A = synth.random_csr(40, 30, 3, max_len=6)
    rows = np.array([7, 0, 39, 7])
    S = sub_rows(A, rows)
    for k, r in enumerate(rows):
        assert np.array_equal(S.col[S.row_ptr[k]:S.row_ptr[k + 1]], A.col[A.row_ptr[r]:A.row_ptr[r + 1]])
        assert np.array_equal(S.val[S.row_ptr[k]:S.row_ptr[k + 1]], A.val[A.row_ptr[r]:A.row_ptr[r + 1]])


def test_binary32_reordered_sums_pass_and_a_planted_error_fails():
    A = synth.random_csr(400, 300, 5, max_len=40).astype(np.float32)
    x = synth.dense_x(300, 5).astype(np.float32).astype(np.float64)
    y = f32_rows_reversed(A, x)
    assert_rows(y, A, x, value_bytes=4)
    # the same binary32 result does not meet the binary64 bound
    with pytest.raises(AssertionError):
        assert_rows(y, A, x, value_bytes=8)
    # one row off by a dropped term: outside its own bound although the norm is within 1e-5
    ref = oracle.csr_spmv(A, x)
    i = int(np.argmax(np.diff(A.row_ptr)))
    k = A.row_ptr[i]
    bad = ref.copy()
    bad[i] -= float(A.val[k]) * x[A.col[k]] * 1e-3
    assert oracle.rel_l2(bad, ref) < 1e-5
    with pytest.raises(AssertionError):
        assert_rows(bad, A, x, value_bytes=4)


def test_sampled_rows_and_many_right_hand_sides():
    A = synth.hh_like(3000, seed=8)
    x = synth.dense_x(A.n_cols, 8)
    ref = oracle.csr_spmv(A, x)
    rows = np.array([5, 2999, 0, 1200])
    assert_rows(ref[rows], A, x, rows=rows)
    with pytest.raises(AssertionError):
        assert_rows(ref[rows[::-1]], A, x, rows=rows)            # rows swapped
    X = synth.dense_x(A.n_cols, 9, k=3).reshape(A.n_cols, 3)
    Y = oracle.csr_spmmv(A, X)
    assert_rows_mm(Y, A, X)
    Y[17, 1] *= 1 + 1e-13
    with pytest.raises(AssertionError):
        assert_rows_mm(Y, A, X)


def test_axpby_bound():
    A = synth.random_csr(200, 200, 11, max_len=12)
    x = synth.dense_x(200, 11)
    z = synth.dense_x(200, 12)
    y = 2.0 * oracle.csr_spmv(A, x) - 0.5 * z
    assert_rows_axpby(y, A, x, 2.0, -0.5, z)
    with pytest.raises(AssertionError):
        assert_rows_axpby(y, A, x, 2.0, 0.5, z)                   # wrong sign of b


def test_empty_rows_must_be_exactly_zero():
    A = synth.random_csr(100, 50, 13, max_len=5, empty_frac=0.5)
    x = synth.dense_x(50, 13)
    y = oracle.csr_spmv(A, x)
    empty = np.flatnonzero(np.diff(A.row_ptr) == 0)
    assert empty.size
    y[empty[0]] = 1e-300
    with pytest.raises(AssertionError):
        assert_rows(y, A, x)
