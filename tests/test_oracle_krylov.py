"""Pins for the Lanczos oracle: closed-form Laplacian eigenvalues, scipy's eigsh, basis
independence, and the tridiagonal identity A V = V T + beta v e^T."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle import krylov


def test_largest_ritz_value_of_laplacian_converges_to_closed_form():
    # the 2D Dirichlet Laplacian on n x n has eigenvalues 4 - 2cos(p pi/(n+1)) - 2cos(q pi/(n+1))
    A = synth.laplacian_2d(32)
    a, b = krylov.lanczos(A, synth.dense_x(A.n_cols, 3), 200)
    lam_max = 4 + 4 * np.cos(np.pi / 33)
    lam_min = 4 - 4 * np.cos(np.pi / 33)
    r = krylov.ritz_values(a, b)
    assert abs(r.max() - lam_max) < 1e-9 and abs(r.min() - lam_min) < 1e-9


def test_extreme_ritz_values_match_eigsh():
    A = synth.hh_like(20000, seed=7)
    M = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    a, b = krylov.lanczos(A, synth.dense_x(A.n_cols, 5), 150)
    r = krylov.ritz_values(a, b)
    top = spla.eigsh(M, k=1, which="LA", return_eigenvectors=False)[0]
    assert abs(r.max() - top) < 1e-8 * abs(top)


def test_coefficients_do_not_depend_on_the_basis():
    A = synth.hh_like(5000, seed=8)
    v = synth.dense_x(A.n_cols, 9)
    P = oracle.pjds_build(A, b_r=64, symmetric=True)
    perm = P["perm"]
    # P A P^T as CSR: row i is original row perm[i], columns renumbered by invperm
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm), dtype=perm.dtype)
    lens = np.diff(A.row_ptr)[perm]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([inv[A.col[A.row_ptr[r]:A.row_ptr[r + 1]]] for r in perm]).astype(np.int32)
    val = np.concatenate([A.val[A.row_ptr[r]:A.row_ptr[r + 1]] for r in perm])
    B = synth.CSR(A.n_rows, A.n_cols, rp, col, val)
    a1, b1 = krylov.lanczos(A, v, 25)
    a2, b2 = krylov.lanczos(B, v[perm], 25)
    assert np.allclose(a1, a2, rtol=1e-10, atol=1e-12) and np.allclose(b1, b2, rtol=1e-10, atol=1e-12)


def test_three_term_recurrence_identity():
    # with exact arithmetic A v_j = beta_j v_{j-1} + alpha_j v_j + beta_{j+1} v_{j+1}
    A = synth.random_csr(300, 300, 4, max_len=6)
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(300, 300))
    S = (S + S.T).tocsr()
    S.sort_indices()
    A = synth.CSR(300, 300, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data)
    a, b = krylov.lanczos(A, synth.dense_x(300, 5), 6)
    V = []
    v = synth.dense_x(300, 5)
    v = v / np.linalg.norm(v)
    vp = np.zeros(300)
    for j in range(6):
        V.append(v)
        w = S @ v - b[j] * vp - a[j] * v
        vp, v = v, w / b[j + 1]
    V = np.array(V)
    for j in range(1, 5):
        lhs = S @ V[j]
        rhs = b[j] * V[j - 1] + a[j] * V[j] + b[j + 1] * V[j + 1]
        assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(lhs)


def test_axpby_definition():
    A = synth.random_csr(50, 40, 3, max_len=5, integer=True)
    x = synth.dense_x(40, 3, integer=True)
    z = synth.dense_x(50, 4, integer=True)
    D = np.zeros((50, 40))
    for i in range(50):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col[k]] += A.val[k]
    assert np.array_equal(krylov.axpby(A, x, 2.0, -3.0, z), 2.0 * (D @ x) - 3.0 * z)
    assert np.array_equal(krylov.axpby(A, x, 1.0, 5.0, None), D @ x)
