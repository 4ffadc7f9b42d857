"""Pins for the CPU oracle: each check ties it to something other than itself (brute force,
a library routine, a closed form, an invariant or a number the paper prints)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(A):
    D = np.zeros((A.n_rows, A.n_cols))
    for i in range(A.n_rows):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            D[i, A.col[k]] += A.val[k]
    return D


# ---------------------------------------------------------------- y = A x itself

@pytest.mark.parametrize("seed", range(6))
def test_spmv_equals_dense_bruteforce_integer(seed):
    # small integer entries: every partial sum is exact, so equality is exact
    A = synth.random_csr(37, 29, seed, max_len=9, integer=True)
    x = synth.dense_x(29, seed, integer=True)
    assert np.array_equal(oracle.csr_spmv(A, x), dense(A) @ x)


@pytest.mark.parametrize("seed", range(4))
def test_spmv_matches_scipy(seed):
    A = synth.random_csr(500, 300, seed, max_len=20)
    x = synth.dense_x(300, seed + 10)
    M = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    assert oracle.rel_l2(oracle.csr_spmv(A, x), M @ x) < 1e-14


def test_spmv_empty_and_degenerate():
    A = synth.random_csr(10, 0, 1)              # no columns, all rows empty
    assert np.array_equal(oracle.csr_spmv(A, np.zeros(0)), np.zeros(10))
    A = synth.random_csr(0, 5, 1)
    assert oracle.csr_spmv(A, np.ones(5)).shape == (0,)


def test_laplacian_times_ones_closed_form():
    # 4 - (#neighbours): 0 inside, 1 on the 4*126 non-corner edge nodes, 2 on the corners
    A = synth.laplacian_2d(128)
    y = oracle.csr_spmv(A, np.ones(A.n_cols))
    r, c = np.divmod(np.arange(A.n_rows), 128)
    edges = (r == 0).astype(int) + (r == 127) + (c == 0) + (c == 127)
    assert np.array_equal(y, edges.astype(float))
    assert (y == 0).sum() == 15876 and (y == 1).sum() == 504 and (y == 2).sum() == 4
    assert y.sum() == 512.0


@pytest.mark.parametrize("p,q", [(1, 1), (3, 7), (64, 2), (128, 128)])
def test_laplacian_sine_eigenvectors(p, q):
    # v(r,c) = sin(p pi (r+1)/129) sin(q pi (c+1)/129), lambda = 4 - 2cos(p pi/129) - 2cos(q pi/129)
    A = synth.laplacian_2d(128)
    r, c = np.divmod(np.arange(A.n_rows), 128)
    # reduce the angles exactly (sin has period 2*pi = 258 * pi/129) before calling sin
    v = np.sin(np.pi * ((p * (r + 1)) % 258) / 129) * np.sin(np.pi * ((q * (c + 1)) % 258) / 129)
    lam = 4 - 2 * np.cos(p * np.pi / 129) - 2 * np.cos(q * np.pi / 129)
    # rounding error scales with ||A|| ||v|| (terms up to 4|v_i|), not with lambda ||v||
    err = np.linalg.norm(oracle.csr_spmv(A, v) - lam * v)
    assert err <= 8 * 2.0 ** -52 * 8 * np.linalg.norm(v)


def test_identity_diagonal_permutation():
    n = 50
    perm = np.argsort(synth.uniform01(4, 1, n))
    d = synth.uniform_pm1(4, 2, n)
    x = synth.dense_x(n, 4)
    eye = synth.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n))
    diag = synth.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d)
    pm = synth.CSR(n, n, np.arange(n + 1, dtype=np.int64), perm.astype(np.int32), np.ones(n))
    assert np.array_equal(oracle.csr_spmv(eye, x), x)
    assert np.array_equal(oracle.csr_spmv(diag, x), d * x)
    assert np.array_equal(oracle.csr_spmv(pm, x), x[perm])


def test_f32_values_are_widened_exactly():
    A = synth.random_csr(200, 150, 9, max_len=12)
    A32 = A.astype(np.float32)
    x = synth.dense_x(150, 9)
    wide = synth.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A32.val.astype(np.float64))
    assert np.array_equal(oracle.csr_spmv(A32, x), oracle.csr_spmv(wide, x))


@pytest.mark.parametrize("k", [1, 4, 7])
def test_spmmv_equals_dense_bruteforce(k):
    A = synth.random_csr(40, 33, 5, max_len=10, integer=True)
    X = synth.dense_x(33, 5, k=k, integer=True).reshape(33, k)
    assert np.array_equal(oracle.csr_spmmv(A, X), dense(A) @ X)


# ---------------------------------------------------------------- pJDS construction

def slot(P, i, j):
    """Stored position of entry j of sorted row i: Listing 2's col_start[j] + i, the block
    tile's block_start[b] + j b_r + r, or with T lanes per row step j // T of the block, lane
    slot r T + j % T."""
    if P["layout"] == "jd":
        return P["offsets"][j] + i
    b_r, T = P["b_r"], P.get("lanes", 1)
    return P["offsets"][i // b_r] + (j // T) * (b_r * T) + (i % b_r) * T + j % T


def decode_pjds(P, A):
    """Read the stored arrays back through the addressing rule."""
    rows = []
    for i in range(P["n_rows"]):
        ent = []
        for j in range(P["row_len"][i]):
            a = slot(P, i, j)
            ent.append((int(P["col_p"][a]), float(P["val_p"][a])))
        rows.append(ent)
    return rows


def check_invariants(A, P, window):
    n, b_r = A.n_rows, P["b_r"]
    lens = np.diff(A.row_ptr)
    perm = P["perm"]
    # bijection
    assert np.array_equal(np.sort(perm), np.arange(n))
    # row_len is the permuted length, padding rows are empty
    assert np.array_equal(P["row_len"][:n], lens[perm])
    assert np.all(P["row_len"][n:] == 0)
    assert P["row_len"].sum() == A.nnz
    # non-increasing within each window, and rows never leave their window
    w = n if window is None or window >= n else window
    for w0 in range(0, n, max(w, 1)):
        seg = P["row_len"][w0:min(n, w0 + w)]
        assert np.all(np.diff(seg) <= 0)
        assert np.all((perm[w0:min(n, w0 + w)] >= w0) & (perm[w0:min(n, w0 + w)] < w0 + w))
    # ties keep the original order (stable)
    for i in range(n - 1):
        if P["row_len"][i] == P["row_len"][i + 1] and (i // w) == ((i + 1) // w):
            assert perm[i] < perm[i + 1]
    # stored count = b_r * sum of block maxima (T lanes: b_r T * sum of ceil(M_b / T))
    T = P.get("lanes", 1)
    assert P["nnz_stored"] == b_r * T * int(((P["block_max"] + T - 1) // T).sum())
    # round trip: entries and their order reproduce the input exactly
    rows = decode_pjds(P, A)
    for i in range(n):
        src = perm[i]
        a, b = A.row_ptr[src], A.row_ptr[src + 1]
        assert rows[i] == list(zip(A.col[a:b].tolist(), A.val[a:b].tolist()))
    # every slot not used by a row is padding: value 0 and column 0
    used = np.zeros(P["nnz_stored"], bool)
    for i in range(P["n_pad"]):
        for j in range(P["row_len"][i]):
            a = slot(P, i, j)
            assert not used[a]
            used[a] = True
    assert np.all(P["val_p"][~used] == 0) and np.all(P["col_p"][~used] == 0)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("b_r", [1, 2, 4, 32, 64])
def test_pjds_invariants_global(seed, b_r):
    A = synth.random_csr(203, 90, seed, max_len=13)
    for layout in ("jd", "block"):
        P = oracle.pjds_build(A, b_r=b_r, layout=layout)
        check_invariants(A, P, None)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("b_r,window", [(4, 4), (4, 16), (32, 64), (64, 128), (2, 1000)])
def test_pjds_invariants_window(seed, b_r, window):
    A = synth.random_csr(301, 120, seed + 20, max_len=17)
    P = oracle.pjds_build(A, b_r=b_r, window=window, layout="block")
    check_invariants(A, P, window)


def test_pjds_jd_needs_global_sort():
    A = synth.random_csr(100, 100, 1)
    with pytest.raises(ValueError):
        oracle.pjds_build(A, b_r=4, window=8, layout="jd")


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("layout,window", [("jd", None), ("block", None), ("block", 64)])
def test_pjds_product_equals_plain_product(seed, layout, window):
    # Listing 2 sums a row in stored order, which is CSR order, so the permuted product is
    # bit-identical to the plain one read through perm.
    A = synth.random_csr(257, 190, seed, max_len=21)
    x = synth.dense_x(190, seed)
    P = oracle.pjds_build(A, b_r=32, window=window, layout=layout)
    assert np.array_equal(oracle.pjds_spmv(P, x), oracle.csr_spmv(A, x)[P["perm"]])


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("b_r,lanes,window", [(32, 2, None), (16, 4, 64), (8, 8, 128), (1, 64, None), (3, 5, 9)])
def test_pjds_lanes_invariants_and_product(seed, b_r, lanes, window):
    # T lanes per row (the sliced ELLR-T idea of the outlook, Sect. 4): same sort, same rows,
    # each block stored as ceil(M_b / T) steps of b_r T slots; the product in stored order is
    # still CSR order, so it is bit-identical to the plain one
    A = synth.random_csr(311, 150, seed + 40, max_len=70)
    P = oracle.pjds_build(A, b_r=b_r, window=window, layout="block", lanes=lanes)
    check_invariants(A, P, window)
    x = synth.dense_x(150, seed)
    assert np.array_equal(oracle.pjds_spmv(P, x), oracle.csr_spmv(A, x)[P["perm"]])


def test_pjds_one_lane_is_the_block_layout():
    A = synth.random_csr(500, 300, 9, max_len=25)
    P1 = oracle.pjds_build(A, b_r=64, window=128, layout="block", lanes=1)
    P0 = oracle.pjds_build(A, b_r=64, window=128, layout="block")
    for k in ("perm", "row_len", "offsets", "col_p", "val_p"):
        assert np.array_equal(P1[k], P0[k]), k


def test_pjds_lanes_single_row_is_the_row_itself():
    # one row of length 100, b_r = 1 and T = 64: the row is stored contiguously in its own
    # order, padded to the next multiple of 64 (two steps of 64 slots)
    row = synth.CSR(1, 500, np.array([0, 100], np.int64), np.arange(0, 500, 5, dtype=np.int32),
                    np.arange(1, 101, dtype=np.float64))
    P = oracle.pjds_build(row, b_r=1, layout="block", lanes=64)
    assert P["nnz_stored"] == 128 and list(P["offsets"]) == [0, 128]
    assert np.array_equal(P["val_p"][:100], row.val) and np.array_equal(P["col_p"][:100], row.col)
    assert np.all(P["val_p"][100:] == 0) and np.all(P["col_p"][100:] == 0)


def test_pjds_lanes_hand_worked_block():
    # rows of lengths 3 and 2 (values 1 2 3 | 4 5), one block of b_r = 2 rows, T = 2 lanes:
    # step 0 holds row 0's entries 0, 1 then row 1's entries 0, 1; step 1 holds row 0's
    # entry 2, then padding
    A = synth.CSR(2, 4, np.array([0, 3, 5], np.int64), np.array([0, 1, 3, 1, 2], np.int32),
                  np.array([1.0, 2.0, 3.0, 4.0, 5.0]))
    P = oracle.pjds_build(A, b_r=2, layout="block", lanes=2)
    assert list(P["offsets"]) == [0, 8]
    assert list(P["val_p"]) == [1.0, 2.0, 4.0, 5.0, 3.0, 0.0, 0.0, 0.0]
    assert list(P["col_p"]) == [0, 1, 1, 2, 3, 0, 0, 0]


@pytest.mark.parametrize("L,T", [(8, 2), (8, 4), (12, 4), (16, 16)])
def test_pjds_lanes_constant_length_no_overhead(L, T):
    # every row of length L with T dividing L: no padding at all, nnz_stored = N_pad L
    n = 64 * 5
    A = synth.CSR(n, n, np.arange(0, n * L + 1, L, dtype=np.int64),
                  (np.arange(n * L, dtype=np.int64) % n).astype(np.int32), np.ones(n * L))
    P = oracle.pjds_build(A, b_r=64 // T, layout="block", lanes=T)
    assert P["nnz_stored"] == n * L


def test_pjds_symmetric_renumbering():
    # P A P^T (P x) = P (A x): with columns renumbered, x and y both live in the permuted basis
    A = synth.hh_like(3000, seed=7)
    x = synth.dense_x(3000, 7)
    P = oracle.pjds_build(A, b_r=64, symmetric=True)
    xp = x[P["perm"]]
    y = oracle.pjds_spmv(P, xp)
    assert np.array_equal(y, oracle.csr_spmv(A, x)[P["perm"]])
    assert P["col_p"].min() >= 0 and P["col_p"].max() < 3000


def test_hand_worked_example_b4():
    # 9 x 6 matrix, row lengths (by row) 2,0,3,1,3,2,4,1,2; values encode (row, slot).
    lens = [2, 0, 3, 1, 3, 2, 4, 1, 2]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cols, vals = [], []
    for r, L in enumerate(lens):
        for j in range(L):
            cols.append((r + j) % 6)
            vals.append(10 * r + j + 0.5)
    A = synth.CSR(9, 6, rp, np.array(cols, np.int32), np.array(vals))
    P = oracle.pjds_build(A, b_r=4, layout="jd")
    # sort, longest first, ties by original index: 6(4) 2(3) 4(3) 0(2) 5(2) 8(2) 3(1) 7(1) 1(0)
    assert P["perm"].tolist() == [6, 2, 4, 0, 5, 8, 3, 7, 1]
    # pad: N_pad = 12, blocks {6,2,4,0} -> 4, {5,8,3,7} -> 2, {1,-,-,-} -> 0
    assert P["row_len"].tolist() == [4, 3, 3, 2, 2, 2, 1, 1, 0, 0, 0, 0]
    assert P["block_max"].tolist() == [4, 2, 0]
    # columns 0,1 hold 8 rows, columns 2,3 hold 4 rows
    assert P["offsets"].tolist() == [0, 8, 16, 20, 24]
    assert P["nnz_stored"] == 24
    # JD column 0 = first entries of the 8 rows in sorted order, then column 1, ...
    first = [60.5, 20.5, 40.5, 0.5, 50.5, 80.5, 30.5, 70.5]
    second = [61.5, 21.5, 41.5, 1.5, 51.5, 81.5, 0.0, 0.0]
    third = [62.5, 22.5, 42.5, 0.0]
    fourth = [63.5, 0.0, 0.0, 0.0]
    assert P["val_p"].tolist() == first + second + third + fourth
    # block layout: each block is its own b_r x M_b column-major tile
    Q = oracle.pjds_build(A, b_r=4, layout="block")
    assert Q["offsets"].tolist() == [0, 16, 24, 24]
    assert Q["val_p"][:8].tolist() == [60.5, 20.5, 40.5, 0.5, 61.5, 21.5, 41.5, 1.5]
    assert Q["val_p"][16:24].tolist() == [50.5, 80.5, 30.5, 70.5, 51.5, 81.5, 0.0, 0.0]


def test_config1_exact_arrays():
    # 128x128 Laplacian: 15876 interior rows of length 5 (first interior node is 129), 504
    # edge rows of length 4, corners 0, 127, 16256, 16383 of length 3.  With b_r = 64,
    # 15876 = 248*64 + 4, so blocks 0..248 have maximum 5 and blocks 249..255 maximum 4.
    A = synth.laplacian_2d(128)
    P = oracle.pjds_build(A, b_r=64, layout="jd")
    assert P["nnz_stored"] == 64 * (249 * 5 + 7 * 4) == 81472
    assert P["offsets"].tolist() == [0, 16384, 32768, 49152, 65536, 81472]
    assert P["perm"][:3].tolist() == [129, 130, 131]
    assert P["perm"][15876:15879].tolist() == [1, 2, 3]
    assert P["perm"][-4:].tolist() == [0, 127, 16256, 16383]


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))["storage_constant_row_length"]["cases"])
def test_paper_constant_row_length_no_overhead(case):
    n, L, b_r = case["n"], case["row_len"], case["b_r"]
    rp = np.arange(n + 1, dtype=np.int64) * L
    col = (np.arange(n * L) % n).astype(np.int32)
    A = synth.CSR(n, n, rp, col, np.ones(n * L))
    P = oracle.pjds_build(A, b_r=b_r)
    E = oracle.ellr_build(A, pad_to=b_r)
    assert P["nnz_stored"] == n * L == E["n_pad"] * E["max_len"]


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))["storage_one_full_row"]["cases"])
def test_paper_one_full_row(case):
    n, b_r = case["n"], case["b_r"]
    lens = np.ones(n, dtype=np.int64)
    lens[n // 3] = n
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([np.arange(L) if L == n else [i] for i, L in enumerate(lens)]).astype(np.int32)
    A = synth.CSR(n, n, rp, col, np.ones(int(lens.sum())))
    P = oracle.pjds_build(A, b_r=b_r)
    E = oracle.ellr_build(A, pad_to=b_r)
    assert P["nnz_stored"] == case["pjds"]
    assert E["n_pad"] * E["max_len"] == case["ellpack"]


@pytest.mark.parametrize("seed", range(5))
def test_jds_special_case_no_padding(seed):
    # b_r = 1 is classic JDS: nothing is padded
    A = synth.random_csr(150, 80, seed, max_len=15)
    assert oracle.pjds_build(A, b_r=1)["nnz_stored"] == A.nnz


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("b_r", [4, 32, 64])
def test_padding_bound_global_sort(seed, b_r):
    # within a sorted block the padding is at most (b_r-1)(M_b - m_b); the block ranges
    # telescope, so the total is at most (b_r-1)(L_max - L_min'), L_min' = 0 if rows are padded
    A = synth.random_csr(333, 100, seed, max_len=30, empty_frac=0.0)
    P = oracle.pjds_build(A, b_r=b_r)
    lens = np.diff(A.row_ptr)
    lmin = 0 if P["n_pad"] > A.n_rows else lens.min()
    assert P["nnz_stored"] - A.nnz <= (b_r - 1) * (lens.max() - lmin)


def test_single_block_is_ellpack_of_sorted_rows():
    # one block holding every row: the block tile is exactly the ELLPACK-R rectangle of the
    # row-sorted matrix
    A = synth.random_csr(64, 40, 3, max_len=9)
    P = oracle.pjds_build(A, b_r=64, layout="block")
    perm = P["perm"]
    lens = np.diff(A.row_ptr)[perm]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([A.col[A.row_ptr[r]:A.row_ptr[r + 1]] for r in perm]).astype(np.int32)
    val = np.concatenate([A.val[A.row_ptr[r]:A.row_ptr[r + 1]] for r in perm])
    E = oracle.ellr_build(synth.CSR(64, 40, rp, col, val), pad_to=64)
    assert np.array_equal(P["val_p"], E["val"]) and np.array_equal(P["col_p"], E["col"])


# ---------------------------------------------------------------- ELLPACK-R

@pytest.mark.parametrize("seed", range(3))
def test_ellr_layout_and_product(seed):
    A = synth.random_csr(130, 70, seed, max_len=11, integer=True)
    E = oracle.ellr_build(A, pad_to=64)
    assert E["n_pad"] == 192 and E["max_len"] == int(np.diff(A.row_ptr).max())
    x = synth.dense_x(70, seed, integer=True)
    # Listing 1 read literally, on tiny integer data (exact)
    y = np.zeros(130)
    for i in range(130):
        for j in range(E["rowmax"][i]):
            y[i] += E["val"][j * E["n_pad"] + i] * x[E["col"][j * E["n_pad"] + i]]
    assert np.array_equal(y, dense(A) @ x)
    assert np.all(E["rowmax"][130:] == 0)


def test_rel_l2_hand_computed():
    # ||(3, 4) - (0, 0)|| / ||(0, 0)|| takes the absolute branch: 5
    assert oracle.rel_l2(np.array([3.0, 4.0]), np.zeros(2)) == 5.0
    # ||(1, 2, 2) - (0, 0, 0)|| / ... with y_ref = (2, 0, 0): d = (-1, 2, 2), ||d|| = 3, ||ref|| = 2
    assert oracle.rel_l2(np.array([1.0, 2.0, 2.0]), np.array([2.0, 0.0, 0.0])) == 1.5
    # the denominator is the reference's norm, not the candidate's: swapping the arguments
    # gives 3 / 3
    assert oracle.rel_l2(np.array([2.0, 0.0, 0.0]), np.array([1.0, 2.0, 2.0])) == 1.0
    # equal vectors, and float32 input widened exactly
    assert oracle.rel_l2(np.array([0.1, -7.0]), np.array([0.1, -7.0])) == 0.0
    assert oracle.rel_l2(np.float32([0.5, 0.25]), np.array([0.5, 0.0])) == 0.5
    # matrices are flattened: a difference [[0, 3], [4, 0]] of norm 5 against a reference
    # of norm 10
    assert oracle.rel_l2(np.array([[6.0, 3.0], [4.0, 8.0]]), np.array([[6.0, 0.0], [0.0, 8.0]])) == 0.5
    assert oracle.rel_l2(np.zeros(0), np.zeros(0)) == 0.0


@pytest.mark.parametrize("c0,c1", [(0, 29), (5, 17), (0, 0), (28, 29)])
def test_split_columns_pinned_by_dense_brute_force(c0, c1):
    # the two parts of the column split, as dense matrices: they add up to A, the local part
    # lives in columns [c0, c1) only, the other part outside them; every row keeps its order
    A = synth.random_csr(37, 29, 7, max_len=9, integer=True)
    (rl, cl, vl), (rn, cn, vn) = oracle.split_columns(A, c0, c1)
    L_ = synth.CSR(37, 29, rl, cl, vl)
    N_ = synth.CSR(37, 29, rn, cn, vn)
    DL, DN, DA = dense(L_), dense(N_), dense(A)
    assert np.array_equal(DL + DN, DA)
    inside = np.zeros(29, bool)
    inside[c0:c1] = True
    assert not DL[:, ~inside].any() and not DN[:, inside].any()
    for i in range(37):
        row = list(A.col[A.row_ptr[i]:A.row_ptr[i + 1]])
        assert list(cl[rl[i]:rl[i + 1]]) == [c for c in row if c0 <= c < c1]
        assert list(cn[rn[i]:rn[i + 1]]) == [c for c in row if not c0 <= c < c1]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_all_core_baseline_equals_the_serial_oracle_bitwise(dtype):
    # the CPU baseline's threaded form runs each row's sum unchanged: the same bits as the
    # serial definition, whatever the thread count
    A = synth.hh_like(100003, seed=12).astype(dtype)
    x = synth.dense_x(A.n_cols, 12)
    y, used = oracle.csr_spmv_threads(A, x)
    assert used >= 1
    assert np.array_equal(y.view(np.uint64), oracle.csr_spmv(A, x).view(np.uint64))
