"""Host conversion of the library vs the oracle's independent construction: every index
array and every stored value must be bit-identical (CPU only, no GPU needed)."""
import numpy as np
import pytest

import oracle
import synth
from paper_1112_5588_amd import _lib as L


def lib_convert(A, b_r=64, window=0, layout="jd", symmetric=False, split_len=0, lanes=1):
    flags = (L.PJDS_LAYOUT_BLOCK if layout == "block" else 0) | (L.PJDS_SYMMETRIC if symmetric else 0)
    flags |= L.PJDS_LANES(lanes.bit_length() - 1)
    row_ptr = np.ascontiguousarray(A.row_ptr, np.int64)
    info = L.pjds_plan(A.n_rows, A.n_cols, row_ptr, b_r, window, flags, split_len)
    h = dict(perm=np.full(max(info.n_rows, 1), -7, np.int32),
             row_len=np.full(max(info.n_pad, 1), -7, np.int32),
             offsets=np.full(max(info.n_offsets, 1), -7, np.int64),
             col_p=np.full(max(info.nnz_stored, 1), -7, np.int32),
             val_p=np.full(max(info.nnz_stored, 1), -7, A.val.dtype),
             sched=np.full(max(4 * info.n_chunks, 1), -7, np.int32))
    L.pjds_convert(info, row_ptr, np.ascontiguousarray(A.col, np.int32), np.ascontiguousarray(A.val),
                   h["perm"], h["row_len"], h["offsets"], h["col_p"], h["val_p"],
                   h["sched"] if info.n_chunks else None)
    h["perm"] = h["perm"][:info.n_rows]
    h["row_len"] = h["row_len"][:info.n_pad]
    h["offsets"] = h["offsets"][:info.n_offsets]
    h["col_p"] = h["col_p"][:info.nnz_stored]
    h["val_p"] = h["val_p"][:info.nnz_stored]
    h["sched"] = h["sched"][:4 * info.n_chunks].reshape(-1, 4)
    return info, h


def assert_same(A, b_r=64, window=0, layout="jd", symmetric=False, split_len=0, lanes=1):
    info, h = lib_convert(A, b_r, window, layout, symmetric, split_len, lanes)
    P = oracle.pjds_build(A, b_r, window if window else None, layout, symmetric, lanes=lanes)
    assert info.n_pad == P["n_pad"] and info.nnz_stored == P["nnz_stored"]
    assert info.max_row_len == P["max_row_len"] and info.n_blocks == P["n_blocks"]
    for k in ("perm", "row_len", "offsets", "col_p"):
        assert np.array_equal(h[k], P[k]), k
    # values are copies: compare the bit patterns
    assert h["val_p"].dtype == P["val_p"].dtype
    assert np.array_equal(h["val_p"].view(np.uint8), np.ascontiguousarray(P["val_p"]).view(np.uint8))
    return info, h, P


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("b_r", [32, 64, 128])
@pytest.mark.parametrize("layout", ["jd", "block"])
def test_random_global(seed, b_r, layout):
    A = synth.random_csr(1000 + 37 * seed, 700, seed, max_len=40)
    assert_same(A, b_r=b_r, layout=layout)


@pytest.mark.parametrize("seed", range(2))
@pytest.mark.parametrize("b_r,window", [(32, 64), (64, 64), (64, 256), (128, 128), (128, 512)])
def test_random_windows(seed, b_r, window):
    A = synth.random_csr(3001, 900, seed + 5, max_len=30)
    assert_same(A, b_r=b_r, window=window, layout="block")


@pytest.mark.parametrize("b_r", [32, 64, 128])
def test_symmetric_and_float32(b_r):
    A = synth.hh_like(20000, seed=11)
    assert_same(A, b_r=b_r, symmetric=True)
    assert_same(A.astype(np.float32), b_r=b_r, layout="block")


def test_config1_laplacian():
    info, h, P = assert_same(synth.laplacian_2d(128))
    assert info.nnz_stored == 81472 and h["offsets"].tolist() == [0, 16384, 32768, 49152, 65536, 81472]


@pytest.mark.parametrize("window", [0, 1 << 10, 1 << 12])
def test_powerlaw_reduced(window):
    A = synth.powerlaw(1 << 16, seed=3, l_max=4096)
    assert_same(A, b_r=64, window=window, layout="block" if window else "jd")


def test_hh_like_reduced_both_dtypes():
    A = synth.hh_like(1 << 18, seed=2)
    assert_same(A, b_r=64)
    assert_same(A.astype(np.float32), b_r=64)


@pytest.mark.parametrize("n_rows,n_cols", [(0, 0), (0, 5), (1, 1), (5, 0), (63, 10), (65, 1), (129, 3)])
def test_degenerate_shapes(n_rows, n_cols):
    A = synth.random_csr(n_rows, n_cols, 2, max_len=5, empty_frac=0.5)
    for b_r in (32, 64, 128):
        for layout in ("jd", "block"):
            assert_same(A, b_r=b_r, layout=layout)


def test_all_rows_empty_and_one_full_row():
    A = synth.CSR(300, 300, np.zeros(301, np.int64), np.zeros(0, np.int32), np.zeros(0))
    info, h, _ = assert_same(A)
    assert info.nnz_stored == 0 and h["offsets"].tolist() == [0]
    lens = np.ones(256, np.int64)
    lens[17] = 256
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([np.arange(256) if L_ == 256 else [i] for i, L_ in enumerate(lens)]).astype(np.int32)
    info, _, _ = assert_same(synth.CSR(256, 256, rp, col, np.ones(int(lens.sum()))), b_r=64)
    assert info.nnz_stored == 65 * 256 - 64        # (b_r+1) N - b_r, Sect. 2.1


def test_long_row_schedule():
    A = synth.powerlaw(1 << 15, seed=4, l_max=4096)
    info, h, P = assert_same(A, b_r=64, split_len=64)
    groups_max = P["row_len"].reshape(-1, 64).max(axis=1)
    long = np.flatnonzero(groups_max > 64)
    assert info.n_split_groups == len(long)
    assert info.n_chunks == int(sum(-(-groups_max[g] // 64) for g in long))
    s = h["sched"]
    # items of one group are consecutive, numbered 0..nc-1, and point at the group's first item
    w = 0
    for g in long:
        nc = -(-groups_max[g] // 64)
        assert np.array_equal(s[w:w + nc, 0], np.full(nc, g))
        assert np.array_equal(s[w:w + nc, 1], np.arange(nc))
        assert np.all(s[w:w + nc, 2] == nc) and np.all(s[w:w + nc, 3] == w)
        w += nc
    _, h2 = lib_convert(A, b_r=64, split_len=-1)
    assert h2["sched"].size == 0


@pytest.mark.parametrize("seed", range(3))
def test_ellr_matches_oracle(seed):
    A = synth.random_csr(777, 500, seed, max_len=25)
    for M in (A, A.astype(np.float32)):
        info = L.ellr_plan(M.n_rows, M.n_cols, M.row_ptr)
        rowmax = np.empty(info.n_pad, np.int32)
        col_e = np.empty(info.nnz_stored, np.int32)
        val_e = np.empty(info.nnz_stored, M.val.dtype)
        L.ellr_convert(info, M.row_ptr, M.col, M.val, rowmax, col_e, val_e)
        E = oracle.ellr_build(M, pad_to=64)
        assert info.n_pad == E["n_pad"] and info.max_row_len == E["max_len"]
        assert np.array_equal(rowmax, E["rowmax"]) and np.array_equal(col_e, E["col"])
        assert np.array_equal(val_e.view(np.uint8), np.ascontiguousarray(E["val"]).view(np.uint8))


def test_conversion_is_thread_count_independent(monkeypatch):
    A = synth.hh_like(300000, seed=5)
    _, h1 = lib_convert(A, b_r=64, layout="block")
    monkeypatch.setenv("PJDS_NUM_THREADS", "1")
    _, h2 = lib_convert(A, b_r=64, layout="block")
    for k in h1:
        assert np.array_equal(h1[k], h2[k]), k


@pytest.mark.parametrize("lanes", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("window", [0, 64, 256])
def test_lanes_per_row_layout(lanes, window):
    A = synth.powerlaw(3000, seed=21, l_max=300)
    info, h, P = assert_same(A, b_r=64 // lanes, window=window, layout="block", lanes=lanes)
    assert info.n_chunks == 0 and info.split_len == 0
    assert info.nnz_stored % 64 == 0


@pytest.mark.parametrize("lanes", [2, 8])
def test_lanes_symmetric_float32_ragged(lanes):
    A = synth.hh_like(5001, seed=22)
    assert_same(A, b_r=64 // lanes, layout="block", symmetric=True, lanes=lanes)
    assert_same(A.astype(np.float32), b_r=64 // lanes, window=128, layout="block", lanes=lanes)


@pytest.mark.parametrize("c0,c1", [(0, 0), (0, 3000), (700, 1900), (2999, 3000), (1200, 1200)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_split_columns_matches_oracle(c0, c1, dtype):
    # the library's local/non-local split against the oracle's row-by-row definition: every
    # array bit for bit, and the two parts together hold every entry exactly once
    from paper_1112_5588_amd.matrix import split_columns
    A = synth.random_csr(2001, 3000, 61, max_len=25, empty_frac=0.1).astype(dtype)
    loc, nl = split_columns(A, c0, c1)
    (rl, cl, vl), (rn, cn, vn) = oracle.split_columns(A, c0, c1)
    for got, ref in ((loc.row_ptr, rl), (loc.col, cl), (nl.row_ptr, rn), (nl.col, cn)):
        assert np.array_equal(got, ref)
    assert np.array_equal(loc.val.view(np.uint8), vl.view(np.uint8))
    assert np.array_equal(nl.val.view(np.uint8), vn.view(np.uint8))
    assert rl[-1] + rn[-1] == A.nnz
    assert np.all((cl >= c0) & (cl < c1)) and not np.any((cn >= c0) & (cn < c1))


def test_split_columns_refusals():
    A = synth.random_csr(50, 40, 62, max_len=5)
    rp = np.ascontiguousarray(A.row_ptr, np.int64)
    col = np.ascontiguousarray(A.col, np.int32)
    for c0, c1 in ((-1, 10), (10, 5), (0, 41)):
        with pytest.raises(L.PjdsError) as e:
            L.pjds_split_count(A.n_rows, A.n_cols, rp, col, c0, c1)
        assert e.value.code == L.PJDS_ERR_ARG
    bad = col.copy()
    bad[3] = 40
    with pytest.raises(L.PjdsError) as e:
        L.pjds_split_count(A.n_rows, A.n_cols, rp, bad, 0, 10)
    assert e.value.code == L.PJDS_ERR_INDEX
