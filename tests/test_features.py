"""Tuner features: the library (C++) against the oracle's numpy definitions, and the oracle
against closed forms."""
import numpy as np
import pytest

import synth
from oracle.features import features as ref_features
from paper_1112_5588_amd import _lib as L


def lib_features(A):
    return L.pjds_features(A.n_rows, A.n_cols, np.ascontiguousarray(A.row_ptr, np.int64),
                           np.ascontiguousarray(A.col, np.int32))


def test_oracle_laplacian_closed_forms():
    A = synth.laplacian_2d(128)
    f = ref_features(A)
    assert f[0] == 14.0 and f[1] == np.log2(81409.0)
    assert f[2] == 81408 / 16384 and f[6] == 3 and f[7] == np.log2(6.0) and f[9] == 0
    # offsets -128, -1, 0, 1, 128 only; |d| <= 64 on the 3 central diagonals
    assert np.isclose(f[21], np.log(5 / 81408)) and f[22] == 1.0
    assert np.isclose(f[19], (16384 + 2 * (16384 - 128)) / 81408) and f[20] == 1.0
    assert np.isclose(f[16], 128 / 16384)
    # pJDS global sort stores 81472 entries (Sect. 2.1 example worked in the tests of the oracle)
    assert np.isclose(f[14], 81472 / 81408)
    assert np.isclose(f[13], np.log2((16384 * 5 + 1) / 81408))


def test_oracle_constant_rows():
    n, Lr = 640, 7
    rp = np.arange(n + 1, dtype=np.int64) * Lr
    col = ((np.arange(n)[:, None] + np.arange(Lr)[None, :]) % n).ravel().astype(np.int32)
    f = ref_features(synth.CSR(n, n, rp, col, np.ones(n * Lr)))
    assert f[3] == 0 and f[4] == 0 and f[5] == 0 and f[8] == 1.0
    assert f[10] == f[11] == f[12] == 1.0
    assert f[14] == 1.0 and f[15] == 1.0 and f[13] == np.log2((n * Lr + 1) / (n * Lr))


@pytest.mark.parametrize("make", [
    lambda: synth.laplacian_2d(128),
    lambda: synth.hh_like(200000, seed=4),
    lambda: synth.powerlaw(1 << 17, seed=5),
    lambda: synth.banded_stratified(50000, 6),
    lambda: synth.random_csr(3001, 2000, 7, max_len=30),
    lambda: synth.random_csr(70, 5, 8, max_len=4, empty_frac=0.5),
])
def test_library_matches_oracle(make):
    A = make()
    a, b = lib_features(A), ref_features(A)
    assert np.allclose(a, b.astype(np.float32), rtol=2e-6, atol=1e-6), np.c_[a, b]


def test_sampling_kicks_in_above_2_20_entries():
    A = synth.hh_like(200000, seed=9)              # ~2.4M entries: every 3rd entry sampled
    assert A.nnz > (1 << 21)
    assert np.allclose(lib_features(A), ref_features(A).astype(np.float32), rtol=2e-6, atol=1e-6)


def test_features_reject_bad_input():
    with pytest.raises(L.PjdsError):
        L.pjds_features(0, 5, np.zeros(1, np.int64), np.zeros(0, np.int32))


def test_oracle_laplacian_offset_moments_and_segment_reuse():
    # 128 x 128 five-point Laplacian, 81408 entries (fewer than 2^20, so every entry counts):
    # 16384 on offset 0, 2 * 127 * 128 = 32512 on offsets +-1 and 32512 on offsets +-128
    A = synth.laplacian_2d(128)
    f = ref_features(A)
    n, e1, e128 = 81408, 32512, 32512
    mean = (e1 * 1 + e128 * 128) / n
    second = (e1 * 1 + e128 * 128 ** 2) / n
    assert abs(f[17] - mean / 16384) <= 1e-15
    # population standard deviation (divided by the count, not count - 1)
    assert abs(f[18] - np.sqrt(second - mean ** 2) / 16384) <= 1e-15
    # f[23], counted by hand on the 256 blocks of 64 rows (half a grid row each): a block
    # holds 64 * 5 entries minus 64 per missing grid neighbour row and minus the one row at
    # the grid edge (column 0 or 127) with no left or right neighbour; its columns fall in
    # 5 segments of 16 around the diagonal plus 4 for each neighbour grid row present.
    # Interior grid rows: 319 entries / 13 segments; first and last grid row: 255 / 9.
    expect = (252 * 319 / 13 + 4 * 255 / 9) / 256
    assert abs(f[23] - expect) <= 1e-13


def test_oracle_segment_reuse_hand_example():
    # 64 rows, each with the 4 columns 0, 5, 17, 40: the block's 256 entries fall in the
    # 16-column segments 0, 1, 2 (columns 0..15, 16..31, 32..47): 256 / 3
    n = 64
    rp = np.arange(n + 1, dtype=np.int64) * 4
    col = np.tile(np.array([0, 5, 17, 40], np.int32), n)
    f = ref_features(synth.CSR(n, 48, rp, col, np.ones(4 * n)))
    assert abs(f[23] - 256 / 3) <= 1e-13
    # offsets col - row over the sampled entries (all 256): mean and population std of |d| / 64
    rows = np.repeat(np.arange(n), 4)
    a = np.abs(col.astype(np.int64) - rows) / 64.0
    assert abs(f[17] - a.sum() / 256) <= 1e-15
    assert abs(f[18] - np.sqrt((a ** 2).sum() / 256 - (a.sum() / 256) ** 2)) <= 1e-15
    assert f[16] == 63 / 64                       # row 63, column 0


def test_oracle_offset_sampling_rule():
    # a matrix of 2^20 + 1 entries is sampled every 2nd entry (s = ceil(nnz / 2^20) = 2): one
    # entry per row on offset +1 and one on -1 alternating, so every sampled entry (even k)
    # is the row's first entry, offset -1, except row 0 whose first entry is offset +1
    n = (1 << 19) + 1
    rp = np.zeros(n + 1, np.int64)
    lens = np.full(n, 2)
    lens[0] = 1
    lens[-1] = 2
    rp[1:] = np.cumsum(lens)
    nnz = int(rp[-1])
    col = np.empty(nnz, np.int32)
    col[0] = 1
    for_rows = np.arange(1, n)
    col[rp[1:-1]] = (for_rows - 1).astype(np.int32)
    col[rp[1:-1] + 1] = np.minimum(for_rows + 1, n - 1).astype(np.int32)
    assert nnz == (1 << 20) + 1
    f = ref_features(synth.CSR(n, n, rp, col, np.ones(nnz)))
    sampled = np.arange(0, nnz, 2)
    assert len(sampled) == (1 << 19) + 1
    # distinct offsets among the samples: +1 (row 0) and -1 (every other sampled entry)
    assert abs(f[21] - np.log(2 / len(sampled))) <= 1e-12
    assert f[22] == 1.0
