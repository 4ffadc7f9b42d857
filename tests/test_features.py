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
