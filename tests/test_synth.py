"""The input generators: reproducible, and the torch twin of a generator bit-identical to it."""
import numpy as np
import pytest
import torch

import synth
from synth import torchgen


def test_streams_are_reproducible_and_addressable():
    a = synth.stream_u64(5, 3, 100)
    assert np.array_equal(a, synth.stream_u64(5, 3, 100))
    assert np.array_equal(a[40:], synth.stream_u64(5, 3, 60, start=40))
    assert not np.array_equal(a, synth.stream_u64(5, 4, 100))
    u = synth.uniform01(1, 1, 200000)
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.005


def test_splitmix64_reference_values():
    # SplitMix64 with state 0: the published first outputs of the generator
    z = np.array([0x9E3779B97F4A7C15], dtype=np.uint64)
    assert int(synth._mix(z)[0]) == 0xE220A8397B1DCDAF
    z = np.array([(2 * 0x9E3779B97F4A7C15) % (1 << 64)], dtype=np.uint64)
    assert int(synth._mix(z)[0]) == 0x6E789E6AA1B965F4


@pytest.mark.parametrize("n,seed", [(1000, 1000), (4097, 3), (20000, 1017)])
def test_torch_twin_is_bit_identical(n, seed):
    A = synth.banded_stratified(n, seed)
    rp, col, val = torchgen.banded_stratified(n, seed)
    assert np.array_equal(A.row_ptr, rp.numpy())
    assert np.array_equal(A.col, col.numpy())
    assert np.array_equal(A.val.view(np.uint64), val.numpy().view(np.uint64))
    assert np.array_equal(synth.dense_x(n, seed).view(np.uint64), torchgen.dense_x(n, seed).numpy().view(np.uint64))


def test_stratified_columns_distinct_sorted_in_window():
    A = synth.banded_stratified(9000, 11, halo=300)
    lens = np.diff(A.row_ptr)
    assert lens.min() >= 3 and lens.max() <= 60
    for r in range(0, 9000, 97):
        c = A.col[A.row_ptr[r]:A.row_ptr[r + 1]].astype(np.int64)
        assert np.all(np.diff(c) > 0)
        assert c.min() >= max(0, r - 300) and c.max() <= min(8999, r + 300)


def test_generator_shapes():
    A = synth.hh_like(100000, seed=2)
    L = np.diff(A.row_ptr)
    assert L.min() >= 3 and L.max() <= 21
    M = A.row_ptr
    # symmetric pattern and values
    import scipy.sparse as sp
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    assert abs(S - S.T).max() == 0
    P = synth.powerlaw(1 << 16, seed=3)
    L = np.diff(P.row_ptr)
    assert L.min() >= 2 and L.max() <= 4096 and 9 < L.mean() < 15
    sizes = synth.uneven_batch_sizes(512)
    assert sizes.min() >= 1000 and sizes.max() <= 500000
