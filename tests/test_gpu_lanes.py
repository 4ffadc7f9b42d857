"""GPU parity of pJDS with T lanes per row (the sliced ELLR-T idea named in the outlook,
Sect. 4) against the CPU oracle: FP64 within 1e-12 relative L2, FP32 within 1e-5,
integer-valued data bit-exact, results reproducible bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import krylov
from paper_1112_5588_amd import PjdsMatrix
from parity import assert_rows, assert_rows_axpby

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def run(A, x, lanes, window=0, y_permuted=False, symmetric=False):
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=window, lanes=lanes, symmetric=symmetric,
                            keep_host=True)
    assert M.info.block_height == 64 // lanes and M.info.n_chunks == 0
    perm = M.host["perm"]
    y = host(M.spmv(dev(x[perm] if symmetric else x, M.dtype), y_permuted=y_permuted))
    ref = oracle.csr_spmv(A, x)
    # every row against its own error bound (the T partial sums are added in a tree)
    assert_rows(y, A, x, 8 if M.dtype == torch.float64 else 4, rows=perm if y_permuted else None)
    return M, y, (ref[perm] if y_permuted else ref)


@pytest.mark.parametrize("lanes", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("y_permuted", [False, True])
def test_random_ragged_matches_oracle(lanes, y_permuted):
    A = synth.random_csr(5003, 4000, lanes, max_len=150)
    x = synth.dense_x(4000, lanes)
    M, y, ref = run(A, x, lanes, y_permuted=y_permuted)
    assert oracle.rel_l2(y, ref) <= 1e-12


@pytest.mark.parametrize("lanes", [2, 8, 32])
@pytest.mark.parametrize("window", [64, 1024])
def test_heavy_tail_windows_float32(lanes, window):
    A = synth.powerlaw(1 << 15, seed=30 + lanes, l_max=3000).astype(np.float32)
    x = synth.dense_x(A.n_cols, 30).astype(np.float32).astype(np.float64)
    M, y, ref = run(A, x, lanes, window=window)
    assert oracle.rel_l2(y, ref) <= 1e-5


@pytest.mark.parametrize("lanes", [2, 4, 64])
def test_integer_data_bit_exact_and_reproducible(lanes):
    A = synth.laplacian_2d(128)
    M, y, ref = run(A, np.ones(A.n_cols), lanes)
    assert np.array_equal(y, ref)
    x = dev(synth.dense_x(A.n_cols, 8))
    y1 = M.spmv(x)
    y2 = M.spmv(x)
    assert torch.equal(y1, y2)


def test_symmetric_basis_and_fused_update():
    A = synth.hh_like(70001, seed=31)
    x = synth.dense_x(A.n_cols, 31)
    z = synth.dense_x(A.n_rows, 32)
    M, y, ref = run(A, x, 4, y_permuted=True, symmetric=True)
    assert oracle.rel_l2(y, ref) <= 1e-12
    perm = M.host["perm"]
    yz = dev(z[perm])
    M.spmv_axpby(dev(x[perm]), yz, alpha=0.5, beta=-2.0, z=yz, y_permuted=True)
    assert oracle.rel_l2(host(yz), krylov.axpby(A, x, 0.5, -2.0, z)[perm]) <= 1e-12
    assert_rows_axpby(host(yz), A, x, 0.5, -2.0, z, rows=perm)


def test_lanczos_plain_path_takes_lanes():
    A = synth.hh_like(30000, seed=33)
    v = synth.dense_x(A.n_cols, 33)
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=256, lanes=2, symmetric=True, keep_host=True)
    a, b = M.lanczos(dev(v[M.host["perm"]]), 20, x_halo=-1)
    ra, rb = krylov.lanczos(A, v, 20)
    assert np.allclose(host(a), ra, rtol=1e-8, atol=1e-10)
    assert np.allclose(host(b), rb, rtol=1e-8, atol=1e-10)


def test_edge_cases():
    # every row empty; fewer rows than a block; one row much longer than a wave
    Z = synth.CSR(1000, 300, np.zeros(1001, np.int64), np.zeros(0, np.int32), np.zeros(0))
    M = PjdsMatrix.from_csr(Z, layout="block", lanes=8)
    y = torch.full((1000,), 3.0, dtype=torch.float64, device="cuda")
    M.spmv(dev(np.ones(300)), y)
    assert np.array_equal(host(y), np.zeros(1000))
    S = synth.random_csr(5, 40, 3, max_len=30)
    for lanes in (2, 64):
        _, y, ref = run(S, synth.dense_x(40, 3), lanes)
        assert oracle.rel_l2(y, ref) <= 1e-12
    n = 7000
    lens = np.full(n, 3, np.int64)
    lens[0] = 6000
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([np.arange(6000), (np.arange(3 * (n - 1)) * 7) % n]).astype(np.int32)
    L1 = synth.CSR(n, n, rp, col, synth.normal(34, 1, int(rp[-1])))
    for lanes in (16, 64):
        _, y, ref = run(L1, synth.dense_x(n, 34), lanes)
        assert oracle.rel_l2(y, ref) <= 1e-12


def test_powerlaw_full_size_sampled():
    # the heavy-tail workload at full size (N = 2^23, rows up to 4096) with 8 lanes per row
    A = synth.powerlaw(1 << 23, seed=3)
    x = synth.dense_x(A.n_cols, 3)
    M = PjdsMatrix.from_csr(A, layout="block", lanes=8, keep_host=True)
    y = host(M.spmv(dev(x)))
    rows = np.unique(np.concatenate([M.host["perm"][:2048],
                                     (synth.uniform01(79, 1, 4096) * A.n_rows).astype(np.int64)]))
    assert_rows(y[rows], A, x, rows=rows)
    assert np.array_equal(host(M.spmv(dev(x))), y)
