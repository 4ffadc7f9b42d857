"""The product with a fused update (y = a A x + b z), the local/non-local split of a
row-distributed product assembled with it, and the Lanczos recurrence run on the GPU in the
permuted basis -- each against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import krylov
from paper_1112_5588_amd import PjdsMatrix
from paper_1112_5588_amd.matrix import split_columns
from parity import assert_rows, assert_rows_axpby

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("y_permuted", [False, True])
@pytest.mark.parametrize("alias", [False, True])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_axpby_matches_oracle(y_permuted, alias, dtype):
    A = synth.random_csr(9501, 7000, 31, max_len=40).astype(dtype)
    x = synth.dense_x(7000, 31)
    z = synth.dense_x(9501, 32)
    if dtype == np.float32:
        x = x.astype(np.float32).astype(np.float64)
        z = z.astype(np.float32).astype(np.float64)
    M = PjdsMatrix.from_csr(A, keep_host=True)
    perm = M.host["perm"]
    zb = z[perm] if y_permuted else z
    zd = dev(zb, M.dtype)
    y = zd if alias else torch.empty_like(zd)
    M.spmv_axpby(dev(x, M.dtype), y, alpha=-1.5, beta=0.25, z=zd, y_permuted=y_permuted)
    ref = krylov.axpby(A, x, -1.5, 0.25, z)
    if y_permuted:
        ref = ref[perm]
    assert oracle.rel_l2(host(y), ref) <= (1e-12 if dtype == np.float64 else 1e-5)
    assert_rows_axpby(host(y), A, x, -1.5, 0.25, z, 8 if dtype == np.float64 else 4,
                      rows=perm if y_permuted else None)


def test_axpby_long_row_work_items_and_identity():
    A = synth.powerlaw(1 << 15, seed=12, l_max=2048)
    x = synth.dense_x(A.n_cols, 12)
    z = synth.dense_x(A.n_rows, 13)
    M = PjdsMatrix.from_csr(A, split_len=64)
    assert M.info.n_chunks > 0
    y = torch.empty(A.n_rows, dtype=torch.float64, device="cuda")
    M.spmv_axpby(dev(x), y, alpha=2.0, beta=-1.0, z=dev(z))
    assert oracle.rel_l2(host(y), krylov.axpby(A, x, 2.0, -1.0, z)) <= 1e-12
    assert_rows_axpby(host(y), A, x, 2.0, -1.0, z)
    # alpha = 1 without z is the plain product, bit for bit
    M.spmv_axpby(dev(x), y)
    assert torch.equal(y, M.spmv(dev(x)))


def test_local_nonlocal_split_adds_up_to_the_product():
    # rows split over "processes", here one: the local part covers the middle half of the
    # columns, the non-local part the rest; y is written by the first and updated by the second
    A = synth.hh_like(60000, seed=14)
    x = synth.dense_x(A.n_cols, 14)
    loc, nl = split_columns(A, 15000, 45000)
    assert loc.row_ptr[-1] + nl.row_ptr[-1] == A.nnz
    ML, MN = PjdsMatrix.from_csr(loc), PjdsMatrix.from_csr(nl)
    xd = dev(x)
    y = ML.spmv(xd)
    MN.spmv_axpby(xd, y, alpha=1.0, beta=1.0, z=y)
    # the two parts' sums added once more: one extra rounded term per row
    assert_rows(host(y), A, x, extra_terms=1)


@pytest.mark.parametrize("path", ["plain", "lds"])
def test_lanczos_coefficients_match_oracle(path):
    A = synth.hh_like(50000, seed=15)
    v = synth.dense_x(A.n_cols, 15)
    kw = dict(layout="block", sort_window=256) if path == "lds" else {}
    M = PjdsMatrix.from_csr(A, symmetric=True, keep_host=True, **kw)
    perm = M.host["perm"]
    a, b = M.lanczos(dev(v[perm]), 30, x_halo=512 if path == "lds" else -1, tile_rows=512 if path == "lds" else 0)
    ra, rb = krylov.lanczos(A, v, 30)
    assert np.allclose(host(a), ra, rtol=1e-8, atol=1e-10)
    assert np.allclose(host(b), rb, rtol=1e-8, atol=1e-10)


def test_lanczos_ritz_values_laplacian_closed_form():
    A = synth.laplacian_2d(32)
    M = PjdsMatrix.from_csr(A, symmetric=True, keep_host=True)
    v = synth.dense_x(A.n_cols, 3)
    a, b = M.lanczos(dev(v[M.host["perm"]]), 200)
    r = krylov.ritz_values(host(a), host(b))
    assert abs(r.max() - (4 + 4 * np.cos(np.pi / 33))) < 1e-9
    assert abs(r.min() - (4 - 4 * np.cos(np.pi / 33))) < 1e-9


def test_lanczos_is_deterministic_and_graph_capturable():
    A = synth.hh_like(40000, seed=16)
    M = PjdsMatrix.from_csr(A, symmetric=True, layout="block", sort_window=256, keep_host=True)
    v0 = dev(synth.dense_x(A.n_cols, 16)[M.host["perm"]])
    bufs = M.lanczos_buffers()
    alpha = torch.empty(12, dtype=torch.float64, device="cuda")
    beta = torch.empty(13, dtype=torch.float64, device="cuda")
    M.lanczos(v0, 12, x_halo=512, tile_rows=512, alpha=alpha, beta=beta, buffers=bufs)
    ref_a, ref_b = alpha.clone(), beta.clone()
    M.lanczos(v0, 12, x_halo=512, tile_rows=512, alpha=alpha, beta=beta, buffers=bufs)
    assert torch.equal(alpha, ref_a) and torch.equal(beta, ref_b)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            M.lanczos(v0, 12, x_halo=512, tile_rows=512, alpha=alpha, beta=beta, buffers=bufs)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        alpha.fill_(float(rep))
        beta.fill_(-1.0)
        bufs["vectors"].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(alpha, ref_a) and torch.equal(beta, ref_b), rep


def test_lanczos_one_byte_lengths_are_bitwise_the_int32_ones():
    """The staged Lanczos product reading one-byte row lengths gives the same coefficients bit
    for bit; under graph capture with no one-byte copy made yet, the default keeps the int32
    lengths (the copy would exist only inside the graph)."""
    A = synth.hh_like(40000, seed=17)
    M = PjdsMatrix.from_csr(A, symmetric=True, layout="block", sort_window=512, keep_host=True)
    v0 = dev(synth.dense_x(A.n_cols, 17)[M.host["perm"]])
    bufs = M.lanczos_buffers()
    a32 = torch.empty(10, dtype=torch.float64, device="cuda")
    b32 = torch.empty(11, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            M.lanczos(v0, 10, x_halo=768, tile_rows=1024, alpha=a32, beta=b32, buffers=bufs)
    torch.cuda.current_stream().wait_stream(s)
    assert "row_len8" not in M.d
    g.replay()
    torch.cuda.synchronize()
    a8, b8 = M.lanczos(v0, 10, x_halo=768, tile_rows=1024, len8=True)
    ai, bi = M.lanczos(v0, 10, x_halo=768, tile_rows=1024, len8=False)
    assert torch.equal(a8, ai) and torch.equal(b8, bi)
    assert torch.equal(a32, ai) and torch.equal(b32, bi)
    ra, rb = krylov.lanczos(A, synth.dense_x(A.n_cols, 17), 10)
    assert np.allclose(host(a8), ra, rtol=1e-8, atol=1e-10)
    assert np.allclose(host(b8), rb, rtol=1e-8, atol=1e-10)
    with pytest.raises(ValueError):
        M.lanczos(v0, 10, x_halo=-1, len8=True)
