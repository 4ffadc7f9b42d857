"""GPU parity: the HIP kernels (through the C interface) against the CPU oracle on the same
seeded inputs.  FP64 within 1e-12 relative L2, FP32 within 1e-5; integer-valued data and
index arrays bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1112_5588_amd import CsrMatrix, EllrMatrix, PjdsMatrix
from paper_1112_5588_amd import _lib as L
from parity import assert_rows, assert_rows_mm

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def check_pjds(A, x, b_r=64, layout="jd", window=0, y_permuted=False, symmetric=False,
               split_len=0, tol=None):
    M = PjdsMatrix.from_csr(A, block_height=b_r, layout=layout, sort_window=window,
                            symmetric=symmetric, split_len=split_len, keep_host=True)
    perm = M.host["perm"]
    xin = x[perm] if symmetric else x
    y = host(M.spmv(dev(xin, M.dtype), y_permuted=y_permuted))
    # symmetric renumbering changes the basis of x only: slot i of the product is still
    # original row perm[i], written there (y_permuted) or scattered back to row perm[i]
    vb = 8 if M.dtype == torch.float64 else 4
    # slot i holds original row perm[i] when y is permuted
    assert_rows(y, A, x, vb, rows=perm if y_permuted else None, tol=tol)
    return M, y


# ------------------------------------------------------------------ config 1, exact cases

@pytest.mark.parametrize("layout", ["jd", "block"])
@pytest.mark.parametrize("y_permuted", [False, True])
def test_laplacian_times_ones_is_exact(layout, y_permuted):
    A = synth.laplacian_2d(128)
    M = PjdsMatrix.from_csr(A, block_height=64, layout=layout, keep_host=True)
    y = host(M.spmv(dev(np.ones(A.n_cols)), y_permuted=y_permuted))
    r, c = np.divmod(np.arange(A.n_rows), 128)
    expect = ((r == 0).astype(float) + (r == 127) + (c == 0) + (c == 127))
    if y_permuted:
        expect = expect[M.host["perm"]]
    assert np.array_equal(y, expect)


@pytest.mark.parametrize("b_r", [32, 64, 128])
def test_integer_data_bit_exact(b_r):
    # small integers: every sum is exact in any order, so the GPU must reproduce it bit for bit
    A = synth.random_csr(5000, 3000, 8, max_len=30, integer=True)
    x = synth.dense_x(3000, 8, integer=True)
    M = PjdsMatrix.from_csr(A, block_height=b_r)
    assert np.array_equal(host(M.spmv(dev(x))), oracle.csr_spmv(A, x))


def test_config1_random_x():
    A = synth.laplacian_2d(128)
    x = synth.dense_x(A.n_cols, 1)
    for layout in ("jd", "block"):
        for yp in (False, True):
            check_pjds(A, x, layout=layout, y_permuted=yp)


# ------------------------------------------------------------------ format options

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("b_r", [32, 64, 128])
@pytest.mark.parametrize("layout", ["jd", "block"])
@pytest.mark.parametrize("y_permuted", [False, True])
def test_random_matrix_tiles_and_ragged_tail(dtype, b_r, layout, y_permuted):
    # 9501 rows: 37 workgroups of 256 rows plus a ragged tail of 29 rows
    A = synth.random_csr(9501, 7000, 21, max_len=45, empty_frac=0.1).astype(dtype)
    x = synth.dense_x(7000, 21)
    if dtype == np.float32:
        x = x.astype(np.float32).astype(np.float64)
    check_pjds(A, x, b_r=b_r, layout=layout, y_permuted=y_permuted)


@pytest.mark.parametrize("window", [64, 1024, 4096])
@pytest.mark.parametrize("b_r", [32, 64, 128])
def test_sort_windows(window, b_r):
    if window % b_r:
        pytest.skip("window must hold whole blocks")
    A = synth.powerlaw(20000, seed=5, l_max=300)
    check_pjds(A, synth.dense_x(20000, 5), b_r=b_r, layout="block", window=window)


@pytest.mark.parametrize("y_permuted", [False, True])
def test_symmetric_permuted_basis(y_permuted):
    A = synth.hh_like(50000, seed=9)
    check_pjds(A, synth.dense_x(50000, 9), symmetric=True, y_permuted=y_permuted)


@pytest.mark.parametrize("split_len", [-1, 64, 128, 256, 512])
@pytest.mark.parametrize("b_r", [32, 64, 128])
def test_long_rows_split(split_len, b_r):
    A = synth.powerlaw(1 << 16, seed=6, l_max=4096)
    x = synth.dense_x(A.n_cols, 6)
    M, y1 = check_pjds(A, x, b_r=b_r, split_len=split_len)
    if split_len > 0:
        assert M.info.n_chunks > 0
    # bitwise reproducible run to run, and independent of the XCD renumbering
    xd = dev(x)
    for remap in (True, False, True):
        assert np.array_equal(host(M.spmv(xd, xcd_remap=remap)), y1)


def test_padding_never_enters_the_sum():
    # column 0 is never referenced; padding slots point at column 0 -> x[0] = NaN must not leak
    A = synth.random_csr(3000, 2000, 4, max_len=40)
    A = synth.CSR(A.n_rows, A.n_cols + 1, A.row_ptr, A.col + 1, A.val)
    x = synth.dense_x(A.n_cols, 4)
    x[0] = np.nan
    for b_r in (32, 64, 128):
        M = PjdsMatrix.from_csr(A, block_height=b_r)
        assert M.info.nnz_stored > A.nnz
        y = host(M.spmv(dev(x)))
        assert np.all(np.isfinite(y))
        assert_rows(y, A, x)


def test_empty_inputs():
    Z = synth.CSR(1000, 500, np.zeros(1001, np.int64), np.zeros(0, np.int32), np.zeros(0))
    M = PjdsMatrix.from_csr(Z)
    y = torch.full((1000,), 7.0, dtype=torch.float64, device="cuda")
    M.spmv(dev(np.ones(500)), y)
    assert np.array_equal(host(y), np.zeros(1000))
    E = synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert PjdsMatrix.from_csr(E).spmv(torch.zeros(0, dtype=torch.float64, device="cuda")).numel() == 0


# ------------------------------------------------------------------ comparison formats

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_ellr_parity(dtype):
    for A in (synth.laplacian_2d(128), synth.random_csr(9501, 7000, 3, max_len=45)):
        A = A.astype(dtype)
        x = synth.dense_x(A.n_cols, 3)
        if dtype == np.float32:
            x = x.astype(np.float32).astype(np.float64)
        E = EllrMatrix.from_csr(A)
        y = host(E.spmv(dev(x, E.dtype)))
        assert_rows(y, A, x, 8 if E.dtype == torch.float64 else 4)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("variant", [1, 4, 16, 64])
def test_csr_parity(dtype, variant):
    A = synth.random_csr(9501, 7000, 13, max_len=45).astype(dtype)
    x = synth.dense_x(7000, 13)
    if dtype == np.float32:
        x = x.astype(np.float32).astype(np.float64)
    C = CsrMatrix.from_csr(A)
    y1 = host(C.spmv(dev(x, C.dtype), variant=variant))
    assert_rows(y1, A, x, 8 if C.dtype == torch.float64 else 4)
    assert np.array_equal(host(C.spmv(dev(x, C.dtype), variant=variant)), y1)


# ------------------------------------------------------------------ many right-hand sides

@pytest.mark.parametrize("k", [1, 3, 4, 8, 16, 32])
@pytest.mark.parametrize("t", [1, 2, 4, 8, 16, 32])
@pytest.mark.parametrize("vpl", [1, 2, 4])
def test_spmmv_config1(k, t, vpl):
    if k % vpl or t % vpl:
        pytest.skip("k and the tile must be multiples of the vectors per lane")
    A = synth.laplacian_2d(128)
    X = synth.dense_x(A.n_cols, 40, k=k).reshape(A.n_cols, k)
    M = PjdsMatrix.from_csr(A)
    Y = host(M.spmmv(dev(X), vectors_per_tile=t, vectors_per_lane=vpl))
    assert_rows_mm(Y, A, X)
    if k == 1:
        assert np.array_equal(Y[:, 0], host(M.spmv(dev(X[:, 0]))))


@pytest.mark.parametrize("b_r,layout,k,t,vpl", [(32, "block", 8, 8, 2), (64, "jd", 12, 16, 4), (128, "block", 6, 4, 2)])
def test_spmmv_wide_lanes_ragged_tiles(b_r, layout, k, t, vpl):
    # k not a multiple of the tile: the last tile is partly outside [0, k)
    A = synth.random_csr(9501, 7000, 19, max_len=45).astype(np.float64)
    X = synth.dense_x(7000, 43, k=k).reshape(7000, k)
    M = PjdsMatrix.from_csr(A, block_height=b_r, layout=layout, sort_window=1024 if layout == "block" else 0)
    Y = host(M.spmmv(dev(X), vectors_per_tile=t, vectors_per_lane=vpl))
    assert_rows_mm(Y, A, X)
    Y32 = host(PjdsMatrix.from_csr(A.astype(np.float32)).spmmv(dev(X, torch.float32), vectors_per_tile=t, vectors_per_lane=vpl))
    assert_rows_mm(Y32, A.astype(np.float32), X.astype(np.float32).astype(np.float64), value_bytes=4)


def test_spmmv_rejects_misaligned_lanes():
    A = synth.laplacian_2d(32)
    M = PjdsMatrix.from_csr(A)
    with pytest.raises(L.PjdsError):
        M.spmmv(dev(np.ones((A.n_cols, 6))), vectors_per_tile=8, vectors_per_lane=4)    # 6 % 4


@pytest.mark.parametrize("b_r,layout", [(32, "jd"), (64, "block"), (128, "jd")])
def test_spmmv_random(b_r, layout):
    A = synth.random_csr(9501, 7000, 17, max_len=45)
    X = synth.dense_x(7000, 41, k=5).reshape(7000, 5)
    M = PjdsMatrix.from_csr(A, block_height=b_r, layout=layout, keep_host=True)
    for yp in (False, True):
        Y = host(M.spmmv(dev(X), vectors_per_tile=4, vectors_per_lane=1, y_permuted=yp))
        assert_rows_mm(Y, A, X, rows=M.host["perm"] if yp else None)


@pytest.mark.parametrize("window", [256, 4096])
def test_spmmv_xcd_renumbering_is_bitwise_identical(window):
    # renumbering workgroups changes which XCD runs a tile, not the arithmetic
    A = synth.hh_like(100003, seed=18)
    X = dev(synth.dense_x(A.n_cols, 42, k=8).reshape(A.n_cols, 8))
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=window, keep_host=True)
    Y0 = M.spmmv(X, vectors_per_tile=8, vectors_per_lane=4, y_permuted=True)
    Y1 = M.spmmv(X, vectors_per_tile=8, vectors_per_lane=4, y_permuted=True, xcd_remap=True)
    assert torch.equal(Y0, Y1)
    assert_rows_mm(host(Y1), A, host(X), rows=M.host["perm"])


# ------------------------------------------------------------------ SpMMV with X staged in LDS

@pytest.mark.parametrize("k,t,vpl", [(1, 1, 1), (4, 4, 4), (8, 8, 4), (12, 8, 4), (16, 16, 4), (32, 16, 4),
                                     (6, 4, 2), (3, 4, 1)])
@pytest.mark.parametrize("window,halo,tile", [(256, 512, 1024), (128, 0, 256), (512, 3000, 512), (192, 700, 320)])
def test_spmmv_xlds_equals_spmmv_bitwise(k, t, vpl, window, halo, tile):
    # ragged row count (partial tile, partial wave), partial vector tiles (k = 12 with t = 8,
    # lanes past k), halos from none to wider than the 64 KiB cap, tiles that divide the
    # window, are divided by it, or neither; the same FMAs in the same order as pjds_spmmv
    A = synth.hh_like(30011, seed=43, band=600)
    X = dev(synth.dense_x(A.n_cols, 43, k=k).reshape(A.n_cols, k))
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=window, keep_host=True)
    for yp in (False, True):
        Y0 = M.spmmv(X, vectors_per_tile=t, vectors_per_lane=vpl, y_permuted=yp)
        Y1 = M.spmmv_xlds(X, vectors_per_tile=t, vectors_per_lane=vpl, x_halo=halo, tile_rows=tile, y_permuted=yp)
        assert torch.equal(Y0, Y1)
    assert_rows_mm(host(Y1), A, host(X), rows=M.host["perm"])


@pytest.mark.parametrize("k,t", [(4, 4), (8, 8)])
def test_spmmv_xlds_xcd_groups_with_a_tail(k, t):
    # 70001 rows in 256-row tiles: 274 workgroups, two whole rounds of 16 tiles per XCD and
    # 18 left in hardware order; every row computed once, bitwise as pjds_spmmv
    A = synth.hh_like(70001, seed=46)
    X = dev(synth.dense_x(A.n_cols, 46, k=k).reshape(A.n_cols, k))
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=256, keep_host=True)
    assert -(-M.info.n_pad // 256) == 274
    Y = torch.full((A.n_rows, k), float("nan"), dtype=torch.float64, device="cuda")
    M.spmmv_xlds(X, Y, vectors_per_tile=t, vectors_per_lane=4, x_halo=512, tile_rows=256)
    assert torch.equal(Y, M.spmmv(X, vectors_per_tile=t, vectors_per_lane=4))
    assert_rows_mm(host(Y), A, host(X))


@pytest.mark.parametrize("b_r", [32, 128])
def test_spmmv_xlds_block_heights_float32_and_small(b_r):
    for n in (300, 5000):
        A = synth.hh_like(n, seed=44).astype(np.float32)
        X = synth.dense_x(A.n_cols, 44, k=4).reshape(A.n_cols, 4).astype(np.float32)
        M = PjdsMatrix.from_csr(A, block_height=b_r, layout="block", sort_window=128)
        Y0 = M.spmmv(dev(X, torch.float32), vectors_per_tile=4, vectors_per_lane=4)
        Y1 = M.spmmv_xlds(dev(X, torch.float32), vectors_per_tile=4, vectors_per_lane=4, x_halo=256, tile_rows=256)
        assert torch.equal(Y0, Y1)
        assert_rows_mm(host(Y1), A, X.astype(np.float64), value_bytes=4)


def test_spmmv_xlds_refusals():
    A = synth.hh_like(2000, seed=45)
    X = dev(np.ones((A.n_cols, 4)))
    with pytest.raises(L.PjdsError):       # a global sort: nothing to stage by window
        PjdsMatrix.from_csr(A, layout="block").spmmv_xlds(X)
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=256)
    with pytest.raises(L.PjdsError):       # eight lanes per row
        M.spmmv_xlds(dev(np.ones((A.n_cols, 32))), vectors_per_tile=32, vectors_per_lane=4)
    with pytest.raises(L.PjdsError):
        M.spmmv_xlds(X, x_halo=-1)
    with pytest.raises(L.PjdsError):
        M.spmmv_xlds(X, tile_rows=100)


# ------------------------------------------------------------------ full-size workloads

@pytest.fixture(scope="module")
def hh_full():
    return synth.hh_like(1 << 22, seed=2)


def sampled_rows(A, rows):
    lens = np.diff(A.row_ptr)[rows]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    idx = np.concatenate([np.arange(A.row_ptr[r], A.row_ptr[r + 1]) for r in rows])
    return synth.CSR(len(rows), A.n_cols, rp, A.col[idx], A.val[idx])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_hh_like_full_size_sampled(hh_full, dtype):
    A = hh_full.astype(dtype) if dtype == np.float32 else hh_full
    x = synth.dense_x(A.n_cols, 2)
    if dtype == np.float32:
        x = x.astype(np.float32).astype(np.float64)
    M = PjdsMatrix.from_csr(A, block_height=64, keep_host=True)
    assert M.info.max_row_len <= 21
    y = host(M.spmv(dev(x, M.dtype), y_permuted=True))
    rows = np.unique(np.concatenate([np.arange(64), np.arange(A.n_rows - 64, A.n_rows),
                                     (synth.uniform01(77, 1, 4096) * A.n_rows).astype(np.int64)]))
    # permuted slot i holds original row perm[i]
    inv = np.empty_like(M.host["perm"])
    inv[M.host["perm"]] = np.arange(A.n_rows, dtype=np.int32)
    assert_rows(y[inv[rows]], A, x, 8 if M.dtype == torch.float64 else 4, rows=rows)
    # footprint: pJDS stores fewer entries than ELLPACK-R would
    E_info = EllrMatrix.plan(A)
    assert M.info.nnz_stored < E_info.nnz_stored


@pytest.mark.parametrize("window", [512, 256])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_headline_configuration_full_size(hh_full, dtype, window):
    # the benchmark's own launch: block layout, sort window 512 (or 256), x staged in LDS with halo 768
    # and 1024-row tiles (4096 tiles, all in whole XCD groups), two rows per lane, y in the
    # permuted basis; sampled rows against the oracle, the whole vector bitwise against the
    # plain kernel and the one-row LDS form, and run-to-run reproducibility
    A = hh_full.astype(dtype) if dtype == np.float32 else hh_full
    x = synth.dense_x(A.n_cols, 1)
    if dtype == np.float32:
        x = x.astype(np.float32).astype(np.float64)
    M = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=window, keep_host=True)
    xd = dev(x, M.dtype)
    yd = M.spmv_xlds(xd, x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True)
    y = host(yd)
    rows = np.unique(np.concatenate([np.arange(512), np.arange(A.n_rows - 512, A.n_rows),
                                     (synth.uniform01(81, 1, 4096) * A.n_rows).astype(np.int64)]))
    inv = np.empty_like(M.host["perm"])
    inv[M.host["perm"]] = np.arange(A.n_rows, dtype=np.int32)
    assert_rows(y[inv[rows]], A, x, 8 if M.dtype == torch.float64 else 4, rows=rows)
    assert torch.equal(yd, M.spmv(xd, y_permuted=True))
    assert torch.equal(yd, M.spmv_xlds(xd, x_halo=512, tile_rows=512, y_permuted=True))
    assert torch.equal(yd, M.spmv_xlds(xd, x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True))
    # the same launch with the int32 lengths
    assert torch.equal(yd, M.spmv_xlds(xd, x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True, len8=False))


@pytest.mark.parametrize("k,t,tile", [(4, 4, 1024), (8, 8, 512)])
def test_spmmv_xlds_full_size(hh_full, k, t, tile):
    # the benchmark's staged SpMMV launches on the full HH-like matrix: bitwise against the
    # unstaged kernel over all of Y, sampled rows against the oracle
    A = hh_full
    X_np = synth.dense_x(A.n_cols, 4, k=k).reshape(A.n_cols, k)
    X = dev(X_np)
    M = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=256, keep_host=True)
    Y = M.spmmv_xlds(X, vectors_per_tile=t, vectors_per_lane=4, x_halo=512, tile_rows=tile, y_permuted=True)
    assert torch.equal(Y, M.spmmv(X, vectors_per_tile=t, vectors_per_lane=4, y_permuted=True))
    perm = M.host["perm"]
    rows_p = np.unique(np.concatenate([np.arange(256), np.arange(A.n_rows - 256, A.n_rows),
                                       (synth.uniform01(82, 1, 2048) * A.n_rows).astype(np.int64)]))
    assert_rows_mm(host(Y)[rows_p], A, X_np, rows=perm[rows_p])


def test_powerlaw_full_size_sampled():
    A = synth.powerlaw(1 << 23, seed=3)
    x = synth.dense_x(A.n_cols, 3)
    M = PjdsMatrix.from_csr(A, block_height=64, split_len=128, keep_host=True)
    assert M.info.max_row_len == 4096 and M.info.n_chunks > 0
    y = host(M.spmv(dev(x)))
    rows = np.unique(np.concatenate([M.host["perm"][:2048],          # the longest rows (split)
                                     (synth.uniform01(78, 1, 4096) * A.n_rows).astype(np.int64)]))
    assert_rows(y[rows], A, x, rows=rows)
    assert np.array_equal(host(M.spmv(dev(x))), y)


# ------------------------------------------------------------------ x staged in LDS

@pytest.mark.parametrize("b_r,window,halo,tile", [(64, 256, 1024, 0), (64, 1024, 512, 256), (32, 256, 0, 2048),
                                                  (128, 4096, 2048, 1024), (64, 512, 3000, 512), (64, 256, 512, 1024)])
@pytest.mark.parametrize("y_permuted", [False, True])
def test_xlds_matches_oracle_and_plain_kernel(b_r, window, halo, tile, y_permuted):
    # 9501 rows (ragged last workgroup), band plus far off-diagonals: some columns in the
    # staged window, some outside
    A = synth.hh_like(9501, seed=23, band=600)
    x = synth.dense_x(A.n_cols, 23)
    M = PjdsMatrix.from_csr(A, block_height=b_r, layout="block", sort_window=window, keep_host=True)
    xd = dev(x)
    y = host(M.spmv_xlds(xd, x_halo=halo, tile_rows=tile, y_permuted=y_permuted))
    assert_rows(y, A, x, rows=M.host["perm"] if y_permuted else None)
    # the same values reach the same FMAs in the same order: bit-identical to the plain kernel
    assert np.array_equal(y, host(M.spmv(xd, y_permuted=y_permuted)))
    # two adjacent rows per lane: again the same FMAs in the same order
    assert np.array_equal(y, host(M.spmv_xlds(xd, x_halo=halo, tile_rows=tile, y_permuted=y_permuted,
                                              two_rows=True)))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [300, 1000, 70001])
def test_xlds_two_rows_ragged_and_fused_update(dtype, n):
    # row counts that leave a partial tile and a partial 128-row wave; bitwise equal to the
    # plain kernel in every tile shape
    A = synth.hh_like(n, seed=24).astype(dtype) if dtype == np.float32 else synth.hh_like(n, seed=24)
    x = synth.dense_x(A.n_cols, 24)
    if dtype == np.float32:
        x = x.astype(np.float32).astype(np.float64)
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=256, keep_host=True)
    xd = dev(x, M.dtype)
    for tile in (256, 512, 1024):
        y = M.spmv_xlds(xd, x_halo=256, tile_rows=tile, two_rows=True)
        assert_rows(host(y), A, x, 8 if M.dtype == torch.float64 else 4)
        assert torch.equal(y, M.spmv(xd))


def test_xlds_float32_rectangular_and_wide_rows():
    A = synth.random_csr(5000, 3000, 29, max_len=60).astype(np.float32)
    x = synth.dense_x(3000, 29).astype(np.float32).astype(np.float64)
    M = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=1024)
    y = host(M.spmv_xlds(dev(x, torch.float32), x_halo=2048))
    assert_rows(y, A, x, 4)


def test_xlds_rejects_unsupported_layouts():
    A = synth.random_csr(20000, 20000, 30, max_len=10)
    xd = dev(synth.dense_x(20000, 30))
    with pytest.raises(L.PjdsError):
        PjdsMatrix.from_csr(A, layout="jd").spmv_xlds(xd)
    with pytest.raises(L.PjdsError):
        PjdsMatrix.from_csr(A, layout="block", sort_window=64).spmv_xlds(xd)       # not a multiple of 256
    with pytest.raises(L.PjdsError):
        PjdsMatrix.from_csr(A, layout="block", sort_window=1024).spmv_xlds(xd, x_halo=4000)  # > 64 KiB
    with pytest.raises(L.PjdsError):
        PjdsMatrix.from_csr(A, layout="block", sort_window=1024).spmv_xlds(xd, tile_rows=768)  # 768 vs 1024


@pytest.mark.parametrize("b_r,layout,window", [(64, "jd", 0), (32, "jd", 0), (128, "block", 0), (64, "block", 128),
                                               (64, "block", 512), (32, "block", 256)])
@pytest.mark.parametrize("y_permuted", [False, True])
def test_plain_two_rows_bitwise(b_r, layout, window, y_permuted):
    # two adjacent rows per lane: the same FMAs in the same order as one row per lane
    A = synth.random_csr(9503, 7000, 44, max_len=60)
    x = dev(synth.dense_x(7000, 44))
    M = PjdsMatrix.from_csr(A, block_height=b_r, layout=layout, sort_window=window, split_len=-1)
    y1 = M.spmv(x, y_permuted=y_permuted)
    y2 = M.spmv(x, y_permuted=y_permuted, two_rows=True)
    assert torch.equal(y1, y2)
    if not y_permuted:
        assert_rows(host(y2), A, host(x))


def test_plain_two_rows_float32_and_refusals():
    A = synth.hh_like(30001, seed=45).astype(np.float32)
    x = synth.dense_x(A.n_cols, 45).astype(np.float32).astype(np.float64)
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=256, split_len=-1)
    y = host(M.spmv(dev(x, torch.float32), two_rows=True))
    assert_rows(y, A, x, 4)
    P = synth.powerlaw(1 << 14, seed=46, l_max=2000)
    with pytest.raises(L.PjdsError) as e:                   # long rows split into work items
        PjdsMatrix.from_csr(P, split_len=64).spmv(dev(synth.dense_x(P.n_cols, 46)), two_rows=True)
    assert e.value.code == L.PJDS_ERR_UNSUPPORTED
    with pytest.raises(L.PjdsError) as e:                   # a window of 64 rows
        PjdsMatrix.from_csr(A, layout="block", sort_window=64, split_len=-1).spmv(dev(x, torch.float32), two_rows=True)
    assert e.value.code == L.PJDS_ERR_ARG


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("two_rows,tile,halo,window", [(True, 1024, 768, 256), (True, 512, 256, 512),
                                                       (False, 512, 512, 256), (False, 1024, 256, 1024)])
def test_xlds_one_byte_lengths_give_the_same_bits(dtype, two_rows, tile, halo, window):
    """PJDS_ROW_LEN8: the staged products read one-byte copies of the lengths and give the
    same sums bit for bit; the copies are the lengths themselves."""
    A = synth.hh_like(70001, seed=31)
    A = A.astype(dtype) if dtype == np.float32 else A
    x = synth.dense_x(A.n_cols, 31)
    if dtype == np.float32:
        x = x.astype(np.float32).astype(np.float64)
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=window, keep_host=True)
    r8 = M.row_len8()
    assert r8 is not None and np.array_equal(host(r8)[:M.info.n_pad], M.host["row_len"].astype(np.uint8))
    xd = dev(x, M.dtype)
    y8 = M.spmv_xlds(xd, x_halo=halo, tile_rows=tile, y_permuted=True, two_rows=two_rows, len8=True)
    y4 = M.spmv_xlds(xd, x_halo=halo, tile_rows=tile, y_permuted=True, two_rows=two_rows, len8=False)
    assert torch.equal(y8, y4)
    perm = M.host["perm"]
    ys = np.empty_like(host(y8))
    ys[perm] = host(y8)
    assert_rows(ys, A, x, 8 if M.dtype == torch.float64 else 4)


def test_xlds_one_byte_lengths_refused_for_long_rows():
    # 1000 rows, the first of 300 entries: the lengths no longer fit a byte
    lens = np.ones(1000, np.int64)
    lens[0] = 300
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.concatenate([np.arange(300), (np.arange(1, 1000) * 3) % 3000]).astype(np.int32)
    B = synth.CSR(1000, 3000, rp, col, synth.uniform_pm1(32, 1, int(rp[-1])))
    M = PjdsMatrix.from_csr(B, layout="block", sort_window=256)
    assert M.row_len8() is None
    xd = dev(synth.dense_x(3000, 32))
    with pytest.raises(ValueError):
        M.spmv_xlds(xd, len8=True)
    y = M.spmv_xlds(xd)              # falls back to the int32 lengths
    assert_rows(host(y), B, synth.dense_x(3000, 32))


def test_kernel_timing_hook_times_the_product_kernel():
    """pjds_time_next_launch: the armed call's product kernel records both events (a duration
    inside the events recorded around the calls), one launch takes the hook, the product is
    unchanged, and a hook disarmed before any launch records nothing."""
    A = synth.hh_like(1 << 16, seed=3)
    M = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=512)
    x = dev(synth.dense_x(A.n_cols, 1))
    y0 = M.spmv_xlds(x, x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True)
    torch.cuda.synchronize()
    k1, k2 = L.KernelTimer(), L.KernelTimer()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    k1.arm()
    y1 = M.spmv_xlds(x, x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True)
    y2 = M.spmv(x, y_permuted=True)         # launched after the hook was taken
    s1.record()
    k2.arm()
    k2.disarm()
    torch.cuda.synchronize()
    t = k1.ms()
    assert t is not None and 0 < t <= s0.elapsed_time(s1)
    assert k2.ms() is None
    assert torch.equal(y0, y1)
    assert_rows(host(y2), A, synth.dense_x(A.n_cols, 1), 8, rows=M.d["perm"].cpu().numpy())


def test_timing_hook_is_taken_by_every_one_kernel_entry_point():
    """Each one-kernel product entry point (and the probe) launches its main kernel with the
    armed events; a call refused on the host launches nothing and leaves the hook armed for
    the next launch."""
    A = synth.hh_like(1 << 15, seed=4)
    x = synth.dense_x(A.n_cols, 4)
    xd = dev(x)
    M = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=512)
    X = dev(synth.dense_x(A.n_cols, 4, k=4).reshape(A.n_cols, 4))
    E, C = EllrMatrix.from_csr(A), CsrMatrix.from_csr(A)
    buf = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    out = torch.empty(2048, dtype=torch.float64, device="cuda")
    y = torch.empty(A.n_rows, dtype=torch.float64, device="cuda")
    d = M.d
    calls = {
        "pjds_spmv": lambda: M.spmv(xd, y_permuted=True),
        "pjds_spmv_xlds": lambda: M.spmv_xlds(xd, x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True),
        "pjds_spmv_noalloc": lambda: L.pjds_spmv_noalloc(M.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"],
                                                         d["perm"], d["sched"] if M.info.n_chunks else None, xd, y, L.PJDS_Y_PERMUTED),
        "pjds_spmmv": lambda: M.spmmv(X, y_permuted=True),
        "pjds_spmmv_xlds": lambda: M.spmmv_xlds(X, x_halo=512, tile_rows=1024, y_permuted=True),
        "ellr_spmv": lambda: E.spmv(xd),
        "csr_spmv": lambda: C.spmv(xd, variant=4),
        "pjds_probe": lambda: L.pjds_probe(0, buf, out, 1 << 20),
    }
    timers = {}
    for name, fn in calls.items():
        t = L.KernelTimer()
        t.arm()
        fn()
        t.disarm()
        timers[name] = t
    torch.cuda.synchronize()
    for name, t in timers.items():
        ms = t.ms()
        assert ms is not None and ms > 0, name
    # a refused call takes nothing: the next launch records the events
    t = L.KernelTimer()
    t.arm()
    with pytest.raises(Exception):
        M.spmv(xd[: A.n_cols // 2])                 # x too short: refused before any launch
    M.spmv(xd, y_permuted=True)
    t.disarm()
    torch.cuda.synchronize()
    assert t.ms() is not None
    assert_rows(host(M.spmv(xd, y_permuted=True)), A, x, 8, rows=d["perm"].cpu().numpy())
