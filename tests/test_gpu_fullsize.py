"""Full-size parity of every product form the benchmark times, on the benchmark's own matrices
and launch configurations: the Holstein-Hubbard-like matrix (N = 2^22) and the power-law
matrix (N = 2^23, rows up to 4096).  Whole result vectors against the oracle, row by row
(each row within its own rounding bound) and by relative L2 error, plus bitwise equalities
between forms that add the same terms in the same order."""
import numpy as np
import pytest
import torch

import synth
from paper_1112_5588_amd import CsrMatrix, EllrMatrix, PjdsMatrix
from paper_1112_5588_amd.matrix import split_columns
from parity import RowReference

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def original_order(y, perm):
    """A result in the permuted basis (slot i = original row perm[i]) in original row order."""
    torch.cuda.synchronize()
    out = torch.empty_like(y)
    out[perm.long()] = y
    return out.double().cpu().numpy()


def host(y):
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


@pytest.fixture(scope="module")
def hh():
    A = synth.hh_like(1 << 22, seed=2)
    x = synth.dense_x(A.n_cols, 1)
    print(f"[fullsize] HH-like N={A.n_rows} nnz={A.nnz}", flush=True)
    return A, x, RowReference(A, x)


@pytest.fixture(scope="module")
def pl():
    P = synth.powerlaw(1 << 23, seed=3)
    x = synth.dense_x(P.n_cols, 3)
    print(f"[fullsize] power law N={P.n_rows} nnz={P.nnz}", flush=True)
    return P, x, RowReference(P, x)


def test_hh_comparison_formats(hh):
    # ELLPACK-R (Listing 1) and the CSR kernels with 1, 4 and 16 lanes per row
    A, x, R = hh
    xd = dev(x)
    E = EllrMatrix.from_csr(A)
    R.check(host(E.spmv(xd)))
    del E
    C = CsrMatrix.from_csr(A)
    for v in (1, 4, 16):
        y = C.spmv(xd, variant=v)
        R.check(host(y))
        assert torch.equal(y, C.spmv(xd, variant=v))          # reproducible


def test_hh_plain_product_forms(hh):
    # the headline storage through the plain kernel: y scattered back, y permuted with the XCD
    # renumbering, and the paper's plain form (global sort, jagged-diagonal layout)
    A, x, R = hh
    xd = dev(x)
    M = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=256)
    R.check(host(M.spmv(xd, y_permuted=False)))
    yp = M.spmv(xd, y_permuted=True, xcd_remap=True)
    R.check(original_order(yp, M.d["perm"]))
    # the same terms in the same order as the headline LDS product: bit for bit
    assert torch.equal(yp, M.spmv_xlds(xd, x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True))
    del M
    J = PjdsMatrix.from_csr(A, block_height=64)
    R.check(host(J.spmv(xd)))


@pytest.mark.parametrize("lanes,window", [(2, 256), (4, 256), (8, 256), (1, 64), (4, 64)])
def test_hh_lanes_and_sliced_forms(hh, lanes, window):
    A, x, R = hh
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=window, lanes=lanes)
    R.check(original_order(M.spmv(dev(x), y_permuted=True), M.d["perm"]))


def test_hh_fp32_headline(hh):
    A, x, _ = hh
    A32 = A.astype(np.float32)
    x32 = x.astype(np.float32)
    R32 = RowReference(A32, x32.astype(np.float64))
    M = PjdsMatrix.from_csr(A32, layout="block", sort_window=256)
    y = M.spmv_xlds(dev(x32, torch.float32), x_halo=768, tile_rows=1024, y_permuted=True, two_rows=True)
    R32.check(original_order(y, M.d["perm"]), value_bytes=4)


@pytest.mark.parametrize("k,window,remap", [(16, 4096, True), (32, 4096, True), (16, 256, False)])
def test_hh_spmmv_wide(hh, k, window, remap):
    # k = 16 and 32: the unstaged SpMMV with XCD renumbering on windows of 4096, as the bench
    # times it; sampled rows against the oracle, every vector
    A, _, _ = hh
    X_np = synth.dense_x(A.n_cols, 4, k=k).reshape(A.n_cols, k)
    M = PjdsMatrix.from_csr(A, layout="block", sort_window=window)
    Y = M.spmmv(dev(X_np), vectors_per_tile=min(k, 16), vectors_per_lane=4, y_permuted=True, xcd_remap=remap)
    Yo = original_order(Y, M.d["perm"])
    rows = np.unique(np.concatenate([np.arange(256), (synth.uniform01(85, 1, 2048) * A.n_rows).astype(np.int64)]))
    from parity import assert_rows_mm
    assert_rows_mm(Yo[rows], A, X_np, rows=rows)


def test_hh_split_local_nonlocal(hh):
    A, x, R = hh
    loc, nl = split_columns(A, 0, A.n_cols // 2)
    ML, MN = PjdsMatrix.from_csr(loc), PjdsMatrix.from_csr(nl)
    xd = dev(x)
    y = ML.spmv(xd)
    MN.spmv_axpby(xd, y, alpha=1.0, beta=1.0, z=y)
    R.check(host(y), extra_terms=1)


def test_powerlaw_global_split_and_windows(pl):
    # global sort with long rows split every 512 entries, windows 2^10 and 2^16 and 64-row
    # slices with the same split: every row split the same way, so the same bits; the unsplit
    # product equal to it on every row of at most 512 entries
    P, x, R = pl
    xd = dev(x)
    M = PjdsMatrix.from_csr(P, layout="block", split_len=512)
    assert M.info.n_chunks > 0 and M.info.max_row_len == 4096
    y_split = original_order(M.spmv(xd, y_permuted=True), M.d["perm"])
    R.check(y_split)
    del M
    for window in (1 << 10, 1 << 16, 64):
        W = PjdsMatrix.from_csr(P, layout="block", sort_window=window, split_len=512)
        yw = original_order(W.spmv(xd, y_permuted=True), W.d["perm"])
        assert np.array_equal(yw.view(np.uint64), y_split.view(np.uint64)), window
        del W
    U = PjdsMatrix.from_csr(P, layout="block", split_len=-1)
    y_un = original_order(U.spmv(xd, y_permuted=True), U.d["perm"])
    R.check(y_un)
    short = np.diff(P.row_ptr) <= 512
    assert np.array_equal(y_un[short].view(np.uint64), y_split[short].view(np.uint64))


def test_powerlaw_lanes(pl):
    # four lanes per row: global sort and 64-row slices (sliced ELLR-T's padding) add the same
    # four partial sums in the same butterfly: the same bits
    P, x, R = pl
    xd = dev(x)
    G = PjdsMatrix.from_csr(P, layout="block", lanes=4)
    yg = original_order(G.spmv(xd, y_permuted=True), G.d["perm"])
    R.check(yg)
    del G
    S = PjdsMatrix.from_csr(P, layout="block", sort_window=64, lanes=4)
    ys = original_order(S.spmv(xd, y_permuted=True), S.d["perm"])
    assert np.array_equal(ys.view(np.uint64), yg.view(np.uint64))
