"""The allocation-free product (pjds_spmv_noalloc) against pjds_spmv, through the C interface.

Both run the same kernels in the same order, so their results must agree bit for bit; the
first is also checked against the oracle (relative L2 error and the per-row bound).  The
matrices have long rows cut into work items, so the fixed scratch array really holds partial
sums and completion counters.  Two calls in a row, the second on a smaller matrix, check that
a call does not depend on what the previous one left in the shared array.
"""
import numpy as np
import pytest

import synth
from tests import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _product_pair(A, x_np, dtype, **kw):
    from paper_1112_5588_amd import PjdsMatrix, _lib as L
    M = PjdsMatrix.from_csr(A.astype(dtype) if dtype != np.float64 else A, device="cuda", **kw)
    assert M.info.n_chunks > 0, "the case must use the long-row workspace"
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    x = torch.from_numpy(x_np).to("cuda", tdt)
    d = M.d
    y_ref = torch.full((M.n_rows,), float("nan"), dtype=tdt, device="cuda")
    L.pjds_spmv(M.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"], d["perm"], d["sched"], d["work"],
                x, y_ref, 0)
    y = torch.full((M.n_rows,), float("nan"), dtype=tdt, device="cuda")
    L.pjds_spmv_noalloc(M.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"], d["perm"], d["sched"],
                        x, y, 0)
    torch.cuda.synchronize()
    return M, y.cpu().numpy(), y_ref.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_equals_spmv_on_two_calls_second_smaller(dtype):
    cases = [
        # (rows, seed, conversion): long rows cut every 64 / 128 entries
        (200_003, 31, dict(layout="jd", split_len=64)),
        (40_961, 32, dict(layout="block", sort_window=4096, split_len=128)),
    ]
    for n, seed, kw in cases:
        print(f"noalloc case n={n} seed={seed} {kw} {np.dtype(dtype).name}", flush=True)
        A = synth.powerlaw(n, seed=seed)
        x_np = synth.dense_x(A.n_cols, seed)
        if dtype == np.float32:
            x_np = x_np.astype(np.float32).astype(np.float64)
            Ad = A.astype(np.float32)
        else:
            Ad = A
        M, y, y_ref = _product_pair(A, x_np, dtype, **kw)
        assert np.array_equal(y.view(np.uint8), y_ref.view(np.uint8)), "not bitwise equal to pjds_spmv"
        parity.assert_rows(y.astype(np.float64), Ad, x_np, value_bytes=np.dtype(dtype).itemsize)


def test_noalloc_plain_matrix_without_long_rows():
    """No work items: nothing of the scratch array is used, the product is pjds_spmv's."""
    from paper_1112_5588_amd import PjdsMatrix, _lib as L
    A = synth.laplacian_2d(64)
    x_np = synth.dense_x(A.n_cols, 5)
    M = PjdsMatrix.from_csr(A, device="cuda")
    assert M.info.n_chunks == 0
    x = torch.from_numpy(x_np).cuda()
    d = M.d
    y = torch.full((M.n_rows,), float("nan"), dtype=torch.float64, device="cuda")
    L.pjds_spmv_noalloc(M.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"], d["perm"], None, x, y, 0)
    torch.cuda.synchronize()
    parity.assert_rows(y.cpu().numpy(), A, x_np)
