"""GPU parity of the many-matrix batch (persistent kernel in a HIP graph, per-member graph,
direct launches) against the oracle, and against the single-matrix kernel bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth import torchgen
from paper_1112_5588_amd import PjdsBatch, PjdsMatrix
from paper_1112_5588_amd import _lib as L
from parity import assert_rows

pytestmark = pytest.mark.gpu

MODES = [L.PJDS_BATCH_PERSISTENT, L.PJDS_BATCH_GRAPH, L.PJDS_BATCH_DIRECT]


def small_batch(count=24, seed=31, dtype=np.float64, **kw):
    sizes = synth.uneven_batch_sizes(count, 50, 20000, seed=seed)
    sizes[3] = 1            # a one-row member
    mats, As, xs_np = [], [], []
    for m, n in enumerate(sizes):
        A = synth.banded_stratified(int(n), 1000 + m).astype(dtype)
        As.append(A)
        mats.append(PjdsMatrix.from_csr(A, split_len=-1, keep_host=True, **kw))
        x = synth.dense_x(A.n_cols, 1000 + m)
        if dtype == np.float32:
            x = x.astype(np.float32).astype(np.float64)
        xs_np.append(x)
    tdt = mats[0].dtype
    xs = [torch.from_numpy(x).to("cuda", tdt) for x in xs_np]
    return As, mats, xs, xs_np


def run_batch(mats, xs, mode, y_permuted=False, groups_per_tile=0, x_halo=None):
    ys = [torch.full((M.n_rows,), float("nan"), dtype=M.dtype, device="cuda") for M in mats]
    B = PjdsBatch(mats, xs, ys, mode=mode, y_permuted=y_permuted, groups_per_tile=groups_per_tile,
                  x_halo=x_halo)
    B.launch()
    torch.cuda.synchronize()
    return B, ys


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("y_permuted", [False, True])
def test_batch_matches_oracle(mode, y_permuted):
    As, mats, xs, xs_np = small_batch()
    B, ys = run_batch(mats, xs, mode, y_permuted)
    for A, M, y, x in zip(As, mats, ys, xs_np):
        assert_rows(y.cpu().numpy(), A, x, rows=M.host["perm"] if y_permuted else None)
    B.close()


@pytest.mark.parametrize("b_r,layout,gpt", [(32, "jd", 1), (64, "block", 3), (128, "jd", 16)])
def test_persistent_equals_single_kernel_bitwise(b_r, layout, gpt):
    As, mats, xs, _ = small_batch(count=17, seed=32, block_height=b_r, layout=layout)
    B, ys = run_batch(mats, xs, L.PJDS_BATCH_PERSISTENT, groups_per_tile=gpt)
    n_tiles, grid = B.info()
    assert n_tiles >= len(mats) and grid > 0
    for M, x, y in zip(mats, xs, ys):
        assert torch.equal(M.spmv(x), y)
    B.close()


def test_float32_batch():
    As, mats, xs, xs_np = small_batch(count=12, seed=33, dtype=np.float32)
    B, ys = run_batch(mats, xs, L.PJDS_BATCH_PERSISTENT)
    for A, y, x in zip(As, ys, xs_np):
        assert_rows(y.double().cpu().numpy(), A, x, 4)
    B.close()


@pytest.mark.parametrize("mode", [L.PJDS_BATCH_PERSISTENT, L.PJDS_BATCH_GRAPH])
def test_graph_replays_are_idempotent(mode):
    # replay the captured graph several times with eager work and synchronisation between
    # replays; every replay must reproduce the eager result
    As, mats, xs, _ = small_batch(count=10, seed=34)
    ys = [torch.empty(M.n_rows, dtype=M.dtype, device="cuda") for M in mats]
    B = PjdsBatch(mats, xs, ys, mode=mode)
    ref = [M.spmv(x) for M, x in zip(mats, xs)]
    for rep in range(4):
        for y in ys:
            y.fill_(float(rep) - 7.0)
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for r, y in zip(ref, ys):
            assert torch.equal(r, y), rep
    B.close()


@pytest.mark.parametrize("b_r,window,yp", [(64, 256, False), (64, 256, True), (32, 128, True), (128, 512, False)])
def test_two_rows_per_lane_batch_bitwise(b_r, window, yp):
    # members sorted in windows of whole 128-row groups and an even tile size: the persistent
    # kernel takes two rows per lane; it must still equal the single-matrix kernel bit for bit
    sizes = [600, 1000, 4097, 20000, 513, 777]      # every member longer than its window
    mats, xs, As = [], [], []
    for m, n in enumerate(sizes):
        A = synth.banded_stratified(n, 2000 + m)
        As.append(A)
        mats.append(PjdsMatrix.from_csr(A, block_height=b_r, layout="block", sort_window=window, split_len=-1,
                                        keep_host=True))
        xs.append(torch.from_numpy(synth.dense_x(n, 2000 + m)).cuda())
    B, ys = run_batch(mats, xs, L.PJDS_BATCH_PERSISTENT, y_permuted=yp, groups_per_tile=4)
    for A, M, x, y in zip(As, mats, xs, ys):
        assert torch.equal(M.spmv(x, y_permuted=yp), y)
        assert_rows(y.cpu().numpy(), A, x.cpu().numpy(), rows=M.host["perm"] if yp else None)
    B.close()


@pytest.mark.parametrize("window", [0, 256])
def test_full_size_uneven_batch_sampled(window):
    # 512 members, rows log-uniform in [1e3, 5e5], 3..60 entries per row: generated on the
    # GPU by the torch twin of the generator, converted on the host, one persistent launch;
    # global sort (one row per lane) and windows of 256 (two rows per lane), as the benchmark
    sizes = synth.uneven_batch_sizes(512)
    mats, xs = [], []
    kw = dict(layout="block", sort_window=window) if window else {}
    for m, n in enumerate(sizes):
        rp, col, val = torchgen.banded_stratified(int(n), 1000 + m, device="cuda")
        mats.append(PjdsMatrix.from_arrays(int(n), int(n), rp, col, val, split_len=-1, **kw))
        xs.append(torchgen.dense_x(int(n), 1000 + m, device="cuda"))
        del rp, col, val
    total_nnz = sum(M.info.nnz for M in mats)
    assert total_nnz > 1_000_000_000
    B, ys = run_batch(mats, xs, L.PJDS_BATCH_PERSISTENT)
    # the same members with x staged in LDS (halo 4096, the generator's band): bit for bit
    Bs, ys_s = run_batch(mats, xs, L.PJDS_BATCH_PERSISTENT, x_halo=4096)
    for y, y_s in zip(ys, ys_s):
        assert torch.equal(y, y_s)
    Bs.close()
    del ys_s
    # sampled members checked in full against the oracle (numpy generator: same bits)
    for m in (0, 1, int(np.argmax(sizes)), int(np.argmin(sizes)), 255, 511):
        A = synth.banded_stratified(int(sizes[m]), 1000 + m)
        assert_rows(ys[m].cpu().numpy(), A, synth.dense_x(A.n_cols, 1000 + m))
    # every member: the batch equals the single-matrix kernel bit for bit
    for M, x, y in zip(mats, xs, ys):
        assert torch.equal(M.spmv(x), y)
    B.close()


# ------------------------------------------------------------------ x staged in LDS

def windowed_members(sizes, window, seed, dtype=np.float64, b_r=64):
    # members shorter than the window are sorted globally, as the benchmark builds them
    mats, xs, As = [], [], []
    for m, n in enumerate(sizes):
        A = synth.banded_stratified(int(n), seed + m).astype(dtype)
        As.append(A)
        kw = dict(sort_window=window) if 0 < window < n else {}
        mats.append(PjdsMatrix.from_csr(A, block_height=b_r, layout="block", split_len=-1, keep_host=True, **kw))
        x = synth.dense_x(A.n_cols, seed + m)
        if dtype == np.float32:
            x = x.astype(np.float32).astype(np.float64)
        xs.append(torch.from_numpy(x).to("cuda", mats[-1].dtype))
    return As, mats, xs


@pytest.mark.parametrize("window,halo,gpt,yp", [(256, 4096, 16, True), (256, 0, 16, False), (256, 700, 4, True),
                                                (192, 1000, 3, True), (128, 300, 2, False), (0, 4096, 16, True),
                                                (512, 100000, 64, False)])
def test_xlds_batch_equals_single_kernel_bitwise(window, halo, gpt, yp):
    # windows of 256 and 512 with even tiles (two rows per lane), 192 (one row: not whole
    # 128-row groups) and 128 with members shorter than the window (globally sorted, so one
    # row), a global sort throughout (each member staged whole, up to the cap), no halo, and
    # a halo far beyond the 78 KiB cap (the rest read from global memory); members from 1 to
    # 20000 rows, ragged last tiles
    sizes = [20000, 1, 4097, 600, 63, 1000, 777, 9000, 513, 130]
    if window in (256, 512):
        sizes = [n for n in sizes if n > window]          # every member windowed: pairs on
    As, mats, xs = windowed_members(sizes, window, 3000)
    B, ys = run_batch(mats, xs, L.PJDS_BATCH_PERSISTENT, y_permuted=yp, groups_per_tile=gpt, x_halo=halo)
    n_tiles, grid = B.info()
    assert n_tiles >= len(mats) and grid > 0
    for A, M, x, y in zip(As, mats, xs, ys):
        assert torch.equal(M.spmv(x, y_permuted=yp), y)
        assert_rows(y.cpu().numpy(), A, x.cpu().numpy(), rows=M.host["perm"] if yp else None)
    B.close()


@pytest.mark.parametrize("b_r", [32, 128])
def test_xlds_batch_block_heights_and_float32(b_r):
    As, mats, xs = windowed_members([5000, 300, 12000, 64], 256, 3100, dtype=np.float32, b_r=b_r)
    B, ys = run_batch(mats, xs, L.PJDS_BATCH_PERSISTENT, groups_per_tile=8, x_halo=4096)
    for A, M, x, y in zip(As, mats, xs, ys):
        assert torch.equal(M.spmv(x), y)
        assert_rows(y.double().cpu().numpy(), A, x.double().cpu().numpy(), 4)
    B.close()


def test_xlds_batch_graph_replays_are_idempotent():
    As, mats, xs = windowed_members([3000, 800, 7000, 256, 1500], 256, 3200)
    ys = [torch.empty(M.n_rows, dtype=M.dtype, device="cuda") for M in mats]
    B = PjdsBatch(mats, xs, ys, y_permuted=True, x_halo=2048)
    ref = [M.spmv(x, y_permuted=True) for M, x in zip(mats, xs)]
    for rep in range(4):
        for y in ys:
            y.fill_(float(rep) + 0.5)
        torch.cuda.synchronize()
        B.launch()
        torch.cuda.synchronize()
        for r, y in zip(ref, ys):
            assert torch.equal(r, y), rep
    B.close()


def test_xlds_batch_needs_the_persistent_mode():
    As, mats, xs = windowed_members([1000], 256, 3300)
    ys = [torch.empty(1000, dtype=torch.float64, device="cuda")]
    with pytest.raises(ValueError):
        PjdsBatch(mats, xs, ys, mode=L.PJDS_BATCH_GRAPH, x_halo=512)
