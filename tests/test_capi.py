"""The C interface as a library: it loads without a GPU, exports every function the header
declares, and rejects bad input with a status code and a message, writing nothing."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from paper_1112_5588_amd import _lib as L

HEADER_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "pjds_spmv" in names and "pjds_convert" in names and "ellr_spmv" in names and "csr_spmv" in names
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows every one of them
    assert not set(names) - set(L.EXPORTED)


def test_version_and_error_string():
    assert "gfx950" in L.pjds_version()
    with pytest.raises(L.PjdsError):
        L.pjds_plan(4, 4, np.array([0, 1, 2, 3, 4], np.int64), block_height=48)
    assert "block_height" in L.pjds_last_error()


def rp(*v):
    return np.array(v, dtype=np.int64)


@pytest.mark.parametrize("args,code", [
    ((3, 3, rp(1, 1, 2, 3)), L.PJDS_ERR_INDEX),           # row_ptr[0] != 0
    ((3, 3, rp(0, 2, 1, 3)), L.PJDS_ERR_INDEX),           # decreasing
    ((-1, 3, rp(0)), L.PJDS_ERR_ARG),                      # negative size
    ((1 << 31, 3, rp(0)), L.PJDS_ERR_OVERFLOW),            # rows beyond int32
])
def test_plan_rejects_bad_row_ptr(args, code):
    with pytest.raises(L.PjdsError) as e:
        L.pjds_plan(*args)
    assert e.value.code == code


@pytest.mark.parametrize("kw,code", [
    (dict(block_height=16), L.PJDS_ERR_ARG),
    (dict(block_height=96), L.PJDS_ERR_ARG),
    (dict(sort_window=100, flags=L.PJDS_LAYOUT_BLOCK), L.PJDS_ERR_ARG),   # not a multiple of 64
    (dict(sort_window=128, flags=L.PJDS_LAYOUT_JD), L.PJDS_ERR_ARG),      # JD needs a global sort
    (dict(flags=0x40), L.PJDS_ERR_ARG),
    (dict(split_len=12), L.PJDS_ERR_ARG),
    (dict(block_height=32, flags=L.PJDS_LANES(1)), L.PJDS_ERR_ARG),                       # lanes need blocks
    (dict(block_height=64, flags=L.PJDS_LAYOUT_BLOCK | L.PJDS_LANES(1)), L.PJDS_ERR_ARG),  # b_r must be 32
    (dict(block_height=1, flags=L.PJDS_LAYOUT_BLOCK | L.PJDS_LANES(7)), L.PJDS_ERR_ARG),   # T = 128 > 64
])
def test_plan_rejects_bad_options(kw, code):
    A = synth.random_csr(1000, 50, 1)
    with pytest.raises(L.PjdsError) as e:
        L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, **kw)
    assert e.value.code == code


def test_symmetric_needs_square():
    A = synth.random_csr(100, 50, 1)
    with pytest.raises(L.PjdsError) as e:
        L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, flags=L.PJDS_SYMMETRIC)
    assert e.value.code == L.PJDS_ERR_ARG


def test_convert_rejects_column_out_of_range_without_writing():
    A = synth.random_csr(200, 40, 3, max_len=10, empty_frac=0.0)
    info = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr)
    bad = A.col.copy()
    bad[len(bad) // 2] = 40
    outs = [np.full(info.n_rows, -9, np.int32), np.full(info.n_pad, -9, np.int32),
            np.full(info.n_offsets, -9, np.int64), np.full(info.nnz_stored, -9, np.int32),
            np.full(info.nnz_stored, -9.0)]
    with pytest.raises(L.PjdsError) as e:
        L.pjds_convert(info, A.row_ptr, bad, A.val, *outs)
    assert e.value.code == L.PJDS_ERR_INDEX
    assert "column index 40" in L.pjds_last_error()
    for o in outs:
        assert np.all(o == -9)
    bad[len(bad) // 2] = -1
    with pytest.raises(L.PjdsError):
        L.pjds_convert(info, A.row_ptr, bad, A.val, *outs)


def test_convert_rejects_mismatched_info():
    A = synth.random_csr(200, 40, 3)
    B = synth.random_csr(200, 40, 4)
    info = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr)
    outs = [np.empty(info.n_rows, np.int32), np.empty(info.n_pad, np.int32),
            np.empty(info.n_offsets, np.int64), np.empty(max(info.nnz_stored, 1), np.int32),
            np.empty(max(info.nnz_stored, 1))]
    # the binding refuses B's shorter arrays itself; the C library, called directly, refuses
    # the plan of another matrix
    with pytest.raises(ValueError):
        L.pjds_convert(info, B.row_ptr, B.col, B.val, *outs)
    big = [np.resize(o, 4 * o.size + 64) for o in outs]
    rc = L.lib().pjds_convert(ctypes.byref(info), B.row_ptr.ctypes.data, B.col.ctypes.data, B.val.ctypes.data,
                              L.PJDS_F64, *[o.ctypes.data for o in big], None)
    assert rc == L.PJDS_ERR_ARG


def test_convert_requires_schedule_for_long_rows():
    A = synth.powerlaw(1 << 12, seed=3, l_max=1024)
    info = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, split_len=64)
    assert info.n_chunks > 0
    outs = [np.empty(info.n_rows, np.int32), np.empty(info.n_pad, np.int32),
            np.empty(info.n_offsets, np.int64), np.empty(info.nnz_stored, np.int32),
            np.empty(info.nnz_stored)]
    # the binding asks for the schedule itself; the C library, called directly, refuses too
    with pytest.raises(ValueError):
        L.pjds_convert(info, A.row_ptr, A.col, A.val, *outs, None)
    rc = L.lib().pjds_convert(ctypes.byref(info), A.row_ptr.ctypes.data, A.col.ctypes.data, A.val.ctypes.data,
                              L.PJDS_F64, *[o.ctypes.data for o in outs], None)
    assert rc == L.PJDS_ERR_ARG and "sched" in L.pjds_last_error()


def test_ellr_plan_reports_size_of_skewed_matrix():
    # The power-law matrix (N = 2^23, longest row 4096) would need n_pad * 4096 entries in
    # ELLPACK-R: the planner reports it so the caller can refuse to allocate.
    n = 1 << 23
    lens = np.full(n, 12, np.int64)
    lens[5] = 4096
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    info = L.ellr_plan(n, n, row_ptr)
    assert info.nnz_stored == n * 4096
    assert info.nnz_stored * 12 > 288 * 2 ** 30        # over an MI355X's HBM in FP64


def test_device_entry_points_validate_before_touching_the_gpu():
    A = synth.random_csr(100, 100, 1)
    info = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr)
    lib = L.lib()
    # NULL arrays / bad dtype / bad flags are refused on the host
    assert lib.pjds_spmv(ctypes.byref(info), None, None, None, None, None, None, None, 0, None, None, 0, None) == L.PJDS_ERR_ARG
    assert lib.pjds_spmv(ctypes.byref(info), None, None, None, None, None, None, None, 7, None, None, 0, None) == L.PJDS_ERR_ARG
    assert lib.pjds_spmv(ctypes.byref(info), None, None, None, None, None, None, None, 0, None, None, 0x100, None) == L.PJDS_ERR_ARG
    assert lib.pjds_spmmv(ctypes.byref(info), None, None, None, None, None, 0, 4, 3, 1, None, None, 0, None) == L.PJDS_ERR_ARG
    assert lib.pjds_spmmv(ctypes.byref(info), None, None, None, None, None, 0, 6, 8, 4, None, None, 0, None) == L.PJDS_ERR_ARG
    assert lib.csr_spmv(10, 10, None, None, None, 0, None, None, 5, None) == L.PJDS_ERR_ARG
    assert lib.pjds_probe(3, None, None, 10, None) == L.PJDS_ERR_ARG


def test_noalloc_product_refuses_plans_beyond_its_fixed_scratch():
    """pjds_spmv_noalloc takes the long-row workspace from a fixed 16 MiB array: a plan that
    needs more is refused with an overflow status before anything reaches the GPU (only the
    row pointers are needed to plan)."""
    n, length = 1 << 18, 256
    row_ptr = np.arange(n + 1, dtype=np.int64) * length
    info = L.pjds_plan(n, n, row_ptr, 64, 0, L.PJDS_LAYOUT_JD, 8)
    need = L.pjds_workspace_size(info, np.float64)
    assert need > L.PJDS_NOALLOC_SCRATCH_BYTES
    lib = L.lib()
    rc = lib.pjds_spmv_noalloc(ctypes.byref(info), None, None, None, None, None, None, 0, None, None, 0, None)
    assert rc == L.PJDS_ERR_OVERFLOW
    assert "scratch" in L.pjds_last_error()
    # a plan within the limit passes the size check and fails on the NULL arrays instead
    small = L.pjds_plan(4096, 4096, np.arange(4097, dtype=np.int64) * length, 64, 0, L.PJDS_LAYOUT_JD, 64)
    assert 0 < L.pjds_workspace_size(small, np.float64) <= L.PJDS_NOALLOC_SCRATCH_BYTES
    assert lib.pjds_spmv_noalloc(ctypes.byref(small), None, None, None, None, None, None, 0, None, None, 0,
                                 None) == L.PJDS_ERR_ARG
    assert lib.pjds_spmv_noalloc(ctypes.byref(small), None, None, None, None, None, None, 0, None, None, 0x100,
                                 None) == L.PJDS_ERR_ARG


def test_lanes_matrix_is_refused_by_the_products_that_do_not_take_it():
    A = synth.random_csr(500, 500, 3, max_len=30)
    info = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, 16, 128, L.PJDS_LAYOUT_BLOCK | L.PJDS_LANES(2), 0)
    assert info.block_height == 16 and info.n_chunks == 0 and info.split_len == 0
    lib = L.lib()
    assert lib.pjds_spmmv(ctypes.byref(info), None, None, None, None, None, 0, 4, 4, 1, None, None, 0, None) == L.PJDS_ERR_UNSUPPORTED
    assert lib.pjds_spmv_xlds(ctypes.byref(info), None, None, None, None, None, 0, None, None, 512, 512, 0, None) == L.PJDS_ERR_UNSUPPORTED
    assert lib.pjds_spmmv_xlds(ctypes.byref(info), None, None, None, None, None, 0, 4, 4, 4, None, None, 512, 512, 0, None) == L.PJDS_ERR_UNSUPPORTED
    m = L.pjds_batch_member(info=ctypes.pointer(info))
    out = ctypes.c_void_p()
    assert lib.pjds_batch_create(1, ctypes.byref(m), 0, L.PJDS_Y_PERMUTED, 0, 8, ctypes.byref(out)) == L.PJDS_ERR_UNSUPPORTED
    assert lib.pjds_batch_create_xlds(1, ctypes.byref(m), 0, L.PJDS_Y_PERMUTED, 16, 512, ctypes.byref(out)) == L.PJDS_ERR_UNSUPPORTED
    # the product itself takes it (and checks its arrays first)
    assert lib.pjds_spmv(ctypes.byref(info), None, None, None, None, None, None, None, 0, None, None, 0, None) == L.PJDS_ERR_ARG


def test_batch_create_validates_on_the_host():
    A = synth.random_csr(100, 100, 1)
    i64 = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, block_height=64)
    i32 = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, block_height=32)
    lib = L.lib()
    h = ctypes.c_void_p()
    arr = (L.pjds_batch_member * 2)()
    arr[0] = L.pjds_batch_member(ctypes.pointer(i64), None, None, None, None, None, None, None)
    arr[1] = L.pjds_batch_member(ctypes.pointer(i32), None, None, None, None, None, None, None)
    assert lib.pjds_batch_create(2, arr, 0, 0, 0, 0, ctypes.byref(h)) == L.PJDS_ERR_ARG
    assert lib.pjds_batch_create(0, arr, 0, 0, 0, 0, ctypes.byref(h)) == L.PJDS_ERR_ARG
    assert lib.pjds_batch_create(1, arr, 0, 0, 9, 0, ctypes.byref(h)) == L.PJDS_ERR_ARG
    assert lib.pjds_batch_create(1, arr, 0, 0x40, 0, 0, ctypes.byref(h)) == L.PJDS_ERR_ARG
    assert h.value is None
    # the LDS-staged form: the same member checks, and a halo that is not negative
    assert lib.pjds_batch_create_xlds(1, arr, 0, 0, 16, -1, ctypes.byref(h)) == L.PJDS_ERR_ARG
    assert "x_halo" in L.pjds_last_error()
    assert lib.pjds_batch_create_xlds(2, arr, 0, 0, 16, 512, ctypes.byref(h)) == L.PJDS_ERR_ARG
    assert lib.pjds_batch_create_xlds(1, arr, 0, 0x40, 16, 512, ctypes.byref(h)) == L.PJDS_ERR_ARG
    assert lib.pjds_batch_create_xlds(1, arr, 7, 0, 16, 512, None) == L.PJDS_ERR_ARG
    assert h.value is None


def test_spmmv_xlds_validates_on_the_host():
    A = synth.random_csr(3000, 3000, 5, max_len=20)
    lib = L.lib()
    win = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, 64, 256, L.PJDS_LAYOUT_BLOCK, 0)
    glob = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, 64, 0, L.PJDS_LAYOUT_BLOCK, 0)
    jd = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, 64, 0, 0, 0)

    def call(info, k=4, t=4, vpl=4, halo=512, tile=1024, flags=0):
        return lib.pjds_spmmv_xlds(ctypes.byref(info), None, None, None, None, None, 0, k, t, vpl, None, None,
                                   halo, tile, flags, None)
    assert call(glob) == L.PJDS_ERR_ARG and "sort window" in L.pjds_last_error()
    assert call(jd) == L.PJDS_ERR_ARG
    assert call(win, vpl=3) == L.PJDS_ERR_ARG
    assert call(win, k=6, t=8, vpl=4) == L.PJDS_ERR_ARG          # k not a multiple of the lane width
    assert call(win, k=32, t=32, vpl=4) == L.PJDS_ERR_ARG        # eight lanes per row
    assert call(win, halo=-1) == L.PJDS_ERR_ARG
    assert call(win, tile=100) == L.PJDS_ERR_ARG
    assert call(win, flags=L.PJDS_XCD_REMAP) == L.PJDS_ERR_ARG
    assert call(win, k=0) == L.PJDS_ERR_ARG
    # valid arguments reach the device-array check
    assert call(win) == L.PJDS_ERR_ARG and "NULL" in L.pjds_last_error()


def test_timing_hook_is_armed_and_disarmed_on_the_host():
    """pjds_time_next_launch takes both events or neither; it only stores them (no GPU call)."""
    lib = L.lib()
    assert lib.pjds_time_next_launch(ctypes.c_void_p(0x1000), None) == L.PJDS_ERR_ARG
    assert lib.pjds_time_next_launch(None, ctypes.c_void_p(0x1000)) == L.PJDS_ERR_ARG
    assert "both events" in L.pjds_last_error()
    assert lib.pjds_time_next_launch(None, None) == L.PJDS_OK


def test_lanczos_flags_are_checked_on_the_host():
    """pjds_lanczos takes PJDS_ROW_LEN8 only with the staged product, and no other flag; both
    refusals come before any device array is looked at."""
    A = synth.laplacian_2d(32)
    info = L.pjds_plan(A.n_rows, A.n_cols, A.row_ptr, 64, 256, L.PJDS_LAYOUT_BLOCK | L.PJDS_SYMMETRIC)
    lib = L.lib()
    args = (None, None, None, None, None, None, None, 3)
    assert lib.pjds_lanczos(ctypes.byref(info), *args, -1, 0, L.PJDS_ROW_LEN8, None, None, None, None,
                            None) == L.PJDS_ERR_ARG
    assert "x_halo" in L.pjds_last_error()
    assert lib.pjds_lanczos(ctypes.byref(info), *args, 256, 256, 0x100, None, None, None, None,
                            None) == L.PJDS_ERR_ARG
    assert "flags" in L.pjds_last_error()
    # accepted flags get as far as the NULL arrays
    assert lib.pjds_lanczos(ctypes.byref(info), *args, 256, 256, L.PJDS_ROW_LEN8, None, None, None, None,
                            None) == L.PJDS_ERR_ARG
    assert "NULL" in L.pjds_last_error()
