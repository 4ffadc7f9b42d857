"""The Python binding refuses operands that do not fit the matrix before any pointer reaches a
kernel, and the C library refuses an inconsistent plan before it writes a host buffer.  Runs
on the CPU: device arrays are stand-ins that carry a device type, a dtype and a size, and the
refusal comes before any GPU call."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_1112_5588_amd import _lib as L


class FakeDev:
    """Duck-typed stand-in for a torch tensor on the GPU (never dereferenced)."""

    def __init__(self, n, dtype, device="cuda:0", shape=None):
        self.n, self.dtype, self.device = n, dtype, torch.device(device)
        self.is_cuda = True
        self.shape = shape or (n,)

    def numel(self):
        return self.n

    def element_size(self):
        return torch.empty(0, dtype=self.dtype).element_size()


def planned(A, **kw):
    return L.pjds_plan(A.n_rows, A.n_cols, np.ascontiguousarray(A.row_ptr, np.int64), 64,
                       kw.get("sort_window", 0), kw.get("flags", 0), kw.get("split_len", 0))


def operands(info, dtype=torch.float64, x=None, y=None, val=None):
    return dict(d_row_len=FakeDev(info.n_pad, torch.int32), d_offsets=FakeDev(info.n_offsets, torch.int64),
                d_col_p=FakeDev(info.nnz_stored, torch.int32),
                d_val_p=val if val is not None else FakeDev(info.nnz_stored, dtype),
                d_perm=FakeDev(info.n_rows, torch.int32),
                d_x=x if x is not None else FakeDev(info.n_cols, dtype),
                d_y=y if y is not None else FakeDev(info.n_rows, dtype))


A = synth.random_csr(1000, 700, 3, max_len=12)
INFO = planned(A)


@pytest.mark.parametrize("bad,exc", [
    (dict(x=FakeDev(700, torch.float32)), TypeError),              # x float32, matrix float64
    (dict(y=FakeDev(1000, torch.float32)), TypeError),             # y float32: val_p would be read as float
    (dict(x=FakeDev(699, torch.float64)), ValueError),             # x too short: read past its end
    (dict(y=FakeDev(999, torch.float64)), ValueError),             # y too short: written past its end
    (dict(x=FakeDev(700, torch.float64, device="cuda:1")), ValueError),
    (dict(val=FakeDev(10, torch.float64)), ValueError),
])
def test_product_operands_are_checked(bad, exc):
    ops = operands(INFO, **bad)
    with pytest.raises(exc):
        L.pjds_spmv(INFO, ops["d_row_len"], ops["d_offsets"], ops["d_col_p"], ops["d_val_p"], ops["d_perm"],
                    None, None, ops["d_x"], ops["d_y"])
    with pytest.raises(exc):
        L.pjds_spmv_xlds(INFO, ops["d_row_len"], ops["d_offsets"], ops["d_col_p"], ops["d_val_p"], ops["d_perm"],
                         ops["d_x"], ops["d_y"], 256)


def test_host_tensor_is_refused():
    ops = operands(INFO)
    with pytest.raises(ValueError):
        L.pjds_spmv(INFO, ops["d_row_len"], ops["d_offsets"], ops["d_col_p"], ops["d_val_p"], ops["d_perm"],
                    None, None, torch.zeros(700, dtype=torch.float64), ops["d_y"])


def test_spmmv_needs_k_columns():
    ops = operands(INFO)
    X = FakeDev(700 * 3, torch.float64)
    Y = FakeDev(1000 * 4, torch.float64)
    with pytest.raises(ValueError):                  # X holds 3 columns, k = 4
        L.pjds_spmmv(INFO, ops["d_row_len"], ops["d_offsets"], ops["d_col_p"], ops["d_val_p"], ops["d_perm"],
                     4, 4, X, Y)


def test_axpby_z_and_scatter_perm():
    ops = operands(INFO)
    with pytest.raises(ValueError):
        L.pjds_spmv_axpby(INFO, ops["d_row_len"], ops["d_offsets"], ops["d_col_p"], ops["d_val_p"], ops["d_perm"],
                          None, None, ops["d_x"], 1.0, 1.0, FakeDev(10, torch.float64), ops["d_y"])
    with pytest.raises(ValueError):                  # scattering y needs perm
        L.pjds_spmv(INFO, ops["d_row_len"], ops["d_offsets"], ops["d_col_p"], ops["d_val_p"], None,
                    None, None, ops["d_x"], ops["d_y"])


def test_ellr_and_csr_operands():
    E = L.ellr_plan(A.n_rows, A.n_cols, np.ascontiguousarray(A.row_ptr, np.int64))
    with pytest.raises(TypeError):
        L.ellr_spmv(E, FakeDev(E.n_pad, torch.int32), FakeDev(E.nnz_stored, torch.int32),
                    FakeDev(E.nnz_stored, torch.float64), FakeDev(700, torch.float32), FakeDev(1000, torch.float64))
    with pytest.raises(ValueError):
        L.csr_spmv(1000, 700, FakeDev(1001, torch.int64), FakeDev(A.nnz, torch.int32),
                   FakeDev(A.nnz - 1, torch.float64), FakeDev(700, torch.float64), FakeDev(1000, torch.float64),
                   nnz=A.nnz)


def test_convert_checks_host_buffers():
    rp = np.ascontiguousarray(A.row_ptr, np.int64)
    col = np.ascontiguousarray(A.col, np.int32)
    val = np.ascontiguousarray(A.val)
    i = INFO

    def bufs(**over):
        b = dict(perm=np.empty(i.n_rows, np.int32), row_len=np.empty(i.n_pad, np.int32),
                 offsets=np.empty(i.n_offsets, np.int64), col_p=np.empty(i.nnz_stored, np.int32),
                 val_p=np.empty(i.nnz_stored, np.float64))
        b.update(over)
        return b
    L.pjds_convert(i, rp, col, val, **bufs())
    with pytest.raises(TypeError):                   # float32 values buffer for float64 values
        L.pjds_convert(i, rp, col, val, **bufs(val_p=np.empty(i.nnz_stored, np.float32)))
    with pytest.raises(ValueError):
        L.pjds_convert(i, rp, col, val, **bufs(col_p=np.empty(i.nnz_stored - 1, np.int32)))
    with pytest.raises(ValueError):
        L.pjds_convert(i, rp, col, val, **bufs(row_len=np.empty(i.n_rows - 1, np.int32)))


def _raw_convert(info, rp, col, val, b):
    lib = L.lib()
    return lib.pjds_convert(ctypes.byref(info), rp.ctypes.data, col.ctypes.data, val.ctypes.data, L.PJDS_F64,
                            b["perm"].ctypes.data, b["row_len"].ctypes.data, b["offsets"].ctypes.data,
                            b["col_p"].ctypes.data, b["val_p"].ctypes.data, None)


@pytest.mark.parametrize("field,delta", [("n_pad", -64), ("n_pad", 64), ("n_blocks", 1), ("n_offsets", -1),
                                         ("max_row_len", -1), ("n_split_groups", 1), ("sort_window", -1)])
def test_c_convert_refuses_an_inconsistent_plan(field, delta):
    # through the C interface directly: the library checks every size against its own plan
    # before it allocates from it or writes; the buffers here are generously sized sentinels
    rp = np.ascontiguousarray(A.row_ptr, np.int64)
    col = np.ascontiguousarray(A.col, np.int32)
    val = np.ascontiguousarray(A.val)
    info = planned(A)
    setattr(info, field, getattr(info, field) + delta)
    big = 4 * (INFO.nnz_stored + INFO.n_pad + 64)
    b = dict(perm=np.full(big, -7, np.int32), row_len=np.full(big, -7, np.int32), offsets=np.full(big, -7, np.int64),
             col_p=np.full(big, -7, np.int32), val_p=np.full(big, -7.0))
    rc = _raw_convert(info, rp, col, val, b)
    assert rc == L.PJDS_ERR_ARG, L.pjds_last_error()
    for k, v in b.items():
        assert np.all(v == -7), f"{k} was written"


def test_c_ellr_convert_refuses_an_inconsistent_plan():
    rp = np.ascontiguousarray(A.row_ptr, np.int64)
    E = L.ellr_plan(A.n_rows, A.n_cols, rp)
    E.max_row_len = E.max_row_len - 1
    E.nnz_stored = E.n_pad * E.max_row_len
    lib = L.lib()
    rowmax = np.full(E.n_pad, -7, np.int32)
    col_e = np.full(E.n_pad * (E.max_row_len + 1), -7, np.int32)
    val_e = np.full(E.n_pad * (E.max_row_len + 1), -7.0)
    rc = lib.ellr_convert(ctypes.byref(E), rp.ctypes.data, np.ascontiguousarray(A.col, np.int32).ctypes.data,
                          np.ascontiguousarray(A.val).ctypes.data, L.PJDS_F64, rowmax.ctypes.data, col_e.ctypes.data,
                          val_e.ctypes.data)
    assert rc == L.PJDS_ERR_ARG
    assert np.all(rowmax == -7) and np.all(col_e == -7)


def test_c_staged_products_refuse_a_null_x_without_entries():
    # a matrix with no entries still copies x into LDS per tile: a NULL x is refused up front
    Z = synth.CSR(4096, 4096, np.zeros(4097, np.int64), np.zeros(0, np.int32), np.zeros(0))
    info = planned(Z, sort_window=1024, flags=L.PJDS_LAYOUT_BLOCK)
    assert info.nnz_stored == 0
    lib = L.lib()
    dummy = ctypes.c_void_p(16)                      # never dereferenced: the call must refuse first
    rc = lib.pjds_spmv_xlds(ctypes.byref(info), dummy, dummy, None, None, dummy, L.PJDS_F64, None, dummy,
                            256, 1024, L.PJDS_Y_PERMUTED, None)
    assert rc == L.PJDS_ERR_ARG and "d_x" in L.pjds_last_error()
    rc = lib.pjds_spmmv_xlds(ctypes.byref(info), dummy, dummy, None, None, dummy, L.PJDS_F64, 4, 4, 4, None,
                             dummy, 256, 1024, L.PJDS_Y_PERMUTED, None)
    assert rc == L.PJDS_ERR_ARG and "d_X" in L.pjds_last_error()


def test_one_byte_lengths_are_checked():
    """With PJDS_ROW_LEN8 the lengths must be the uint8 copy (an int32 array there would be
    read as bytes); pjds_pack_lengths wants an int32 source and a uint8 destination."""
    B = synth.random_csr(3000, 3000, 5, max_len=12)
    info = planned(B, sort_window=256, flags=L.PJDS_LAYOUT_BLOCK)
    ops = operands(info)
    with pytest.raises(TypeError):
        L.pjds_spmv_xlds(info, ops["d_row_len"], ops["d_offsets"], ops["d_col_p"], ops["d_val_p"], ops["d_perm"],
                         ops["d_x"], ops["d_y"], 256, 0, L.PJDS_ROW_LEN8)
    with pytest.raises(TypeError):
        L.pjds_pack_lengths(info, FakeDev(info.n_pad, torch.int32), FakeDev(info.n_pad, torch.int32))
    with pytest.raises(ValueError):
        L.pjds_pack_lengths(info, FakeDev(info.n_pad, torch.int32), FakeDev(info.n_pad - 1, torch.uint8))


def test_one_byte_lengths_refused_for_long_rows_before_any_launch():
    lens = np.ones(2000, np.int64)
    lens[7] = 256
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    info = L.pjds_plan(2000, 2000, row_ptr, 64, 256, L.PJDS_LAYOUT_BLOCK, 0)
    assert info.max_row_len == 256
    lib = L.lib()
    dummy = ctypes.c_void_p(16)
    assert lib.pjds_pack_lengths(ctypes.byref(info), dummy, dummy, None) == L.PJDS_ERR_UNSUPPORTED
    assert "byte" in L.pjds_last_error()
    rc = lib.pjds_spmv_xlds(ctypes.byref(info), dummy, dummy, dummy, dummy, dummy, L.PJDS_F64, dummy, dummy,
                            256, 0, L.PJDS_Y_PERMUTED | L.PJDS_ROW_LEN8, None)
    assert rc == L.PJDS_ERR_UNSUPPORTED
