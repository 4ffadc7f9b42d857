"""ctypes binding of libpjds (include/pjds.h): the same entry points, argument marshalling only.

Host arrays are numpy arrays; device arrays are torch tensors on a ROCm device (used only
as device memory); streams are ``torch.cuda.Stream`` objects or raw ``hipStream_t``
integers.  Every call checks the status and raises ``PjdsError`` with the library's
message.  Loading fails loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpjds.so")

PJDS_OK = 0
PJDS_ERR_ARG = -1
PJDS_ERR_INDEX = -2
PJDS_ERR_OVERFLOW = -3
PJDS_ERR_NOMEM = -4
PJDS_ERR_HIP = -5
PJDS_ERR_UNSUPPORTED = -6

PJDS_F64 = 0
PJDS_F32 = 1

PJDS_LAYOUT_JD = 0x0
PJDS_LAYOUT_BLOCK = 0x1
PJDS_SYMMETRIC = 0x2
PJDS_Y_PERMUTED = 0x4
PJDS_XCD_REMAP = 0x8
PJDS_TWO_ROWS = 0x10
PJDS_ROW_LEN8 = 0x20
PJDS_LANES_SHIFT = 8
PJDS_NOALLOC_SCRATCH_BYTES = 16 << 20
PJDS_LANES_MASK = 0x7 << PJDS_LANES_SHIFT


def PJDS_LANES(k: int) -> int:
    """Conversion flag for T = 2^k lanes per sorted row (block layout, block height 64 / T)."""
    return (int(k) << PJDS_LANES_SHIFT) & PJDS_LANES_MASK


class PjdsError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


class pjds_info(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("n_pad", ctypes.c_int64),
        ("n_blocks", ctypes.c_int64), ("nnz", ctypes.c_int64), ("nnz_stored", ctypes.c_int64),
        ("sort_window", ctypes.c_int64), ("n_offsets", ctypes.c_int64),
        ("block_height", ctypes.c_int32), ("max_row_len", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("split_len", ctypes.c_int32),
        ("n_chunks", ctypes.c_int64), ("n_split_groups", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


PJDS_BATCH_PERSISTENT = 0
PJDS_BATCH_GRAPH = 1
PJDS_BATCH_DIRECT = 2


class pjds_batch_member(ctypes.Structure):
    _fields_ = [("info", ctypes.POINTER(pjds_info)), ("d_row_len", ctypes.c_void_p),
                ("d_offsets", ctypes.c_void_p), ("d_col_p", ctypes.c_void_p),
                ("d_val_p", ctypes.c_void_p), ("d_perm", ctypes.c_void_p),
                ("d_x", ctypes.c_void_p), ("d_y", ctypes.c_void_p)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_ip = ctypes.POINTER(pjds_info)

# name -> argtypes (all return int unless listed in _RESTYPE)
_SIGS = {
    "pjds_plan": [_i64, _i64, _vp, _i32, _i64, _u32, _i32, _ip],
    "pjds_convert": [_ip, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
    "pjds_workspace_size": [_ip, _i32, ctypes.POINTER(ctypes.c_int64)],
    "pjds_workspace_init": [_ip, _i32, _vp, _vp],
    "pjds_spmv": [_ip, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _u32, _vp],
    "pjds_spmv_noalloc": [_ip, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _u32, _vp],
    "pjds_spmmv": [_ip, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _u32, _vp],
    "pjds_spmmv_xlds": [_ip, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _u32, _vp],
    "pjds_spmv_axpby": [_ip, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp, _u32, _vp],
    "pjds_lanczos_workspace": [_ip, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "pjds_lanczos": [_ip, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _u32, _vp, _vp, _vp, _vp, _vp],
    "pjds_spmv_xlds": [_ip, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _i32, _u32, _vp],
    "pjds_pack_lengths": [_ip, _vp, _vp, _vp],
    "pjds_split_count": [_i64, _i64, _vp, _vp, _i64, _i64, ctypes.POINTER(_i64)],
    "pjds_split_columns": [_i64, _i64, _vp, _vp, _vp, _i32, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp],
    "ellr_plan": [_i64, _i64, _vp, _ip],
    "ellr_convert": [_ip, _vp, _vp, _vp, _i32, _vp, _vp, _vp],
    "ellr_spmv": [_ip, _vp, _vp, _vp, _i32, _vp, _vp, _vp],
    "csr_spmv": [_i64, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp],
    "pjds_probe": [_i32, _vp, _vp, _i64, _vp],
    "pjds_time_next_launch": [_vp, _vp],
    "pjds_features": [_i64, _i64, _vp, _vp, _vp],
    "mlp_param_count": [_i32, _i32, ctypes.POINTER(_i64)],
    "mlp_workspace_size": [_i32, _i32, _i64, ctypes.POINTER(_i64)],
    "mlp_forward": [_vp, _i32, _i32, _i64, _vp, _vp, _vp],
    "mlp_backward": [_vp, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "mlp_adam_step": [_vp, _vp, _vp, _vp, _i64, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp],
    "mlp_infer": [_vp, _i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "pjds_batch_create": [_i32, ctypes.POINTER(pjds_batch_member), _i32, _u32, _i32, _i32, ctypes.POINTER(_vp)],
    "pjds_batch_create_xlds": [_i32, ctypes.POINTER(pjds_batch_member), _i32, _u32, _i32, _i32, ctypes.POINTER(_vp)],
    "pjds_batch_launch": [_vp, _vp],
    "pjds_batch_info": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "pjds_batch_destroy": [_vp],
    "pjds_last_error": [],
    "pjds_version": [],
}
_RESTYPE = {"pjds_last_error": ctypes.c_char_p, "pjds_version": ctypes.c_char_p}
EXPORTED = tuple(_SIGS)


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1112_5588_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _RESTYPE.get(name, ctypes.c_int)
        _lib = L
    return _lib


def _check(rc: int, where: str) -> None:
    if rc != PJDS_OK:
        raise PjdsError(rc, where, pjds_last_error())


def _host(a, dtype=None):
    """Pointer of a contiguous numpy array (None -> NULL)."""
    if a is None:
        return None
    if dtype is not None and a.dtype != np.dtype(dtype):
        raise TypeError(f"expected {np.dtype(dtype)}, got {a.dtype}")
    if not a.flags.c_contiguous:
        raise ValueError("host arrays must be C-contiguous")
    return a.ctypes.data if a.size else a.ctypes.data or None


def _dev(t):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device arrays must be torch tensors on the GPU")
    if not t.is_contiguous():
        raise ValueError("device arrays must be contiguous")
    return t.data_ptr() or None


def _dev_vec(t, n: int, code: int, name: str, like=None, required: bool = True):
    """Checks a device array argument before its pointer goes to a kernel: a torch tensor on
    the GPU (on ``like``'s device), of the kernel's value type ``code`` and with at least n
    elements.  A kernel would otherwise read or write past its end, or reinterpret its bytes."""
    if t is None:
        if required and n > 0:
            raise ValueError(f"{name} is required")
        return None
    if not hasattr(t, "is_cuda") or not t.is_cuda:
        raise ValueError(f"{name} must be a torch tensor on the GPU")
    if code is not None and _dtype_code(t.dtype) != code:
        raise TypeError(f"{name} has dtype {t.dtype}, the matrix values are {'float64' if code == PJDS_F64 else 'float32'}")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, {n} needed")
    if like is not None and t.device != like.device:
        raise ValueError(f"{name} is on {t.device}, the matrix on {like.device}")
    return t


def _dev_int(t, n: int, dtype, name: str, like=None, required: bool = True):
    """An index array on the device: its integer type and at least n elements."""
    if t is None:
        if required and n > 0:
            raise ValueError(f"{name} is required")
        return None
    if not hasattr(t, "is_cuda") or not t.is_cuda:
        raise ValueError(f"{name} must be a torch tensor on the GPU")
    if str(t.dtype).replace("torch.", "") != np.dtype(dtype).name:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {np.dtype(dtype).name}")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements, {n} needed")
    if like is not None and t.device != like.device:
        raise ValueError(f"{name} is on {t.device}, the matrix on {like.device}")
    return t


def _host_arr(a, n: int, dtype, name: str, required: bool = True):
    """A host array argument: its type and at least n elements."""
    if a is None:
        if required and n > 0:
            raise ValueError(f"{name} is required")
        return
    if dtype is not None and a.dtype != np.dtype(dtype):
        raise TypeError(f"{name} has dtype {a.dtype}, expected {np.dtype(dtype)}")
    if a.size < n:
        raise ValueError(f"{name} holds {a.size} elements, {n} needed")


def _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_x, d_y, k: int = 1,
                   need_perm: bool = True, len8: bool = False):
    """The device operands of a product on a pJDS matrix, checked against its sizes: values
    and x, y of one type, x of n_cols * k and y of n_rows * k elements, index arrays of the
    planned lengths.  Returns the dtype code."""
    if d_y is None:
        raise ValueError("y is required")
    code = _dtype_code(d_y.dtype)
    _dev_vec(d_y, info.n_rows * k, code, "y")
    _dev_vec(d_x, info.n_cols * k, code, "x", like=d_y)
    _dev_vec(d_val_p, info.nnz_stored, code, "val_p", like=d_y)
    _dev_int(d_col_p, info.nnz_stored, np.int32, "col_p", like=d_y)
    _dev_int(d_row_len, info.n_pad, np.uint8 if len8 else np.int32, "row_len", like=d_y)
    _dev_int(d_offsets, info.n_offsets, np.int64, "offsets", like=d_y)
    _dev_int(d_perm, info.n_rows, np.int32, "perm", like=d_y, required=need_perm)
    return code


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _dtype_code(dt) -> int:
    name = str(dt).replace("torch.", "")
    if name.startswith("<class"):                 # numpy scalar types such as np.float64
        name = np.dtype(dt).name
    if name in ("float64", "double"):
        return PJDS_F64
    if name in ("float32", "float"):
        return PJDS_F32
    raise TypeError(f"unsupported value type {dt}")


# ------------------------------------------------------------------ entry points

def pjds_last_error() -> str:
    return (lib().pjds_last_error() or b"").decode()


def pjds_version() -> str:
    return lib().pjds_version().decode()


def pjds_plan(n_rows: int, n_cols: int, row_ptr: np.ndarray, block_height: int = 64,
              sort_window: int = 0, flags: int = 0, split_len: int = 0) -> pjds_info:
    info = pjds_info()
    _check(lib().pjds_plan(n_rows, n_cols, _host(row_ptr, np.int64), block_height, sort_window,
                           flags, split_len, ctypes.byref(info)), "pjds_plan")
    return info


def pjds_convert(info: pjds_info, row_ptr, col_idx, val, perm, row_len, offsets, col_p, val_p,
                 sched=None) -> None:
    _host_arr(row_ptr, info.n_rows + 1, np.int64, "row_ptr")
    _host_arr(col_idx, info.nnz, np.int32, "col_idx")
    _host_arr(val, info.nnz, None, "val")
    _host_arr(perm, info.n_rows, np.int32, "perm")
    _host_arr(row_len, info.n_pad, np.int32, "row_len")
    _host_arr(offsets, info.n_offsets, np.int64, "offsets")
    _host_arr(col_p, info.nnz_stored, np.int32, "col_p")
    _host_arr(val_p, info.nnz_stored, val.dtype, "val_p")
    _host_arr(sched, 4 * info.n_chunks, np.int32, "sched", required=info.n_chunks > 0)
    _check(lib().pjds_convert(ctypes.byref(info), _host(row_ptr, np.int64), _host(col_idx, np.int32),
                              _host(val), _dtype_code(val.dtype), _host(perm, np.int32),
                              _host(row_len, np.int32), _host(offsets, np.int64),
                              _host(col_p, np.int32), _host(val_p), _host(sched, np.int32)),
           "pjds_convert")


def pjds_workspace_size(info: pjds_info, dtype) -> int:
    out = ctypes.c_int64(0)
    _check(lib().pjds_workspace_size(ctypes.byref(info), _dtype_code(dtype), ctypes.byref(out)),
           "pjds_workspace_size")
    return out.value


def pjds_workspace_init(info: pjds_info, dtype, d_work, stream=None) -> None:
    _check(lib().pjds_workspace_init(ctypes.byref(info), _dtype_code(dtype), _dev(d_work),
                                     _stream(stream)), "pjds_workspace_init")


def pjds_spmv(info: pjds_info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_sched, d_work,
              d_x, d_y, flags: int = 0, stream=None) -> None:
    _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_x, d_y,
                   need_perm=not flags & PJDS_Y_PERMUTED)
    _dev_int(d_sched, 4 * info.n_chunks, np.int32, "sched", like=d_y, required=info.n_chunks > 0)
    _check(lib().pjds_spmv(ctypes.byref(info), _dev(d_row_len), _dev(d_offsets), _dev(d_col_p),
                           _dev(d_val_p), _dev(d_perm), _dev(d_sched), _dev(d_work),
                           _dtype_code(d_y.dtype), _dev(d_x), _dev(d_y), flags, _stream(stream)),
           "pjds_spmv")


def pjds_spmv_noalloc(info: pjds_info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_sched,
                      d_x, d_y, flags: int = 0, stream=None) -> None:
    """pjds_spmv without a workspace argument: the library's fixed device scratch holds the
    long-row partial sums (calls that overlap on one GPU race)."""
    _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_x, d_y,
                   need_perm=not flags & PJDS_Y_PERMUTED)
    _dev_int(d_sched, 4 * info.n_chunks, np.int32, "sched", like=d_y, required=info.n_chunks > 0)
    _check(lib().pjds_spmv_noalloc(ctypes.byref(info), _dev(d_row_len), _dev(d_offsets), _dev(d_col_p),
                                   _dev(d_val_p), _dev(d_perm), _dev(d_sched), _dtype_code(d_y.dtype),
                                   _dev(d_x), _dev(d_y), flags, _stream(stream)), "pjds_spmv_noalloc")


def pjds_spmv_xlds(info: pjds_info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_x, d_y,
                   x_halo: int, tile_rows: int = 0, flags: int = 0, stream=None) -> None:
    """With PJDS_ROW_LEN8 in flags, d_row_len is the uint8 copy from pjds_pack_lengths."""
    _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_x, d_y,
                   need_perm=not flags & PJDS_Y_PERMUTED, len8=bool(flags & PJDS_ROW_LEN8))
    _check(lib().pjds_spmv_xlds(ctypes.byref(info), _dev(d_row_len), _dev(d_offsets), _dev(d_col_p),
                                _dev(d_val_p), _dev(d_perm), _dtype_code(d_y.dtype), _dev(d_x), _dev(d_y),
                                x_halo, tile_rows, flags, _stream(stream)), "pjds_spmv_xlds")


def pjds_pack_lengths(info: pjds_info, d_row_len, d_row_len8, stream=None) -> None:
    """One-byte copies of the row lengths (d_row_len8: uint8 tensor of n_pad elements)."""
    _dev_int(d_row_len, info.n_pad, np.int32, "row_len")
    _dev_int(d_row_len8, info.n_pad, np.uint8, "row_len8", like=d_row_len)
    _check(lib().pjds_pack_lengths(ctypes.byref(info), _dev(d_row_len), _dev(d_row_len8), _stream(stream)),
           "pjds_pack_lengths")


def pjds_spmmv(info: pjds_info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, k: int,
               vectors_per_tile: int, d_X, d_Y, flags: int = 0, stream=None,
               vectors_per_lane: int = 1) -> None:
    _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_X, d_Y, k=max(k, 0),
                   need_perm=not flags & PJDS_Y_PERMUTED)
    _check(lib().pjds_spmmv(ctypes.byref(info), _dev(d_row_len), _dev(d_offsets), _dev(d_col_p),
                            _dev(d_val_p), _dev(d_perm), _dtype_code(d_Y.dtype), k,
                            vectors_per_tile, vectors_per_lane, _dev(d_X), _dev(d_Y), flags,
                            _stream(stream)), "pjds_spmmv")


def pjds_spmmv_xlds(info: pjds_info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, k: int,
                    vectors_per_tile: int, vectors_per_lane: int, d_X, d_Y, x_halo: int, tile_rows: int,
                    flags: int = 0, stream=None) -> None:
    _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_X, d_Y, k=max(k, 0),
                   need_perm=not flags & PJDS_Y_PERMUTED)
    _check(lib().pjds_spmmv_xlds(ctypes.byref(info), _dev(d_row_len), _dev(d_offsets), _dev(d_col_p),
                                 _dev(d_val_p), _dev(d_perm), _dtype_code(d_Y.dtype), k,
                                 vectors_per_tile, vectors_per_lane, _dev(d_X), _dev(d_Y), x_halo,
                                 tile_rows, flags, _stream(stream)), "pjds_spmmv_xlds")


def pjds_split_count(n_rows: int, n_cols: int, row_ptr, col_idx, c0: int, c1: int) -> int:
    _host_arr(row_ptr, n_rows + 1, np.int64, "row_ptr")
    out = _i64(0)
    _check(lib().pjds_split_count(n_rows, n_cols, _host(row_ptr, np.int64), _host(col_idx, np.int32), c0, c1,
                                  ctypes.byref(out)), "pjds_split_count")
    return out.value


def pjds_split_columns(n_rows: int, n_cols: int, row_ptr, col_idx, val, c0: int, c1: int,
                       rp_loc, col_loc, val_loc, rp_nl, col_nl, val_nl) -> None:
    _host_arr(row_ptr, n_rows + 1, np.int64, "row_ptr")
    nnz = int(row_ptr[n_rows])
    _host_arr(col_idx, nnz, np.int32, "col_idx")
    _host_arr(val, nnz, None, "val")
    loc = pjds_split_count(n_rows, n_cols, row_ptr, col_idx, c0, c1)
    for name, a, n, dt in (("rp_loc", rp_loc, n_rows + 1, np.int64), ("rp_nl", rp_nl, n_rows + 1, np.int64),
                           ("col_loc", col_loc, loc, np.int32), ("col_nl", col_nl, nnz - loc, np.int32),
                           ("val_loc", val_loc, loc, val.dtype), ("val_nl", val_nl, nnz - loc, val.dtype)):
        _host_arr(a, n, dt, name)
    _check(lib().pjds_split_columns(n_rows, n_cols, _host(row_ptr, np.int64), _host(col_idx, np.int32), _host(val),
                                    _dtype_code(val.dtype), c0, c1, _host(rp_loc, np.int64), _host(col_loc, np.int32),
                                    _host(val_loc), _host(rp_nl, np.int64), _host(col_nl, np.int32), _host(val_nl)),
           "pjds_split_columns")


def ellr_plan(n_rows: int, n_cols: int, row_ptr: np.ndarray) -> pjds_info:
    info = pjds_info()
    _check(lib().ellr_plan(n_rows, n_cols, _host(row_ptr, np.int64), ctypes.byref(info)), "ellr_plan")
    return info


def ellr_convert(info: pjds_info, row_ptr, col_idx, val, rowmax, col_e, val_e) -> None:
    _host_arr(row_ptr, info.n_rows + 1, np.int64, "row_ptr")
    _host_arr(col_idx, info.nnz, np.int32, "col_idx")
    _host_arr(val, info.nnz, None, "val")
    _host_arr(rowmax, info.n_pad, np.int32, "rowmax")
    _host_arr(col_e, info.nnz_stored, np.int32, "col_e")
    _host_arr(val_e, info.nnz_stored, val.dtype, "val_e")
    _check(lib().ellr_convert(ctypes.byref(info), _host(row_ptr, np.int64), _host(col_idx, np.int32),
                              _host(val), _dtype_code(val.dtype), _host(rowmax, np.int32),
                              _host(col_e, np.int32), _host(val_e)), "ellr_convert")


def ellr_spmv(info: pjds_info, d_rowmax, d_col_e, d_val_e, d_x, d_y, stream=None) -> None:
    if d_y is None:
        raise ValueError("y is required")
    code = _dtype_code(d_y.dtype)
    _dev_vec(d_y, info.n_rows, code, "y")
    _dev_vec(d_x, info.n_cols, code, "x", like=d_y)
    _dev_vec(d_val_e, info.nnz_stored, code, "val_e", like=d_y)
    _dev_int(d_col_e, info.nnz_stored, np.int32, "col_e", like=d_y)
    _dev_int(d_rowmax, info.n_pad, np.int32, "rowmax", like=d_y)
    _check(lib().ellr_spmv(ctypes.byref(info), _dev(d_rowmax), _dev(d_col_e), _dev(d_val_e),
                           _dtype_code(d_y.dtype), _dev(d_x), _dev(d_y), _stream(stream)), "ellr_spmv")


def csr_spmv(n_rows: int, n_cols: int, d_row_ptr, d_col, d_val, d_x, d_y, variant: int = 1,
             stream=None, nnz: int | None = None) -> None:
    """``nnz`` (optional, the caller's count of entries) checks the sizes of col and val."""
    if d_y is None:
        raise ValueError("y is required")
    code = _dtype_code(d_y.dtype)
    _dev_vec(d_y, n_rows, code, "y")
    _dev_vec(d_x, n_cols, code, "x", like=d_y)
    _dev_int(d_row_ptr, n_rows + 1, np.int64, "row_ptr", like=d_y)
    if nnz is not None:
        _dev_vec(d_val, nnz, code, "val", like=d_y)
        _dev_int(d_col, nnz, np.int32, "col", like=d_y)
    _check(lib().csr_spmv(n_rows, n_cols, _dev(d_row_ptr), _dev(d_col), _dev(d_val),
                          _dtype_code(d_y.dtype), _dev(d_x), _dev(d_y), variant, _stream(stream)),
           "csr_spmv")


def pjds_probe(mode: int, d_in, d_out, n: int, stream=None) -> None:
    _dev_vec(d_in, n, PJDS_F64, "in")
    _dev_vec(d_out, n if mode == 1 else 2048, PJDS_F64, "out", like=d_in)
    _check(lib().pjds_probe(mode, _dev(d_in), _dev(d_out), n, _stream(stream)), "pjds_probe")


def pjds_time_next_launch(start_event, stop_event) -> None:
    """Arm the kernel timing hook with two hipEvent_t handles, or disarm it with (None, None)."""
    _check(lib().pjds_time_next_launch(start_event, stop_event), "pjds_time_next_launch")


class KernelTimer:
    """Two HIP events for pjds_time_next_launch.  `arm()` before a call, `disarm()` after it;
    once the stream has synchronized, `ms()` is the armed kernel's own duration, or None when
    no kernel recorded the events.  The events come from the HIP runtime the library and torch
    already share (libamdhip64.so.7)."""

    _hip = None

    def __init__(self):
        if KernelTimer._hip is None:
            h = ctypes.CDLL("libamdhip64.so.7")
            h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
            h.hipEventDestroy.argtypes = [ctypes.c_void_p]
            h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
            KernelTimer._hip = h
        self.ev = [ctypes.c_void_p(), ctypes.c_void_p()]
        for e in self.ev:
            rc = KernelTimer._hip.hipEventCreate(ctypes.byref(e))
            if rc != 0:
                raise PjdsError(PJDS_ERR_HIP, "hipEventCreate", f"error {rc}")

    def arm(self) -> None:
        pjds_time_next_launch(self.ev[0], self.ev[1])

    @staticmethod
    def disarm() -> None:
        pjds_time_next_launch(None, None)

    def ms(self):
        out = ctypes.c_float()
        rc = KernelTimer._hip.hipEventElapsedTime(ctypes.byref(out), self.ev[0], self.ev[1])
        if rc != 0:
            KernelTimer._hip.hipGetLastError()      # the failed query is no launch error
            return None
        return float(out.value)

    def __del__(self):
        if KernelTimer._hip is not None:
            for e in self.ev:
                if e.value:
                    KernelTimer._hip.hipEventDestroy(e)


def _batch_members(members: list, flags: int):
    """The C array of batch members, each member's operands checked against its sizes."""
    arr = (pjds_batch_member * len(members))()
    for k, (info, rl, off, cp, vp, perm, x, y) in enumerate(members):
        try:
            _pjds_operands(info, rl, off, cp, vp, perm, x, y, need_perm=not flags & PJDS_Y_PERMUTED)
        except (TypeError, ValueError) as e:
            raise type(e)(f"batch member {k}: {e}") from None
        arr[k] = pjds_batch_member(ctypes.pointer(info), _dev(rl), _dev(off), _dev(cp), _dev(vp),
                                   _dev(perm), _dev(x), _dev(y))
    return arr


def pjds_batch_create(members: list, dtype, flags: int = 0, mode: int = PJDS_BATCH_PERSISTENT,
                      groups_per_tile: int = 0) -> int:
    """members: list of (info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_x, d_y).
    Returns the opaque handle (an integer address)."""
    arr = _batch_members(members, flags)
    h = _vp()
    _check(lib().pjds_batch_create(len(members), arr, _dtype_code(dtype), flags, mode,
                                   groups_per_tile, ctypes.byref(h)), "pjds_batch_create")
    return h.value


def pjds_batch_create_xlds(members: list, dtype, flags: int = 0, groups_per_tile: int = 0,
                           x_halo: int = 4096) -> int:
    """Like pjds_batch_create (persistent mode) with x staged in LDS per tile."""
    arr = _batch_members(members, flags)
    h = _vp()
    _check(lib().pjds_batch_create_xlds(len(members), arr, _dtype_code(dtype), flags, groups_per_tile,
                                        x_halo, ctypes.byref(h)), "pjds_batch_create_xlds")
    return h.value


def pjds_batch_launch(handle: int, stream=None) -> None:
    _check(lib().pjds_batch_launch(handle, _stream(stream)), "pjds_batch_launch")


def pjds_batch_info(handle: int) -> tuple[int, int]:
    t, g = _i32(0), _i32(0)
    _check(lib().pjds_batch_info(handle, ctypes.byref(t), ctypes.byref(g)), "pjds_batch_info")
    return t.value, g.value


def pjds_batch_destroy(handle: int) -> None:
    _check(lib().pjds_batch_destroy(handle), "pjds_batch_destroy")


def pjds_features(n_rows: int, n_cols: int, row_ptr, col_idx) -> np.ndarray:
    out = np.zeros(24, np.float32)
    _check(lib().pjds_features(n_rows, n_cols, _host(row_ptr, np.int64), _host(col_idx, np.int32),
                               _host(out)), "pjds_features")
    return out


def mlp_param_count(d_in: int, d_out: int) -> int:
    n = _i64(0)
    _check(lib().mlp_param_count(d_in, d_out, ctypes.byref(n)), "mlp_param_count")
    return n.value


def mlp_workspace_size(d_in: int, d_out: int, batch: int) -> int:
    n = _i64(0)
    _check(lib().mlp_workspace_size(d_in, d_out, batch, ctypes.byref(n)), "mlp_workspace_size")
    return n.value


def _mlp_operands(d_params, d_in: int, d_out: int, d_X, batch_outputs: dict) -> None:
    """The tuner network's device operands: float32, params of the planned count, X of
    batch x d_in and each named output of batch x (its width)."""
    n = mlp_param_count(d_in, d_out)
    _dev_vec(d_params, n, PJDS_F32, "params")
    batch = d_X.shape[0] if d_X is not None else 0
    _dev_vec(d_X, batch * d_in, PJDS_F32, "X", like=d_params)
    for name, (t, width, code) in batch_outputs.items():
        if code is None:
            _dev_int(t, batch * width, np.int32, name, like=d_params, required=False)
        else:
            _dev_vec(t, batch * width, code, name, like=d_params, required=False)


def mlp_forward(d_params, d_in: int, d_out: int, d_X, d_P, stream=None) -> None:
    _mlp_operands(d_params, d_in, d_out, d_X, {"P": (d_P, d_out, PJDS_F32)})
    _dev_vec(d_P, d_X.shape[0] * d_out, PJDS_F32, "P")
    _check(lib().mlp_forward(_dev(d_params), d_in, d_out, d_X.shape[0], _dev(d_X), _dev(d_P),
                             _stream(stream)), "mlp_forward")


def mlp_backward(d_params, d_in: int, d_out: int, d_X, d_T, d_M, d_grad, d_loss, d_work, stream=None) -> None:
    _mlp_operands(d_params, d_in, d_out, d_X, {"T": (d_T, d_out, PJDS_F32), "M": (d_M, d_out, PJDS_F32)})
    _dev_vec(d_T, d_X.shape[0] * d_out, PJDS_F32, "T")
    _dev_vec(d_grad, mlp_param_count(d_in, d_out), PJDS_F32, "grad", like=d_params)
    ws = mlp_workspace_size(d_in, d_out, d_X.shape[0])
    if d_work is None or d_work.numel() * d_work.element_size() < ws:
        raise ValueError(f"work holds fewer than the {ws} bytes mlp_backward needs")
    _check(lib().mlp_backward(_dev(d_params), d_in, d_out, d_X.shape[0], _dev(d_X), _dev(d_T), _dev(d_M),
                              _dev(d_grad), _dev(d_loss), _dev(d_work), _stream(stream)), "mlp_backward")


def mlp_adam_step(d_params, d_grad, d_m, d_v, step: int, lr: float = 1e-3, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    n = d_params.numel()
    for name, t in (("grad", d_grad), ("m", d_m), ("v", d_v)):
        _dev_vec(t, n, PJDS_F32, name, like=d_params)
    _check(lib().mlp_adam_step(_dev(d_params), _dev(d_grad), _dev(d_m), _dev(d_v), d_params.numel(), step,
                               lr, beta1, beta2, eps, _stream(stream)), "mlp_adam_step")


def mlp_infer(d_params, d_in: int, d_out: int, d_X, d_scale, d_shift, d_valid, d_idx, d_margin, stream=None) -> None:
    _mlp_operands(d_params, d_in, d_out, d_X, {"idx": (d_idx, 1, None), "margin": (d_margin, 1, PJDS_F32)})
    for name, t in (("scale", d_scale), ("shift", d_shift), ("valid", d_valid)):
        _dev_vec(t, d_out, PJDS_F32, name, like=d_params, required=False)
    _dev_int(d_idx, d_X.shape[0], np.int32, "idx")
    _check(lib().mlp_infer(_dev(d_params), d_in, d_out, d_X.shape[0], _dev(d_X), _dev(d_scale), _dev(d_shift),
                           _dev(d_valid), _dev(d_idx), _dev(d_margin), _stream(stream)), "mlp_infer")


def pjds_spmv_axpby(info: pjds_info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_sched, d_work,
                    d_x, alpha: float, beta: float, d_z, d_y, flags: int = 0, stream=None) -> None:
    code = _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, d_perm, d_x, d_y,
                          need_perm=not flags & PJDS_Y_PERMUTED)
    _dev_vec(d_z, info.n_rows, code, "z", like=d_y, required=False)
    _dev_int(d_sched, 4 * info.n_chunks, np.int32, "sched", like=d_y, required=info.n_chunks > 0)
    _check(lib().pjds_spmv_axpby(ctypes.byref(info), _dev(d_row_len), _dev(d_offsets), _dev(d_col_p),
                                 _dev(d_val_p), _dev(d_perm), _dev(d_sched), _dev(d_work),
                                 _dtype_code(d_y.dtype), _dev(d_x), alpha, beta, _dev(d_z), _dev(d_y),
                                 flags, _stream(stream)), "pjds_spmv_axpby")


def pjds_lanczos_workspace(info: pjds_info) -> tuple[int, int]:
    a, b = _i64(0), _i64(0)
    _check(lib().pjds_lanczos_workspace(ctypes.byref(info), ctypes.byref(a), ctypes.byref(b)),
           "pjds_lanczos_workspace")
    return a.value, b.value


def pjds_lanczos(info: pjds_info, d_row_len, d_offsets, d_col_p, d_val_p, d_sched, d_work, d_v0,
                 steps: int, x_halo: int, tile_rows: int, d_alpha, d_beta, d_vectors, d_scratch,
                 stream=None, flags: int = 0) -> None:
    if steps > 0 and info.n_rows > 0:
        _pjds_operands(info, d_row_len, d_offsets, d_col_p, d_val_p, None, d_v0, d_v0, need_perm=False,
                       len8=bool(flags & PJDS_ROW_LEN8))
        _dev_vec(d_alpha, steps, PJDS_F64, "alpha", like=d_v0)
        _dev_vec(d_beta, steps + 1, PJDS_F64, "beta", like=d_v0)
        vb, sb = pjds_lanczos_workspace(info)
        _dev_vec(d_vectors, vb // 8, PJDS_F64, "vectors", like=d_v0)
        _dev_vec(d_scratch, sb // 8, PJDS_F64, "scratch", like=d_v0)
    _check(lib().pjds_lanczos(ctypes.byref(info), _dev(d_row_len), _dev(d_offsets), _dev(d_col_p),
                              _dev(d_val_p), _dev(d_sched), _dev(d_work), _dev(d_v0), steps, x_halo,
                              tile_rows, flags, _dev(d_alpha), _dev(d_beta), _dev(d_vectors), _dev(d_scratch),
                              _stream(stream)), "pjds_lanczos")
