"""Device-resident sparse matrices built through the C interface.

``PjdsMatrix.from_csr`` plans and converts on the host (pjds_plan / pjds_convert), then
copies the arrays to the GPU once; ``spmv`` / ``spmmv`` launch the HIP kernels on the
current (or given) stream.  ``EllrMatrix`` and ``CsrMatrix`` do the same for the two
comparison formats.  Inputs are any object with ``n_rows, n_cols, row_ptr, col, val``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


def _to_dev(a: np.ndarray, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def _tdtype(np_dtype) -> torch.dtype:
    return {np.dtype(np.float64): torch.float64, np.dtype(np.float32): torch.float32}[np.dtype(np_dtype)]


class PjdsMatrix:
    """A pJDS matrix on the GPU (Sect. 2.1 of the paper; see include/pjds.h)."""

    def __init__(self):
        self.info: L.pjds_info | None = None
        self.host: dict = {}

    @classmethod
    def from_csr(cls, A, block_height: int = 64, sort_window: int = 0, layout: str = "jd",
                 symmetric: bool = False, split_len: int = 0, device="cuda",
                 keep_host: bool = False, lanes: int = 1) -> "PjdsMatrix":
        """Convert CSR ``A`` (host arrays) and copy the pJDS arrays to ``device``.  ``lanes``
        = T > 1 (a power of two, block layout) lets T lanes share each row; the block height
        is then 64 / T whatever ``block_height`` says."""
        self = cls()
        flags = (L.PJDS_LAYOUT_BLOCK if layout == "block" else L.PJDS_LAYOUT_JD) | (L.PJDS_SYMMETRIC if symmetric else 0)
        if lanes != 1:
            k = int(lanes).bit_length() - 1
            if lanes < 1 or (1 << k) != lanes or lanes > 64:
                raise ValueError(f"lanes per row {lanes}: must be a power of two up to 64")
            flags |= L.PJDS_LANES(k)
            block_height = 64 // lanes
        row_ptr = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(A.col, dtype=np.int32)
        val = np.ascontiguousarray(A.val)
        info = L.pjds_plan(A.n_rows, A.n_cols, row_ptr, block_height, sort_window, flags, split_len)
        h = dict(
            perm=np.empty(max(info.n_rows, 1), np.int32),
            row_len=np.empty(max(info.n_pad, 1), np.int32),
            offsets=np.empty(max(info.n_offsets, 1), np.int64),
            col_p=np.empty(max(info.nnz_stored, 1), np.int32),
            val_p=np.empty(max(info.nnz_stored, 1), val.dtype),
            sched=np.empty(max(4 * info.n_chunks, 1), np.int32),
        )
        L.pjds_convert(info, row_ptr, col, val, h["perm"], h["row_len"], h["offsets"], h["col_p"],
                       h["val_p"], h["sched"] if info.n_chunks else None)
        self.info = info
        self.dtype = _tdtype(val.dtype)
        self.device = torch.device(device)
        self.d = {k: _to_dev(v, self.device) for k, v in h.items()}
        ws = L.pjds_workspace_size(info, self.dtype)
        self.d["work"] = torch.empty(max(ws, 1), dtype=torch.uint8, device=self.device) if ws else None
        if ws:
            L.pjds_workspace_init(info, self.dtype, self.d["work"])
        if keep_host:
            self.host = {k: (v[:info.n_rows] if k == "perm" else v[:info.n_pad] if k == "row_len"
                             else v[:info.n_offsets] if k == "offsets" else v[:4 * info.n_chunks] if k == "sched"
                             else v[:info.nnz_stored]) for k, v in h.items()}
        return self

    @classmethod
    def from_arrays(cls, n_rows: int, n_cols: int, row_ptr, col, val, **kw) -> "PjdsMatrix":
        """From CSR arrays given as numpy arrays or torch tensors (device tensors are copied to
        the host for the conversion)."""
        class _A:
            pass
        A = _A()
        A.n_rows, A.n_cols = n_rows, n_cols
        A.row_ptr, A.col, A.val = (a.cpu().numpy() if isinstance(a, torch.Tensor) else a for a in (row_ptr, col, val))
        return cls.from_csr(A, **kw)

    @property
    def n_rows(self) -> int:
        return self.info.n_rows

    @property
    def n_cols(self) -> int:
        return self.info.n_cols

    def spmv(self, x: torch.Tensor, y: torch.Tensor | None = None, y_permuted: bool = False,
             xcd_remap: bool = False, stream=None, two_rows: bool = False) -> torch.Tensor:
        if y is None:
            y = torch.empty(self.info.n_rows, dtype=self.dtype, device=self.device)
        flags = (L.PJDS_Y_PERMUTED if y_permuted else 0) | (L.PJDS_XCD_REMAP if xcd_remap else 0)
        flags |= L.PJDS_TWO_ROWS if two_rows else 0
        d = self.d
        L.pjds_spmv(self.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"], d["perm"],
                    d["sched"] if self.info.n_chunks else None, d["work"], x, y, flags, stream)
        return y

    def spmv_axpby(self, x: torch.Tensor, y: torch.Tensor, alpha: float = 1.0, beta: float = 0.0,
                   z: torch.Tensor | None = None, y_permuted: bool = False, stream=None) -> torch.Tensor:
        """y = alpha (A x) + beta z (z may be y: accumulate)."""
        flags = L.PJDS_Y_PERMUTED if y_permuted else 0
        d = self.d
        L.pjds_spmv_axpby(self.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"], d["perm"],
                          d["sched"] if self.info.n_chunks else None, d["work"], x, alpha, beta, z, y,
                          flags, stream)
        return y

    def lanczos_buffers(self) -> dict:
        """Device buffers for lanczos(): reuse them across calls (and inside a captured graph)."""
        vb, sb = L.pjds_lanczos_workspace(self.info)
        return {"vectors": torch.empty(vb // 8, dtype=torch.float64, device=self.device),
                "scratch": torch.empty(sb // 8, dtype=torch.float64, device=self.device)}

    def lanczos(self, v0: torch.Tensor, steps: int, x_halo: int = -1, tile_rows: int = 0,
                alpha: torch.Tensor | None = None, beta: torch.Tensor | None = None,
                buffers: dict | None = None, stream=None, len8: bool | None = None):
        """Lanczos coefficients (alpha [steps], beta [steps+1]) from start vector v0, given in the
        permuted basis; the matrix must have been converted with symmetric=True.  len8: the
        staged product (x_halo >= 0) reads the one-byte row lengths (None: whenever it can)."""
        if alpha is None:
            alpha = torch.empty(max(steps, 1), dtype=torch.float64, device=self.device)
        if beta is None:
            beta = torch.empty(steps + 1, dtype=torch.float64, device=self.device)
        b = buffers or self.lanczos_buffers()
        d = self.d
        if x_halo >= 0:
            rl, flags = self._staged_lengths(len8)
        elif len8:
            raise ValueError("one-byte row lengths need the staged product (x_halo >= 0)")
        else:
            rl, flags = d["row_len"], 0
        L.pjds_lanczos(self.info, rl, d["offsets"], d["col_p"], d["val_p"],
                       d["sched"] if self.info.n_chunks else None, d["work"], v0, steps, x_halo, tile_rows,
                       alpha, beta, b["vectors"], b["scratch"], stream, flags=flags)
        return alpha[:steps], beta

    def row_len8(self) -> torch.Tensor | None:
        """The one-byte copy of the row lengths (made once, on first use), or None when a row
        is longer than 255 entries."""
        if self.info.max_row_len > 255:
            return None
        if "row_len8" not in self.d:
            if torch.cuda.is_current_stream_capturing():
                # made inside a graph, the copy would hold its lengths only after a replay
                raise RuntimeError("make the one-byte row lengths (row_len8()) before capturing a graph")
            t = torch.empty(max(self.info.n_pad, 1), dtype=torch.uint8, device=self.device)
            L.pjds_pack_lengths(self.info, self.d["row_len"], t)
            self.d["row_len8"] = t
        return self.d["row_len8"]

    def _staged_lengths(self, len8: bool | None):
        """The row lengths a staged product reads and the flag that says which: the one-byte
        copy when len8 is True, the int32 array when False; None takes the copy whenever every
        row fits a byte and the copy exists or can be made now (not while a graph is being
        captured)."""
        if len8 is False:
            return self.d["row_len"], 0
        if len8 is None and "row_len8" not in self.d and torch.cuda.is_current_stream_capturing():
            return self.d["row_len"], 0
        r8 = self.row_len8()
        if r8 is None:
            if len8:
                raise ValueError(f"rows of {self.info.max_row_len} entries do not fit one-byte lengths")
            return self.d["row_len"], 0
        return r8, L.PJDS_ROW_LEN8

    def spmv_xlds(self, x: torch.Tensor, y: torch.Tensor | None = None, x_halo: int = 512,
                  tile_rows: int = 0, y_permuted: bool = False, xcd_remap: bool = False,
                  stream=None, two_rows: bool = False, len8: bool | None = None) -> torch.Tensor:
        """y = A x with x staged in LDS per workgroup tile (block layout, sort window % 256 == 0);
        two_rows: each lane takes two adjacent rows with 2-wide loads; len8: read the one-byte
        row lengths (None: whenever every row fits a byte)."""
        if y is None:
            y = torch.empty(self.info.n_rows, dtype=self.dtype, device=self.device)
        flags = (L.PJDS_Y_PERMUTED if y_permuted else 0) | (L.PJDS_XCD_REMAP if xcd_remap else 0)
        flags |= L.PJDS_TWO_ROWS if two_rows else 0
        d = self.d
        rl, f8 = self._staged_lengths(len8)
        flags |= f8
        L.pjds_spmv_xlds(self.info, rl, d["offsets"], d["col_p"], d["val_p"], d["perm"], x, y,
                         x_halo, tile_rows, flags, stream)
        return y

    def spmmv(self, X: torch.Tensor, Y: torch.Tensor | None = None, vectors_per_tile: int | None = None,
              y_permuted: bool = False, stream=None, vectors_per_lane: int | None = None,
              xcd_remap: bool = False) -> torch.Tensor:
        k = X.shape[1]
        if vectors_per_tile is None:
            vectors_per_tile = min(32, 1 << (k - 1).bit_length())
        if vectors_per_lane is None:
            vectors_per_lane = next(v for v in (4, 2, 1) if k % v == 0 and vectors_per_tile % v == 0)
        if Y is None:
            Y = torch.empty((self.info.n_rows, k), dtype=self.dtype, device=self.device)
        flags = (L.PJDS_Y_PERMUTED if y_permuted else 0) | (L.PJDS_XCD_REMAP if xcd_remap else 0)
        d = self.d
        L.pjds_spmmv(self.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"], d["perm"], k,
                     vectors_per_tile, X, Y, flags, stream, vectors_per_lane)
        return Y

    def spmmv_xlds(self, X: torch.Tensor, Y: torch.Tensor | None = None, vectors_per_tile: int | None = None,
                   vectors_per_lane: int | None = None, x_halo: int = 512, tile_rows: int = 1024,
                   y_permuted: bool = False, stream=None) -> torch.Tensor:
        """Y = A X with X staged in LDS per tile (pjds_spmmv_xlds): the block layout with a sort
        window; t / vectors_per_lane lanes per row of 1, 2 or 4 (default t: k, at most 4 lanes)."""
        k = X.shape[1]
        if vectors_per_lane is None:
            vectors_per_lane = next(v for v in (4, 2, 1) if k % v == 0)
        if vectors_per_tile is None:
            lanes = 1
            while lanes < 4 and lanes * vectors_per_lane < k:
                lanes *= 2
            vectors_per_tile = lanes * vectors_per_lane
        if Y is None:
            Y = torch.empty((self.info.n_rows, k), dtype=self.dtype, device=self.device)
        d = self.d
        L.pjds_spmmv_xlds(self.info, d["row_len"], d["offsets"], d["col_p"], d["val_p"], d["perm"], k,
                          vectors_per_tile, vectors_per_lane, X, Y, x_halo, tile_rows,
                          L.PJDS_Y_PERMUTED if y_permuted else 0, stream)
        return Y

    def footprint_bytes(self) -> int:
        """Device bytes of the format: values, column indices, row lengths, offsets, perm."""
        i = self.info
        vb = 8 if self.dtype == torch.float64 else 4
        return i.nnz_stored * (vb + 4) + i.n_pad * 4 + i.n_offsets * 8 + i.n_rows * 4


class EllrMatrix:
    """An ELLPACK-R matrix on the GPU (Listing 1)."""

    @classmethod
    def plan(cls, A) -> L.pjds_info:
        return L.ellr_plan(A.n_rows, A.n_cols, np.ascontiguousarray(A.row_ptr, dtype=np.int64))

    @classmethod
    def from_csr(cls, A, device="cuda", keep_host: bool = False) -> "EllrMatrix":
        self = cls()
        row_ptr = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
        val = np.ascontiguousarray(A.val)
        info = L.ellr_plan(A.n_rows, A.n_cols, row_ptr)
        h = dict(rowmax=np.empty(max(info.n_pad, 1), np.int32),
                 col_e=np.empty(max(info.nnz_stored, 1), np.int32),
                 val_e=np.empty(max(info.nnz_stored, 1), val.dtype))
        L.ellr_convert(info, row_ptr, np.ascontiguousarray(A.col, dtype=np.int32), val, h["rowmax"],
                       h["col_e"], h["val_e"])
        self.info = info
        self.dtype = _tdtype(val.dtype)
        self.device = torch.device(device)
        self.d = {k: _to_dev(v, self.device) for k, v in h.items()}
        self.host = {"rowmax": h["rowmax"][:info.n_pad], "col_e": h["col_e"][:info.nnz_stored],
                     "val_e": h["val_e"][:info.nnz_stored]} if keep_host else {}
        return self

    def spmv(self, x, y=None, stream=None):
        if y is None:
            y = torch.empty(self.info.n_rows, dtype=self.dtype, device=self.device)
        L.ellr_spmv(self.info, self.d["rowmax"], self.d["col_e"], self.d["val_e"], x, y, stream)
        return y

    def footprint_bytes(self) -> int:
        vb = 8 if self.dtype == torch.float64 else 4
        return self.info.nnz_stored * (vb + 4) + self.info.n_pad * 4


class CsrMatrix:
    """The input CSR arrays on the GPU, for the CSR kernels."""

    @classmethod
    def from_csr(cls, A, device="cuda") -> "CsrMatrix":
        self = cls()
        self.n_rows, self.n_cols = A.n_rows, A.n_cols
        self.dtype = _tdtype(np.asarray(A.val).dtype)
        self.device = torch.device(device)
        self.row_ptr = _to_dev(np.asarray(A.row_ptr, np.int64), self.device)
        self.col = _to_dev(np.asarray(A.col, np.int32) if len(A.col) else np.zeros(1, np.int32), self.device)
        self.val = _to_dev(np.asarray(A.val) if len(A.val) else np.zeros(1, np.asarray(A.val).dtype), self.device)
        self.nnz = int(A.row_ptr[-1])
        return self

    def spmv(self, x, y=None, variant: int = 1, stream=None):
        if y is None:
            y = torch.empty(self.n_rows, dtype=self.dtype, device=self.device)
        L.csr_spmv(self.n_rows, self.n_cols, self.row_ptr, self.col, self.val, x, y, variant, stream, nnz=self.nnz)
        return y

    def footprint_bytes(self) -> int:
        vb = 8 if self.dtype == torch.float64 else 4
        return self.nnz * (vb + 4) + (self.n_rows + 1) * 8


class PjdsBatch:
    """y_m = A_m x_m for many pJDS matrices in one call (pjds_batch_* of include/pjds.h).

    ``mats`` are PjdsMatrix objects of one block height and layout; ``xs``/``ys`` their
    device vectors.  The object keeps references to everything the handle points at.
    """

    def __init__(self, mats, xs, ys, mode: int = L.PJDS_BATCH_PERSISTENT, y_permuted: bool = False,
                 groups_per_tile: int = 0, x_halo: int | None = None):
        """``x_halo`` (persistent mode only) stages x in LDS per tile (pjds_batch_create_xlds)."""
        self.mats, self.xs, self.ys = list(mats), list(xs), list(ys)
        members = [(M.info, M.d["row_len"], M.d["offsets"], M.d["col_p"], M.d["val_p"], M.d["perm"], x, y)
                   for M, x, y in zip(self.mats, self.xs, self.ys)]
        flags = L.PJDS_Y_PERMUTED if y_permuted else 0
        if x_halo is not None:
            if mode != L.PJDS_BATCH_PERSISTENT:
                raise ValueError("x_halo needs the persistent mode")
            self.handle = L.pjds_batch_create_xlds(members, self.mats[0].dtype, flags, groups_per_tile, x_halo)
        else:
            self.handle = L.pjds_batch_create(members, self.mats[0].dtype, flags, mode, groups_per_tile)

    def launch(self, stream=None) -> None:
        L.pjds_batch_launch(self.handle, stream)

    def info(self) -> tuple[int, int]:
        return L.pjds_batch_info(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            torch.cuda.synchronize()
            L.pjds_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_columns(A, c0: int, c1: int):
    """A = A_local + A_nonlocal with A_local holding the entries whose column lies in [c0, c1)
    (the local/non-local split of a row-distributed product, pjds_split_columns); both keep A's
    row count and the entries' order.  Returns two objects with n_rows, n_cols, row_ptr, col, val."""
    class _Part:
        pass
    rp = np.ascontiguousarray(A.row_ptr, np.int64)
    col = np.ascontiguousarray(A.col, np.int32)
    val = np.ascontiguousarray(A.val)
    loc = L.pjds_split_count(A.n_rows, A.n_cols, rp, col, c0, c1)
    nl = int(rp[A.n_rows]) - loc
    parts = []
    for n in (loc, nl):
        P = _Part()
        P.n_rows, P.n_cols = A.n_rows, A.n_cols
        P.row_ptr = np.empty(A.n_rows + 1, np.int64)
        P.col = np.empty(n, np.int32)
        P.val = np.empty(n, val.dtype)
        parts.append(P)
    L.pjds_split_columns(A.n_rows, A.n_cols, rp, col, val, c0, c1, parts[0].row_ptr, parts[0].col, parts[0].val,
                         parts[1].row_ptr, parts[1].col, parts[1].val)
    return parts[0], parts[1]
