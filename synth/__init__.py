"""Seeded synthetic inputs shared by the library's tests, the benchmark and the oracle.

This module only *draws* inputs: sparse matrices in CSR form and dense vectors.  It holds
none of the arithmetic of the method under test (no sorting by row length, no padding, no
products), so both the GPU path and the CPU oracle may consume what it produces without
sharing any of the method's code.

All randomness comes from one counter-based generator, SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): output k of a stream is
``mix(key + (k + 1) * 0x9E3779B97F4A7C15)`` with the published finaliser ``mix``.  Every
draw is therefore addressable by (seed, stream, index), which makes the generators
vectorisable and reproducible bit for bit on any host.

The matrix families stand in for the paper's test matrices, which are not public:
* ``laplacian_2d``   - 5-point Dirichlet Laplacian (a textbook operator with closed forms);
* ``hh_like``        - banded symmetric pattern with long contiguous off-diagonals, shaped
                       like the Holstein-Hubbard matrix of the paper's test set (Sect. 1.3);
* ``powerlaw``       - heavy-tailed row lengths with uniformly random columns, the
                       skewed-row stress case for sorting and padding;
* ``banded_random``  - row lengths uniform in [lo, hi], columns near the diagonal (the
                       members of the uneven multi-matrix batch);
* ``random_csr``     - small arbitrary CSR matrices (empty rows, duplicates, unsorted
                       columns) for property tests.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "stream_u64", "uniform01", "uniform_pm1", "normal",
    "laplacian_2d", "hh_like", "powerlaw", "banded_random", "random_csr",
    "uneven_batch_sizes", "dense_x", "banded_stratified",
]

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (vectorised, wrapping uint64 arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    """Key of an independent stream: two mixing rounds over (seed, stream)."""
    s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    t = np.array([stream & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return _mix(_mix(s + _GOLDEN) ^ (t * _M2 + _GOLDEN))[0]


def stream_u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+n-1`` of SplitMix64 stream (seed, stream) as uint64."""
    k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(_key(seed, stream) + k * _GOLDEN)


def _u01_from(z: np.ndarray) -> np.ndarray:
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform01(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of each draw times 2^-53."""
    return _u01_from(stream_u64(seed, stream, n, start))


def uniform_pm1(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [-1, 1): 2u - 1 (exact in binary64)."""
    return 2.0 * uniform01(seed, stream, n, start) - 1.0


def normal(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Standard normals by Box-Muller, one normal from each pair of uniforms."""
    u = uniform01(seed, stream, 2 * n, 2 * start)
    u1 = 1.0 - u[0::2]                      # (0, 1]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def _uniform_int(seed: int, stream: int, n: int, lo: int, hi: int, start: int = 0) -> np.ndarray:
    """Integers uniform in [lo, hi] by multiply-shift of the top 32 bits (hi-lo < 2^32)."""
    span = np.uint64(hi - lo + 1)
    z = stream_u64(seed, stream, n, start) >> np.uint64(32)
    with np.errstate(over="ignore"):
        return (lo + ((z * span) >> np.uint64(32)).astype(np.int64)).astype(np.int64)


@dataclass
class CSR:
    """Compressed sparse rows: ``row_ptr`` int64[n_rows+1], ``col`` int32[nnz], ``val`` f64[nnz]."""
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def astype(self, dtype) -> "CSR":
        """Same pattern, values rounded to nearest in ``dtype`` (float32 set of a matrix)."""
        return CSR(self.n_rows, self.n_cols, self.row_ptr, self.col,
                   self.val.astype(dtype), self.name + f"[{np.dtype(dtype).name}]")


def _from_slots(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray, n_cols: int, name: str) -> CSR:
    """Assemble CSR from a dense (n_rows, slots) layout whose slots are in column order."""
    n_rows = cols.shape[0]
    lens = mask.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    return CSR(n_rows, n_cols, row_ptr, cols[mask].astype(np.int32), vals[mask].astype(np.float64), name)


def laplacian_2d(nx: int = 128, ny: int | None = None) -> CSR:
    """5-point Dirichlet Laplacian on an nx-by-ny grid: 4 on the diagonal, -1 per neighbour.

    Node (r, c) is row r*nx + c; its entries are emitted in ascending column order
    (north, west, centre, east, south) where the neighbour exists.
    """
    ny = nx if ny is None else ny
    n = nx * ny
    i = np.arange(n, dtype=np.int64)
    r, c = i // nx, i % nx
    offs = np.array([-nx, -1, 0, 1, nx], dtype=np.int64)
    cols = i[:, None] + offs[None, :]
    mask = np.stack([r > 0, c > 0, np.ones(n, bool), c < nx - 1, r < ny - 1], axis=1)
    vals = np.where(offs[None, :] == 0, 4.0, -1.0) * np.ones((n, 1))
    cols = np.where(mask, cols, 0)
    return _from_slots(cols, vals, mask, n, f"laplacian2d_{nx}x{ny}")


def _distinct_ints(seed: int, stream: int, count: int, lo: int, hi: int) -> np.ndarray:
    """``count`` distinct integers uniform in [lo, hi], drawn in order, repeats skipped."""
    out: list[int] = []
    k = 0
    while len(out) < count:
        v = int(_uniform_int(seed, stream, 1, lo, hi, start=k)[0])
        k += 1
        if v not in out:
            out.append(v)
    return np.array(out, dtype=np.int64)


def hh_like(n: int = 1 << 22, seed: int = 2, p: float = 0.47, band: int = 1000,
            run: int = 15000) -> CSR:
    """Symmetric banded pattern with long contiguous off-diagonals (Holstein-Hubbard-like).

    Each row has the diagonal and offsets +-1, +-2 (where in range).  Four band offsets in
    [3, band] and four off-band offsets in [band+1, n/2] are drawn per matrix.  A band slot
    is present independently per row with probability ``p``; an off-band slot is switched on
    or off for whole runs of ``run`` consecutive rows, giving contiguous off-diagonals.
    Every upper entry (i, i+d) is mirrored to (i+d, i) with the same N(0,1) value, so the
    matrix is symmetric.  Row length is 5 + (sum of 16 Bernoulli(p)) away from the edges.
    """
    assert n >= 8
    band = min(band, max(3, n // 4))
    band_offs = np.sort(_distinct_ints(seed, 1, 4, 3, band))
    far_hi = max(band + 4, n // 2)
    far_offs = np.sort(_distinct_ints(seed, 2, 4, band + 1, far_hi))
    up_offs = np.concatenate([[1, 2], band_offs, far_offs]).astype(np.int64)  # 10 upper slots
    i = np.arange(n, dtype=np.int64)
    pres_up = np.empty((len(up_offs), n), dtype=bool)
    val_up = np.empty((len(up_offs), n), dtype=np.float64)
    for s, d in enumerate(up_offs):
        if s < 2:
            pres = np.ones(n, dtype=bool)
        elif s < 6:
            pres = uniform01(seed, 10 + s, n) < p
        else:
            runs = uniform01(seed, 10 + s, (n + run - 1) // run) < p
            pres = runs[i // run]
        pres &= (i + d) < n
        pres_up[s] = pres
        val_up[s] = normal(seed, 30 + s, n)
    diag_val = normal(seed, 50, n)
    # Slots in ascending column order: lower (largest offset first), diagonal, upper.
    order = np.argsort(up_offs)
    lower = order[::-1]
    nslot = 2 * len(up_offs) + 1
    cols = np.zeros((n, nslot), dtype=np.int64)
    vals = np.zeros((n, nslot), dtype=np.float64)
    mask = np.zeros((n, nslot), dtype=bool)
    k = 0
    for s in lower:
        d = up_offs[s]
        src = i - d
        ok = src >= 0
        m = np.zeros(n, dtype=bool)
        m[ok] = pres_up[s][src[ok]]
        v = np.zeros(n)
        v[ok] = val_up[s][src[ok]]
        cols[:, k] = np.where(m, src, 0)
        vals[:, k] = v
        mask[:, k] = m
        k += 1
    cols[:, k] = i
    vals[:, k] = diag_val
    mask[:, k] = True
    k += 1
    for s in order:
        d = up_offs[s]
        m = pres_up[s]
        cols[:, k] = np.where(m, i + d, 0)
        vals[:, k] = val_up[s]
        mask[:, k] = m
        k += 1
    del pres_up, val_up
    return _from_slots(cols, vals, mask, n, f"hh_like_n{n}_s{seed}")


def _fill_distinct_sorted(seed: int, stream: int, lens: np.ndarray, lo: np.ndarray,
                          width: np.ndarray) -> np.ndarray:
    """Per row, ``lens[r]`` distinct columns uniform in [lo[r], lo[r]+width[r]), sorted.

    Draw all columns, sort each row, and redraw entries that repeat their left neighbour
    (new draws come from later rounds of the same stream) until every row is distinct.
    Requires lens[r] <= width[r].
    """
    n = len(lens)
    nnz = int(lens.sum())
    row = np.repeat(np.arange(n, dtype=np.int64), lens)
    z = stream_u64(seed, stream, nnz) >> np.uint64(32)
    w64 = width[row].astype(np.uint64)
    with np.errstate(over="ignore"):
        col = lo[row] + ((z * w64) >> np.uint64(32)).astype(np.int64)
    key = (row << np.int64(32)) | col
    key.sort()
    rnd = 1
    while True:
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            break
        r = key[dup] >> np.int64(32)
        z = stream_u64(seed, stream + 1000 * rnd, dup.size) >> np.uint64(32)
        with np.errstate(over="ignore"):
            c = lo[r] + ((z * width[r].astype(np.uint64)) >> np.uint64(32)).astype(np.int64)
        key[dup] = (r << np.int64(32)) | c
        rows = np.unique(r)
        # re-sort only the affected rows
        starts = np.concatenate([[0], np.cumsum(lens)])
        for rr in rows:
            a, b = starts[rr], starts[rr + 1]
            key[a:b].sort()
        rnd += 1
    return (key & np.int64(0xFFFFFFFF)).astype(np.int32)


def powerlaw(n: int = 1 << 23, seed: int = 3, alpha: float = 2.2, x_min: float = 2.5784,
             l_max: int = 4096, n_cols: int | None = None) -> CSR:
    """Heavy-tailed row lengths with uniformly random columns.

    L_i = min(l_max, floor(x_min * U^(-1/(alpha-1)))) with U uniform in (0, 1]: a Pareto
    law of density exponent ``alpha``; x_min = 2.5784 gives E[L] close to 12 for alpha 2.2
    and l_max 4096.  Each row holds L_i distinct columns uniform on [0, n_cols), sorted, with
    values uniform in [-1, 1).
    """
    n_cols = n if n_cols is None else n_cols
    u = 1.0 - uniform01(seed, 1, n)
    lens = np.minimum(l_max, np.floor(x_min * u ** (-1.0 / (alpha - 1.0)))).astype(np.int64)
    lens = np.minimum(lens, n_cols)
    lo = np.zeros(n, dtype=np.int64)
    width = np.full(n, n_cols, dtype=np.int64)
    col = _fill_distinct_sorted(seed, 2, lens, lo, width)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    val = uniform_pm1(seed, 3, int(row_ptr[-1]))
    return CSR(n, n_cols, row_ptr, col, val, f"powerlaw_n{n}_s{seed}")


def banded_random(n: int, seed: int, len_lo: int = 3, len_hi: int = 60, halo: int = 4096) -> CSR:
    """Square matrix, row lengths uniform in [len_lo, len_hi], distinct columns uniform in the
    window [i - halo, i + halo] clipped to the matrix, values uniform in [-1, 1)."""
    lens = _uniform_int(seed, 1, n, len_lo, len_hi)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - halo)
    hi = np.minimum(n - 1, i + halo)
    width = hi - lo + 1
    lens = np.minimum(lens, width)
    col = _fill_distinct_sorted(seed, 2, lens, lo, width)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    val = uniform_pm1(seed, 3, int(row_ptr[-1]))
    return CSR(n, n, row_ptr, col, val, f"banded_n{n}_s{seed}")


def banded_stratified(n: int, seed: int, len_lo: int = 3, len_hi: int = 60, halo: int = 4096) -> CSR:
    """Square matrix, row lengths uniform in [len_lo, len_hi], values uniform in [-1, 1).

    Row i's columns are spread over the window [i - halo, i + halo] clipped to the matrix:
    the window is cut into L_i equal strata and column j is uniform within stratum j, so
    columns are distinct and ascending by construction (stratified uniform sampling).
    ``synth.torchgen.banded_stratified`` computes the same arrays bit for bit with torch.
    """
    lens = _uniform_int(seed, 1, n, len_lo, len_hi)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - halo)
    width = np.minimum(n - 1, i + halo) - lo + 1
    lens = np.minimum(lens, width)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    row = np.repeat(i, lens)
    j = np.arange(nnz, dtype=np.int64) - row_ptr[row]
    L = lens[row]
    w = width[row]
    # stratum j covers [floor(j*w/L), floor((j+1)*w/L)); pick uniformly inside it
    s0 = (j * w) // L
    s1 = ((j + 1) * w) // L
    z = stream_u64(seed, 2, nnz) >> np.uint64(32)
    with np.errstate(over="ignore"):
        off = ((z * (s1 - s0).astype(np.uint64)) >> np.uint64(32)).astype(np.int64)
    col = (lo[row] + s0 + off).astype(np.int32)
    val = uniform_pm1(seed, 3, nnz)
    return CSR(n, n, row_ptr, col, val, f"stratified_n{n}_s{seed}")


def uneven_batch_sizes(count: int = 512, lo: int = 1000, hi: int = 500_000, seed: int = 999) -> np.ndarray:
    """Row counts log-uniform in [lo, hi]: round(exp(U[ln lo, ln hi]))."""
    u = uniform01(seed, 1, count)
    return np.rint(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.int64)


def random_csr(n_rows: int, n_cols: int, seed: int, max_len: int = 8, empty_frac: float = 0.2,
               sorted_cols: bool = False, allow_dup: bool = True, integer: bool = False) -> CSR:
    """Small arbitrary CSR for property tests: some empty rows, optional duplicate and
    unsorted column indices, values uniform in [-1, 1) or small integers."""
    lens = _uniform_int(seed, 1, n_rows, 0, max_len) if n_rows else np.zeros(0, np.int64)
    if n_rows:
        lens[uniform01(seed, 2, n_rows) < empty_frac] = 0
    if n_cols == 0:
        lens[:] = 0
    nnz = int(lens.sum())
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    col = _uniform_int(seed, 3, nnz, 0, max(n_cols - 1, 0)).astype(np.int32) if nnz else np.zeros(0, np.int32)
    if not allow_dup and nnz:
        col = np.concatenate([
            np.sort(_distinct_ints(seed, 100 + r, int(lens[r]), 0, n_cols - 1)) if lens[r] else np.zeros(0, np.int64)
            for r in range(n_rows)]).astype(np.int32)
    if sorted_cols and nnz:
        for r in range(n_rows):
            a, b = row_ptr[r], row_ptr[r + 1]
            col[a:b] = np.sort(col[a:b])
    if integer:
        val = _uniform_int(seed, 4, nnz, -4, 4).astype(np.float64)
    else:
        val = uniform_pm1(seed, 4, nnz)
    return CSR(n_rows, n_cols, row_ptr, col, val, f"random_{n_rows}x{n_cols}_s{seed}")


def dense_x(n: int, seed: int = 1, k: int = 1, integer: bool = False) -> np.ndarray:
    """Dense input: uniform in [-1, 1) (or integers in [-3, 3]); shape (n,) or (n, k)
    row-major, i.e. interleaved X[c*k + v]."""
    if integer:
        x = _uniform_int(seed, 7, n * k, -3, 3).astype(np.float64)
    else:
        x = uniform_pm1(seed, 7, n * k)
    return x if k == 1 else x.reshape(n, k)
