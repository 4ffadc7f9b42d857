"""Reference matrix features of the learned tuner -- TEST INFRASTRUCTURE ONLY.

The same 24 definitions the library implements, written independently with numpy:
 0 log2 N                  1 log2(nnz + 1)            2 mean row length
 3 std (population)        4 skewness                 5 excess kurtosis
 6 min length              7 log2(max + 1)            8 max / mean
 9 empty-row fraction     10-12 p50, p90, p99 / mean (nearest rank)
13 log2((N64 * max + 1) / nnz), ELLPACK-R padding (N64 = rows rounded up to 64)
14 pJDS stored / nnz at block height 64, global sort
15 pJDS stored / nnz at block height 64, sort window 4096
16-18 max, mean, std of |col - row| / max(N, n_cols)      (sampled entries)
19-20 fraction of sampled entries with |col - row| <= 64, <= 4096
21 log(#distinct offsets / #sampled)   22 share of the 16 most used offsets
23 mean over <= 256 evenly spaced 64-row blocks of entries / distinct 16-column segments
Sampling: every s-th entry, s = ceil(nnz / 2^20).
"""
from __future__ import annotations

import numpy as np


def _stored(lens_desc_windows: np.ndarray, window: int) -> float:
    total = 0.0
    n = len(lens_desc_windows)
    for w0 in range(0, n, window):
        w = np.sort(lens_desc_windows[w0:w0 + window])[::-1]
        total += 64.0 * float(w[::64].sum())
    return total


def features(A) -> np.ndarray:
    n, nc = A.n_rows, A.n_cols
    rp = np.asarray(A.row_ptr, np.int64)
    col = np.asarray(A.col, np.int64)
    nnz = int(rp[-1])
    L = np.diff(rp).astype(np.float64)
    f = np.zeros(24)
    mean = nnz / n
    d = L - mean
    m2, m3, m4 = (d ** 2).mean(), (d ** 3).mean(), (d ** 4).mean()
    sd = np.sqrt(m2)
    s = np.sort(L)

    def q(p):
        k = min(n - 1, max(0, int(np.ceil(p * n)) - 1))
        return s[k]
    f[0] = np.log2(n)
    f[1] = np.log2(nnz + 1.0)
    f[2] = mean
    f[3] = sd
    f[4] = m3 / sd ** 3 if sd > 0 else 0.0
    f[5] = m4 / m2 ** 2 - 3.0 if sd > 0 else 0.0
    f[6] = L.min()
    f[7] = np.log2(L.max() + 1.0)
    f[8] = L.max() / mean if mean > 0 else 0.0
    f[9] = (L == 0).mean()
    if mean > 0:
        f[10], f[11], f[12] = q(0.5) / mean, q(0.9) / mean, q(0.99) / mean
    nz = max(nnz, 1)
    n64 = int(np.ceil(n / 64)) * 64
    Lp = np.zeros(n64)
    Lp[:n] = L
    f[13] = np.log2((n64 * L.max() + 1.0) / nz)
    f[14] = _stored(Lp, n64) / nz
    f[15] = _stored(Lp, 4096) / nz
    step = -(-nnz // (1 << 20)) if nnz > (1 << 20) else 1
    k = np.arange(0, nnz, step)
    if len(k):
        rows = np.searchsorted(rp, k, side="right") - 1
        off = col[k] - rows
        a = np.abs(off).astype(np.float64)
        scale = max(n, nc)
        f[16] = a.max() / scale
        f[17] = a.mean() / scale
        f[18] = np.sqrt(max(0.0, (a ** 2).mean() - a.mean() ** 2)) / scale
        f[19] = (a <= 64).mean()
        f[20] = (a <= 4096).mean()
        _, counts = np.unique(off, return_counts=True)
        f[21] = np.log(len(counts) / len(k))
        f[22] = np.sort(counts)[::-1][:16].sum() / len(k)
    blocks = -(-n // 64)
    nb = min(blocks, 256)
    vals = []
    for qq in range(nb):
        b = qq * blocks // nb
        r0, r1 = b * 64, min(n, b * 64 + 64)
        seg = col[rp[r0]:rp[r1]] >> 4
        if len(seg):
            vals.append(len(seg) / len(np.unique(seg)))
    f[23] = np.mean(vals) if vals else 0.0
    return f
