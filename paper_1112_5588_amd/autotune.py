"""Exhaustive autotuner over kernel configurations for y = A x.

For a matrix it converts once per distinct storage (format, block height, sort window,
layout, long-row split), times every catalog entry that uses it (median of `reps`
launches, each bracketed by HIP events on the launch stream, after `warmup` launches), and
returns the fastest.  It is the reference the learned tuner is compared with (regret 0 by
definition) and its fallback.

Results can be appended to a JSON-lines store keyed by (matrix key, configuration,
device), so a long sweep resumes where it stopped.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .matrix import CsrMatrix, EllrMatrix, PjdsMatrix


@dataclass(frozen=True)
class Config:
    name: str
    fmt: str                    # "pjds", "ellr" or "csr"
    block_height: int = 64
    layout: str = "jd"
    sort_window: int = 0
    split_len: int = 0
    xcd_remap: bool = False
    variant: int = 1            # CSR lanes per row
    x_halo: int = -1            # >= 0: x staged in LDS (pjds_spmv_xlds) with this halo
    tile_rows: int = 0          # rows per workgroup of the LDS path
    two_rows: bool = False      # two adjacent rows per lane (PJDS_TWO_ROWS)
    lanes: int = 1              # lanes per sorted row (PJDS_LANES; block height 64 / lanes)

    def storage_key(self):
        if self.fmt == "pjds":
            return ("pjds", self.block_height, self.layout, self.sort_window, self.split_len, self.lanes)
        return (self.fmt,)


# Index 0 is the untuned default: the paper's format with a block height of one wavefront,
# global sort, jagged-diagonal layout, x through the caches.
CATALOG: tuple[Config, ...] = (
    Config("pjds_b64_jd", "pjds", 64, "jd"),
    Config("pjds_b32_jd", "pjds", 32, "jd"),
    Config("pjds_b128_jd", "pjds", 128, "jd"),
    Config("pjds_b64_jd_xcd", "pjds", 64, "jd", xcd_remap=True),
    Config("pjds_b64_w256", "pjds", 64, "block", 256),
    Config("pjds_b64_w1024", "pjds", 64, "block", 1024),
    Config("pjds_b64_w4096", "pjds", 64, "block", 4096),
    Config("pjds_b64_w16384", "pjds", 64, "block", 16384),
    Config("pjds_b64_w65536", "pjds", 64, "block", 65536),
    Config("pjds_b64_w4096_xcd", "pjds", 64, "block", 4096, xcd_remap=True),
    Config("pjds_b64_w65536_xcd", "pjds", 64, "block", 65536, xcd_remap=True),
    Config("ellr", "ellr"),
    Config("csr_v1", "csr", variant=1),
    Config("csr_v4", "csr", variant=4),
    Config("csr_v16", "csr", variant=16),
    Config("pjds_b64_w256_lds512", "pjds", 64, "block", 256, x_halo=512, tile_rows=512),
    Config("pjds_b64_w512_lds512", "pjds", 64, "block", 512, x_halo=512, tile_rows=512),
    Config("pjds_b64_w256_nosplit_2r", "pjds", 64, "block", 256, split_len=-1, two_rows=True),
    Config("pjds_b64_w256_lds768_t1024_2r", "pjds", 64, "block", 256, x_halo=768, tile_rows=1024, two_rows=True),
    Config("pjds_b64_w512_lds768_t1024_2r", "pjds", 64, "block", 512, x_halo=768, tile_rows=1024, two_rows=True),
    # the heavy-tail entries: T lanes per sorted row (global sort, block height 64 / T), and
    # long rows cut every 512 entries instead of the default 128
    Config("pjds_T2_global", "pjds", 32, "block", lanes=2),
    Config("pjds_T4_global", "pjds", 16, "block", lanes=4),
    Config("pjds_b64_jd_split512", "pjds", 64, "jd", split_len=512),
)
# A record's times count for training and evaluation only if they were all taken with the
# current timing (time_median: launches replayed from a graph, the host taken out) on the
# current kernels, which the record marks with "times_rev" >= TIMES_REV; older records'
# times are masked.  REVISED lists the entries whose kernels changed since the first sweep;
# revision 4 re-timed the plain two-rows entry after its groups of steps were pipelined (the
# other entries' kernels were unchanged, so their revision-3 times stand).
REVISED = ("pjds_b64_w256_lds512", "pjds_b64_w512_lds512", "pjds_b64_w256_lds768_t1024_2r",
           "pjds_b64_w512_lds768_t1024_2r", "pjds_b64_w256_nosplit_2r")
TIMES_REV = 4
CONFIG_NAMES = tuple(c.name for c in CATALOG)
DEFAULT = 0

# ELLPACK-R is skipped when its padded storage would exceed this many bytes
ELLR_LIMIT_BYTES = 24 * 2 ** 30


def device_name() -> str:
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def time_median(fn, reps: int = 7, warmup: int = 2, graph: bool = True) -> float:
    """Median milliseconds of one launch of `fn`, with the host taken out of the timing: after
    `warmup` eager calls (which also make anything a first call creates), `batch` calls are
    captured in a HIP graph and the graph is replayed `reps` times between two events on the
    stream; a replay's time over `batch` is one sample.  `batch` is sized from one eager call
    so a replay runs about 2 ms (at most 32 calls).  Launched one by one from Python, a product
    of a few microseconds would be timed as the binding's own overhead.  graph=False times
    single eager calls (for a call that launches a graph of its own)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if not graph:
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    fn()
    s1.record()
    torch.cuda.synchronize()
    batch = int(min(32, max(1, 2.0 // max(s0.elapsed_time(s1), 1e-3))))
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            for _ in range(batch):
                fn()
    torch.cuda.current_stream().wait_stream(cs)
    g.replay()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        g.replay()
        b.record()
    torch.cuda.synchronize()
    del g
    return float(np.median([a.elapsed_time(b) / batch for a, b in ev]))


def _build(A, cfg: Config, device):
    if cfg.fmt == "pjds":
        return PjdsMatrix.from_csr(A, block_height=cfg.block_height, layout=cfg.layout,
                                   sort_window=cfg.sort_window if cfg.sort_window < A.n_rows else 0,
                                   split_len=cfg.split_len, device=device, lanes=cfg.lanes)
    if cfg.fmt == "ellr":
        info = EllrMatrix.plan(A)
        vb = np.asarray(A.val).dtype.itemsize
        if info.nnz_stored * (vb + 4) > ELLR_LIMIT_BYTES:
            return None
        return EllrMatrix.from_csr(A, device=device)
    return CsrMatrix.from_csr(A, device=device)


def _lds_fits(obj, cfg: Config) -> bool:
    """Whether the LDS path takes this matrix: a sort window (not a global sort) that is a
    multiple of 256, and the staged x range within 64 KiB."""
    w, n = obj.info.sort_window, obj.info.n_rows
    esz = 8 if obj.dtype == torch.float64 else 4
    return w < n and w % 256 == 0 and min(max(cfg.tile_rows, w) + 2 * cfg.x_halo, obj.info.n_cols) * esz <= 65536


def _runner(obj, cfg: Config, x, y):
    if cfg.fmt == "pjds" and cfg.x_halo >= 0:
        if not _lds_fits(obj, cfg):
            return None
        return lambda: obj.spmv_xlds(x, y, x_halo=cfg.x_halo, tile_rows=cfg.tile_rows, y_permuted=True,
                                     xcd_remap=cfg.xcd_remap, two_rows=cfg.two_rows)
    if cfg.fmt == "pjds" and cfg.two_rows:
        # a global sort, or windows that are whole 128-row groups, and no long-row work items
        w, n = obj.info.sort_window, obj.info.n_rows
        if obj.info.n_chunks or (w < n and w % 128):
            return None
        return lambda: obj.spmv(x, y, y_permuted=True, xcd_remap=cfg.xcd_remap, two_rows=True)
    if cfg.fmt == "pjds":
        return lambda: obj.spmv(x, y, y_permuted=True, xcd_remap=cfg.xcd_remap)
    if cfg.fmt == "ellr":
        return lambda: obj.spmv(x, y)
    return lambda: obj.spmv(x, y, variant=cfg.variant)


def runnable_mask(n_rows: int, n_cols: int, value_bytes: int, ellr_fits: bool) -> np.ndarray:
    """Which catalog configurations can run on a matrix of this shape, known without converting
    or timing anything (the conditions _runner and _build apply): x staged in LDS needs a sort
    window below n_rows that is a multiple of 256 and a staged range within 64 KiB; two rows
    per lane without split needs windows of whole 128-row groups; ELLPACK-R its storage under
    the size limit."""
    ok = np.ones(len(CATALOG), dtype=bool)
    for c, cfg in enumerate(CATALOG):
        w = cfg.sort_window if cfg.sort_window < n_rows else 0
        if cfg.fmt == "pjds" and cfg.x_halo >= 0:
            ok[c] = 0 < w and w % 256 == 0 and min(max(cfg.tile_rows, w) + 2 * cfg.x_halo, n_cols) * value_bytes <= 65536
        elif cfg.fmt == "pjds" and cfg.two_rows:
            ok[c] = cfg.split_len < 0 and (w == 0 or w % 128 == 0)
        elif cfg.fmt == "ellr":
            ok[c] = bool(ellr_fits)
    return ok


def time_all(A, x: torch.Tensor | None = None, configs=CATALOG, reps: int = 7, warmup: int = 2,
             device="cuda") -> dict[str, float]:
    """Median ms of y = A x for every configuration (inf where a format is not built)."""
    dt = torch.float64 if np.asarray(A.val).dtype == np.float64 else torch.float32
    if x is None:
        import synth
        x = torch.from_numpy(synth.dense_x(A.n_cols, 1)).to(device, dt)
    y = torch.empty(A.n_rows, dtype=dt, device=device)
    out: dict[str, float] = {}
    groups: dict[tuple, list[Config]] = {}
    for c in configs:
        groups.setdefault(c.storage_key(), []).append(c)
    for _, cfgs in groups.items():
        obj = _build(A, cfgs[0], device)
        for c in cfgs:
            run = None if obj is None else _runner(obj, c, x, y)
            out[c.name] = float("inf") if run is None else time_median(run, reps, warmup)
        del obj
    return out


@dataclass
class TuneResult:
    best: Config
    times_ms: dict[str, float] = field(default_factory=dict)

    @property
    def speedup_over_default(self) -> float:
        return self.times_ms[CATALOG[DEFAULT].name] / self.times_ms[self.best.name]


def autotune(A, **kw) -> TuneResult:
    """Exhaustive search: the fastest catalog configuration for A."""
    t = time_all(A, **kw)
    best = min(CATALOG, key=lambda c: t[c.name])
    return TuneResult(best, t)


class ResultStore:
    """Append-only JSON-lines store of sweep records, one per (key, device)."""

    def __init__(self, path: str):
        self.path = path
        self.records: dict[tuple[str, str], dict] = {}
        if os.path.exists(path):
            with open(path) as f:
                for line in f:
                    line = line.strip()
                    if line:
                        r = json.loads(line)
                        self.records[(r["key"], r["device"])] = r

    def has(self, key: str, device: str) -> bool:
        return (key, device) in self.records

    def add(self, record: dict) -> None:
        self.records[(record["key"], record["device"])] = record
        with open(self.path, "a") as f:
            f.write(json.dumps(record) + "\n")

    def rewrite(self) -> None:
        """Rewrite the file with one line per record (later lines of a key replace earlier)."""
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            for r in self.records.values():
                f.write(json.dumps(r) + "\n")
        os.replace(tmp, self.path)


def tune_spmmv(M: PjdsMatrix, k: int, reps: int = 5) -> tuple[tuple[int, int, bool], dict[tuple[int, int, bool], float]]:
    """(vectors per tile, vectors per lane, XCD renumbering) for k right-hand sides: the fastest
    combination with a tile of at most 2k vectors.  Renumbering helps SpMMV more than the
    single product because each XCD's L2 then keeps the rows of X that neighbouring rows share."""
    import synth
    X = torch.from_numpy(synth.dense_x(M.n_cols, 4, k=k).reshape(M.n_cols, k)).to(M.device, M.dtype)
    Y = torch.empty((M.n_rows, k), dtype=M.dtype, device=M.device)
    t_ms = {}
    for vpl in (1, 2, 4):
        if k % vpl:
            continue
        for lpr in (1, 2, 4, 8, 16, 32):
            t = lpr * vpl
            if t > 1 and t // 2 >= k:
                continue
            for remap in (False, True):
                t_ms[(t, vpl, remap)] = time_median(
                    lambda: M.spmmv(X, Y, vectors_per_tile=t, vectors_per_lane=vpl, y_permuted=True,
                                    xcd_remap=remap), reps, 1)
    return min(t_ms, key=t_ms.get), t_ms


def tune_batch(mats, xs, ys, groups=(1, 4, 8, 32), reps: int = 5) -> tuple[int, dict[int, float]]:
    """Tile size (wave groups per tile) of the persistent batch launch."""
    from .matrix import PjdsBatch
    t_ms = {}
    for g in groups:
        B = PjdsBatch(mats, xs, ys, mode=L.PJDS_BATCH_PERSISTENT, y_permuted=True, groups_per_tile=g)
        t_ms[g] = time_median(B.launch, reps, 1, graph=False)    # the launch is a graph already
        B.close()
    return min(t_ms, key=t_ms.get), t_ms
