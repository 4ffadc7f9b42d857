#!/usr/bin/env python3
"""Benchmark: pJDS sparse matrix-vector product on one MI355X.

Default workload: the Holstein-Hubbard-like matrix (N = 2^22 rows, banded symmetric pattern
with contiguous off-diagonals, row lengths 5..20, N(0,1) values), FP64.  Default kernel
configuration: the tuned pJDS form -- block height 64, rows sorted inside windows of 512
(per-block layout), x staged in LDS per 1024-row tile with a halo of 768, two adjacent rows
per lane, one-byte row lengths, y written in the permuted basis (Listing 2).  The paper's plain configuration (global
sort, jagged-diagonal layout) is timed beside it in `extra.autotune`.

One step is one product y = A x with the matrix and x already resident in HBM, run from a
cold Infinity Cache: each step first streams 1 GiB of another buffer through the caches with
ordinary loads (a read-only pass: it evicts the 256 MB cache and leaves nothing dirty), then
runs the product between two HIP events on the product's stream.  `value` is the median over
the timed steps of the algorithmic bytes of the product -- 12 B per non-zero (value + column
index) plus 8 B per row for x and 8 B per row for y -- divided by the product's time;
`roofline.achieved` the same bytes over the mean product time.  `warm` times the same product
back to back (caches warm) for comparison.

Every timed leg is checked against the oracle before the line is printed (the whole vector
of the headline product, sampled rows of the others); a leg outside its tolerance (1e-12
relative in binary64, 1e-5 in binary32) nulls `value`, names the leg in `error` and makes the
exit status 1.

    python bench.py [--steps K] [--warmup W] [--workload hh_like|laplacian|powerlaw]
                    [--dtype f64|f32] [--sort-window W] [--x-halo H] [--tile-rows T] [--one-row]
                    [--lanes T] [--xcd-remap] [--no-cpu] [--no-extra] [--no-batch]

Besides the headline line's own fields, `extra` holds the comparison legs (ELLPACK-R, CSR,
SpMMV with X through the caches or staged in LDS, the 128 x 128 Laplacian's SpMMV against
single products, the exhaustive and learned tuners, Lanczos steps, the host-link model, lanes
per row, the local/non-local split, FP32 and the power-law matrix) and `batch` the 512-matrix
leg (persistent kernel with x through the caches or staged in LDS, per-member graph, direct
launches).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FLUSH_DOUBLES = 1 << 27        # 1 GiB read-only pass before each cold product
TOL = {"f64": 1e-12, "f32": 1e-5}
# every source the headline kernel is compiled from: a counter record taken on other sources
# is not reported
KERNEL_SOURCES = ("paper_1112_5588_amd/csrc/spmv.hip", "paper_1112_5588_amd/csrc/device.h",
                  "paper_1112_5588_amd/csrc/launch.h", "paper_1112_5588_amd/csrc/common.h", "include/pjds.h")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(rel.encode())
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload_key: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it was taken
    on the kernel sources that are built now; otherwise None."""
    p = os.path.join(ROOT, "profiles", "pjds_spmv_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    e = d.get(workload_key)
    if not e or e.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    return e.get("traffic_bytes_per_launch")


def make_workload(name: str, dtype: str):
    import synth
    if name == "hh_like":
        A = synth.hh_like(1 << 22, seed=2)
        desc = "hh_like: Holstein-Hubbard-like symmetric banded matrix, N=4194304, band |d|<=1000 + 4 contiguous off-diagonals (runs of 15000 rows), row lengths 5..20, N(0,1) values, seed 2"
    elif name == "laplacian":
        A = synth.laplacian_2d(128)
        desc = "laplacian: 2D 5-point Dirichlet Laplacian on a 128x128 grid, N=16384"
    elif name == "powerlaw":
        A = synth.powerlaw(1 << 23, seed=3)
        desc = "powerlaw: N=8388608, power-law row lengths (alpha 2.2, mean ~12, max 4096), uniform random columns, U[-1,1) values, seed 3"
    else:
        raise SystemExit(f"unknown workload {name}")
    if dtype == "f32":
        A = A.astype(np.float32)
    return A, desc


def time_launches(fn, steps: int, warmup: int):
    """Average ms per call of `fn` over `steps` back-to-back calls, bracketed by events on the
    stream the kernels are launched on (torch's current stream): caches warm."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


class ColdTimer:
    """Products timed from a cold Infinity Cache: before each one, a read-only pass over 1 GiB
    of another buffer with cached loads (probe mode 2) evicts the caches without leaving dirty
    lines behind.  Each call is timed twice on its stream: by the library's kernel timing hook
    (pjds_time_next_launch: HIP events recorded by the main kernel's own dispatch, the
    kernel's duration as a kernel trace gives it) and by HIP events recorded before and after
    the call (which add the stream's gaps around the dispatch).  `times` returns the kernel's
    own durations when the call's main kernel took the hook, else the bracketing events';
    `last_kind` says which, `last_bracket` holds the bracketing events' times either way."""

    def __init__(self, torch, lib):
        self.torch, self.lib = torch, lib
        self.buf = torch.ones(FLUSH_DOUBLES, dtype=torch.float64, device="cuda")
        self.out = torch.empty(2048, dtype=torch.float64, device="cuda")
        self.last_kind, self.last_bracket = None, []

    def flush(self) -> None:
        self.lib.pjds_probe(2, self.buf, self.out, FLUSH_DOUBLES)

    def times(self, fn, reps: int, warmup: int = 3, hook: bool = True) -> list:
        """`hook`: False for a call that launches several kernels (it is timed by the
        bracketing events only)."""
        torch, lib = self.torch, self.lib
        for _ in range(warmup):
            self.flush()
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        kt = [lib.KernelTimer() for _ in range(reps)]
        for (s0, s1), k in zip(ev, kt):
            self.flush()
            s0.record()
            if hook:
                k.arm()
            fn()
            k.disarm()
            s1.record()
        torch.cuda.synchronize()
        self.last_bracket = [s0.elapsed_time(s1) for s0, s1 in ev]
        own = [k.ms() for k in kt] if hook else [None]
        if all(t is not None for t in own):
            self.last_kind = "kernel"
            return own
        self.last_kind = "bracket"
        return self.last_bracket

    def median(self, fn, reps: int = 20, warmup: int = 3, hook: bool = True) -> float:
        return float(np.median(self.times(fn, reps, warmup, hook)))


def sample_rows(n: int, seed: int, count: int = 4096) -> np.ndarray:
    """First and last 256 rows plus `count` seeded random rows."""
    import synth
    r = (synth.uniform01(seed, 1, count) * n).astype(np.int64)
    return np.unique(np.concatenate([np.arange(min(256, n)), np.arange(max(0, n - 256), n), r]))


def rel_err(y: np.ndarray, ref: np.ndarray) -> float:
    """||y - ref|| / ||ref|| in binary64 (absolute when ref is zero)."""
    d = float(np.linalg.norm(np.asarray(y, np.float64) - np.asarray(ref, np.float64)))
    r = float(np.linalg.norm(np.asarray(ref, np.float64)))
    return d / r if r > 0 else d


def rows_in_original_order(torch, y_dev, rows: np.ndarray, perm_dev=None) -> np.ndarray:
    """y's values for original rows `rows` (y in the permuted basis when perm_dev is given:
    slot i holds original row perm[i])."""
    torch.cuda.synchronize()
    if perm_dev is None:
        return y_dev.double()[torch.from_numpy(rows).to(y_dev.device)].cpu().numpy()
    inv = torch.empty_like(perm_dev)
    inv[perm_dev.long()] = torch.arange(perm_dev.numel(), dtype=perm_dev.dtype, device=perm_dev.device)
    return y_dev.double()[inv[torch.from_numpy(rows).to(y_dev.device)].long()].cpu().numpy()


# ---- the CPU leg: the oracle timed on this host, and the reference values of the checks ----

def cpu_baseline_leg(A, x, b_alg: float, budget_s: float = 10.0):
    """The oracle timed on this host's cores.  Its serial CSR product (the plain definition the
    parity tests compare against) on one core: the median over full products within a budget
    of about `budget_s` seconds, after 2 warm-ups.  Its all-core form (the same per-row sums,
    bitwise the same result, rows shared among OpenMP threads): the median of 20 after 2
    warm-ups.  Returns the serial result, the reference of the headline check."""
    import oracle
    t0 = time.perf_counter()
    y = oracle.csr_spmv(A, x)
    oracle.csr_spmv(A, x)
    one = max((time.perf_counter() - t0) / 2, 1e-4)
    reps = max(5, min(500, int(budget_s / one)))
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.csr_spmv(A, x)
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    yt = np.empty_like(y)
    for _ in range(2):
        _, used = oracle.csr_spmv_threads(A, x, yt)
    tt = []
    for _ in range(20):
        t0 = time.perf_counter()
        _, used = oracle.csr_spmv_threads(A, x, yt)
        tt.append(time.perf_counter() - t0)
    dtt = float(np.median(tt))
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    rec = {"value": round(b_alg / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": f"full matrix, median of {reps} serial CSR products (binary64, no FMA) after 2 warm-ups, {sum(ts):.1f} s",
           "gflops": round(2 * A.nnz / dt / 1e9, 3), "ms_per_product": round(dt * 1e3, 3),
           "all_cores": {"value": round(b_alg / dtt / 1e9, 3), "unit": "GB/s", "cores": int(used),
                         "nproc": os.cpu_count(), "affinity": affinity,
                         "sample": "full matrix, median of 20 products after 2 warm-ups, rows shared among OpenMP threads (bitwise the serial result)",
                         "gflops": round(2 * A.nnz / dtt / 1e9, 3), "ms_per_product": round(dtt * 1e3, 3),
                         "bitwise_equal_to_serial": bool(np.array_equal(yt, y))}}
    return y, rec


def reference_rows(A, x, rows: np.ndarray) -> np.ndarray:
    """The oracle's values of (A x) at original rows `rows` (X with k columns: (len(rows), k))."""
    import oracle
    rows = np.asarray(rows, np.int64)
    rp = np.asarray(A.row_ptr, np.int64)
    lens = rp[rows + 1] - rp[rows]
    new_rp = np.zeros(len(rows) + 1, np.int64)
    new_rp[1:] = np.cumsum(lens)
    idx = np.repeat(rp[rows] - new_rp[:-1], lens) + np.arange(int(new_rp[-1]), dtype=np.int64)

    class _S:
        pass
    S = _S()
    S.n_rows, S.n_cols, S.row_ptr, S.col, S.val = len(rows), A.n_cols, new_rp, np.asarray(A.col)[idx], np.asarray(A.val)[idx]
    S.nnz = int(new_rp[-1])
    if np.ndim(x) == 2:
        return oracle.csr_spmmv(S, x)
    return oracle.csr_spmv(S, x)


def batch_leg(torch, checks: dict) -> dict:
    """512 uneven matrices (rows log-uniform in [1e3, 5e5], 3..60 entries per row, columns
    within +-4096 of the diagonal), FP64: one persistent launch in a HIP graph (x through the
    caches, or staged in LDS per tile with a 4096-value halo) vs one launch per member captured
    in a graph vs one launch per member issued directly; members stored with a global sort (JD
    layout) and with a 256-row sort window (block layout)."""
    import synth
    from synth import torchgen
    from paper_1112_5588_amd import PjdsBatch, PjdsMatrix, _lib
    sizes = synth.uneven_batch_sizes(512)
    out = {"workload": "512 matrices, rows log-uniform in [1e3, 5e5], 3..60 entries per row within +-4096 of the diagonal, U[-1,1) FP64, seeds 1000+m"}
    for label, kw in (("global_sort", dict(layout="jd")), ("window256", dict(layout="block", sort_window=256))):
        log(f"batch ({label}): generating and converting 512 matrices")
        t0 = time.perf_counter()
        mats, xs, ys = [], [], []
        for m, n in enumerate(sizes):
            rp, col, val = torchgen.banded_stratified(int(n), 1000 + m, device="cuda")
            mats.append(PjdsMatrix.from_arrays(int(n), int(n), rp, col, val, split_len=-1,
                                               **(kw if kw.get("sort_window", 0) < n else dict(layout=kw["layout"]))))
            xs.append(torchgen.dense_x(int(n), 1000 + m, device="cuda"))
            ys.append(torch.empty(int(n), dtype=torch.float64, device="cuda"))
            del rp, col, val
        t_setup = time.perf_counter() - t0
        nnz = sum(M.info.nnz for M in mats)
        rows = int(sizes.sum())
        b_alg = 12 * nnz + 16 * rows
        res = {"setup_s": round(t_setup, 1), "nnz_stored": sum(M.info.nnz_stored for M in mats)}
        out["rows"], out["nnz"] = rows, nnz
        # two members against the oracle after every launch form (the numpy generator gives the
        # same bits as the torch one)
        refs = {}
        for m in (int(np.argmin(sizes)), int(np.argmax(sizes))):
            Am = synth.banded_stratified(int(sizes[m]), 1000 + m)
            refs[m] = reference_rows(Am, synth.dense_x(Am.n_cols, 1000 + m), np.arange(Am.n_rows))
        for name, mode, halo in (("persistent_graph", _lib.PJDS_BATCH_PERSISTENT, None),
                                 ("persistent_graph_x_in_lds", _lib.PJDS_BATCH_PERSISTENT, 4096),
                                 ("per_member_graph", _lib.PJDS_BATCH_GRAPH, None),
                                 ("direct_launches", _lib.PJDS_BATCH_DIRECT, None)):
            for y in ys:
                y.fill_(float("nan"))
            B = PjdsBatch(mats, xs, ys, mode=mode, y_permuted=True, x_halo=halo)
            ms = time_launches(B.launch, 10, 2)
            for m, ref in refs.items():
                checks[f"batch_{label}_{name}_m{m}"] = rel_err(
                    rows_in_original_order(torch, ys[m], np.arange(len(ref)), mats[m].d["perm"]), ref)
            res[name] = {"ms": round(ms, 4), "gflops": round(2 * nnz / ms / 1e6, 1), "GBps_alg": round(b_alg / ms / 1e6, 1)}
            if mode == _lib.PJDS_BATCH_PERSISTENT:
                res[name]["tiles"], res[name]["grid"] = B.info()
            B.close()
        out[label] = res
        del mats, xs, ys
        torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="hh_like", choices=["hh_like", "laplacian", "powerlaw"])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--block-height", type=int, default=64)
    ap.add_argument("--layout", default="block", choices=["jd", "block"])
    ap.add_argument("--mode", default="y_permuted", choices=["y_permuted", "scatter", "symmetric"])
    ap.add_argument("--split-len", type=int, default=0)
    ap.add_argument("--sort-window", type=int, default=512, help="0 = global sort")
    ap.add_argument("--xcd-remap", action="store_true")
    ap.add_argument("--x-halo", type=int, default=768,
                    help=">= 0: stage x in LDS with this halo (block layout, window % 256 == 0); -1: x through the caches")
    ap.add_argument("--tile-rows", type=int, default=1024, help="rows per workgroup of the LDS path")
    ap.add_argument("--one-row", dest="two_rows", action="store_false",
                    help="LDS path: one row per lane (default: two adjacent rows per lane, 2-wide loads)")
    ap.add_argument("--lanes", type=int, default=1,
                    help="lanes per row (power of two up to 64, block layout, x through the caches)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline timing (the checks still run)")
    ap.add_argument("--no-extra", action="store_true", help="skip comparison legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-matrix batch leg")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the paper's multi-GPU path is "
                                   "not built here (one GPU per process); run with --gpus 1"}))
        return 2

    import torch
    import synth
    from paper_1112_5588_amd import CsrMatrix, EllrMatrix, PjdsMatrix, _lib

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 2
    if args.lanes > 1 and (args.x_halo >= 0 or args.layout != "block"):
        print(json.dumps({"error": "--lanes > 1 needs --layout block and --x-halo -1"}))
        return 2
    _lib.lib()   # fail loudly if the HIP library is not built

    log(f"generating workload {args.workload} ({args.dtype})")
    t0 = time.perf_counter()
    A, desc = make_workload(args.workload, args.dtype)
    t_gen = time.perf_counter() - t0
    n, nnz = A.n_rows, A.nnz
    x_np = synth.dense_x(A.n_cols, 1)
    if args.dtype == "f32":
        x_np = x_np.astype(np.float32).astype(np.float64)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    vbytes = 8 if args.dtype == "f64" else 4
    tol = TOL[args.dtype]

    log(f"N={n} nnz={nnz} generated in {t_gen:.1f}s; converting")
    t0 = time.perf_counter()
    M = PjdsMatrix.from_csr(A, block_height=args.block_height, layout=args.layout,
                            sort_window=args.sort_window, symmetric=args.mode == "symmetric",
                            split_len=args.split_len, keep_host=args.mode == "symmetric", lanes=args.lanes)
    t_conv = time.perf_counter() - t0
    perm = M.d["perm"]
    x_dev = torch.from_numpy(x_np).to("cuda", tdt)
    if args.mode == "symmetric":
        x_dev = x_dev[perm.long()].contiguous()
    y_dev = torch.empty(n, dtype=tdt, device="cuda")
    y_perm = args.mode in ("y_permuted", "symmetric")

    def product(x, y):
        if args.x_halo >= 0:
            M.spmv_xlds(x, y, x_halo=args.x_halo, tile_rows=args.tile_rows, y_permuted=y_perm,
                        xcd_remap=args.xcd_remap, two_rows=args.two_rows)
        else:
            M.spmv(x, y, y_permuted=y_perm, xcd_remap=args.xcd_remap)

    def step():
        product(x_dev, y_dev)

    # algorithmic bytes: value + index per non-zero, x once, y once (write)
    b_alg = (vbytes + 4) * nnz + 2 * vbytes * n
    if args.mode == "scatter":
        b_alg += 4 * n               # the permutation read to scatter y

    # ---- the timed region: W warm-up steps, then K steps, each a cold product
    cold = ColdTimer(torch, _lib)
    log(f"timing {args.steps} cold steps after {args.warmup} warm-ups")
    for _ in range(args.warmup):
        cold.flush()
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    kt = [_lib.KernelTimer() for _ in range(args.steps)]
    t_wall = time.perf_counter()
    for (s0, s1), k in zip(ev, kt):
        cold.flush()
        s0.record()
        k.arm()
        step()
        k.disarm()
        s1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    # the step is one kernel: its own duration from the timing hook's events; the events
    # recorded around the call, which add the stream's gaps around the dispatch, beside it
    ms_bracket = [s0.elapsed_time(s1) for s0, s1 in ev]
    ms_steps = [k.ms() for k in kt]
    if any(t is None for t in ms_steps):
        raise RuntimeError("the product kernel did not record the timing hook's events")
    ms = float(np.median(ms_steps))
    ms_mean = float(np.mean(ms_steps))
    gbs = b_alg / (ms * 1e-3) / 1e9
    gbs_mean = b_alg / (ms_mean * 1e-3) / 1e9
    gflops = 2 * nnz / (ms * 1e-3) / 1e9
    # the same product back to back, caches warm
    ms_warm = time_launches(step, 200, 20)

    # ---- checks: the headline against the oracle (whole vector), the CPU baseline
    out: dict = {}
    checks: dict = {}
    tol_of: dict = {}                   # legs computed in another precision than the headline
    cpu = None
    y = y_dev.double().cpu().numpy()
    if args.mode == "symmetric":
        ref_idx = M.host["perm"]
    elif y_perm:
        ref_idx = perm.cpu().numpy()
    log("CPU oracle: reference and baseline timing")
    if not args.no_cpu:
        y_ref, cpu = cpu_baseline_leg(A, x_np, b_alg)
    else:
        import oracle
        y_ref = oracle.csr_spmv(A, x_np)
    yr = y_ref[ref_idx] if y_perm else y_ref
    checks["headline"] = out["rel_err_vs_oracle"] = rel_err(y, yr)
    del y

    lanes_key = f"_T{args.lanes}" if args.lanes > 1 else ""
    if args.x_halo >= 0 and args.two_rows:
        lanes_key += "_2rows"
    if args.split_len:
        lanes_key += f"_split{args.split_len}"
    traffic = load_traffic(f"{args.workload}_{args.dtype}_b{args.block_height}_{args.layout}_w{args.sort_window}_h{args.x_halo}_t{args.tile_rows}_{args.mode}{lanes_key}")
    result = {
        "metric": "pJDS spMVM GB/s & %HBM peak; tuned/batched vs plain GFLOP/s at <=1e-12 rel err",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded generator standing in for the paper's Holstein-Hubbard matrix)",
        "config": {"workload": desc, "n_rows": n, "nnz": nnz, "block_height": M.info.block_height,
                   "lanes_per_row": args.lanes,
                   "layout": args.layout, "mode": args.mode, "nnz_stored": M.info.nnz_stored,
                   "sort_window": M.info.sort_window, "xcd_remap": args.xcd_remap, "x_halo": args.x_halo,
                   "tile_rows": args.tile_rows if args.x_halo >= 0 else None,
                   "rows_per_lane": 2 if (args.x_halo >= 0 and args.two_rows) else 1,
                   "row_lengths": "uint8" if (args.x_halo >= 0 and M.info.max_row_len <= 255) else "int32",
                   "split_len": M.info.split_len, "n_chunks": M.info.n_chunks,
                   "protocol": "median of the steps' product times, each product after a 1 GiB read-only pass with cached loads (Infinity Cache cold); "
                               "a product's time is its kernel's own duration, from HIP events its dispatch records (pjds_time_next_launch)"},
        "roofline": {"bound": "hbm", "achieved": round(gbs_mean, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs_mean / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": ("pjds_spmv_lds2_kernel" if args.two_rows else "pjds_spmv_lds_kernel") if args.x_halo >= 0 else
                               ("pjds_lanes_kernel" if args.lanes > 1 else "pjds_spmv_kernel"),
                     "alg_bytes_per_launch": b_alg, "mean_launch_ms": round(ms_mean, 5)},
        "cpu_baseline": cpu,
        "gflops": round(gflops, 2),
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "steps_ms": {"min": round(min(ms_steps), 5), "median": round(ms, 5), "mean": round(ms_mean, 5),
                     "max": round(max(ms_steps), 5), "wall_s_timed_region": round(t_wall, 4),
                     "bracket_events": {"median": round(float(np.median(ms_bracket)), 5),
                                        "mean": round(float(np.mean(ms_bracket)), 5),
                                        "GBps_alg_median": round(b_alg / float(np.median(ms_bracket)) / 1e6, 2),
                                        "protocol": "HIP events recorded on the stream before and after each step"}},
        "warm": {"ms_mean": round(ms_warm, 5), "GBps_alg": round(b_alg / ms_warm / 1e6, 2),
                 "frac": round(b_alg / ms_warm / 1e6 / HBM_PEAK_GBS, 4),
                 "protocol": "mean of 200 back-to-back products after 20 warm-ups"},
        "conversion_s": round(t_conv, 3),
        "footprint_bytes": {"pjds": M.footprint_bytes()},
        "kernel_sources_sha256_16": kernel_source_hash(),
    }
    result.update(out)

    # achievable ceiling: read-only and copy probes over 2 GiB (the copy kernel of known
    # size also calibrates the byte counters of a profiling run)
    nprobe = 1 << 28
    a = torch.empty(nprobe, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty(nprobe, dtype=torch.float64, device="cuda")
    r = torch.empty(2048, dtype=torch.float64, device="cuda")
    ms_r = time_launches(lambda: _lib.pjds_probe(0, a, r, nprobe), 10, 2)
    ms_c = time_launches(lambda: _lib.pjds_probe(1, a, b, nprobe), 10, 2)
    result["hbm_probe"] = {"bytes_read": 8 * nprobe, "read_GBps": round(8 * nprobe / ms_r / 1e6, 1),
                           "copy_bytes": 16 * nprobe, "copy_GBps": round(16 * nprobe / ms_c / 1e6, 1)}
    result["pct_of_probe_read"] = round(100 * gbs / result["hbm_probe"]["read_GBps"], 2)
    del a, b, r

    if not args.no_extra:
        extra = {}
        rows = sample_rows(n, 91)
        ref_rows = y_ref[rows]
        x_orig = torch.from_numpy(x_np).to("cuda", tdt)

        def leg(name, fn, y_out, perm_dev=None, b=b_alg, flops=2 * nnz, ref=ref_rows, rws=rows, reps=20,
                hook=True):
            """Cold median and warm mean of one comparison leg, and its sampled rows checked.
            `ms` is the kernel's own duration (timing hook) for a one-kernel call, else the
            bracketing events' time; `ms_bracket` is the latter in every case."""
            ms_c = cold.median(fn, reps, hook=hook)
            ms_b = float(np.median(cold.last_bracket))
            ms_w = time_launches(fn, 50, 5)
            checks[name] = rel_err(rows_in_original_order(torch, y_out, rws, perm_dev), ref)
            return {"ms": round(ms_c, 5), "ms_bracket": round(ms_b, 5), "timing": cold.last_kind,
                    "ms_warm": round(ms_w, 5), "GBps_alg": round(b / ms_c / 1e6, 1),
                    "gflops": round(flops / ms_c / 1e6, 2), "rel_err_sampled": checks[name]}

        log("ELLPACK-R and CSR legs")
        info_e = EllrMatrix.plan(A)
        ebytes = info_e.nnz_stored * (vbytes + 4) + info_e.n_pad * 4
        result["footprint_bytes"]["ellpack_r"] = ebytes
        result["footprint_bytes"]["csr"] = nnz * (vbytes + 4) + (n + 1) * 8
        if ebytes < 64 * 2 ** 30:
            E = EllrMatrix.from_csr(A)
            ye = torch.empty(n, dtype=tdt, device="cuda")
            extra["ellpack_r"] = leg("ellpack_r", lambda: E.spmv(x_orig, ye), ye)
            del E, ye
        C = CsrMatrix.from_csr(A)
        yc = torch.empty(n, dtype=tdt, device="cuda")
        for v in (1, 4, 16):
            extra[f"csr_v{v}"] = leg(f"csr_v{v}", lambda: C.spmv(x_orig, yc, variant=v), yc)
        del C, yc
        # scatter-y and XCD-renumbering variants of the plain kernel on the headline's storage
        if args.mode != "symmetric":
            ys_ = torch.empty(n, dtype=tdt, device="cuda")
            extra["pjds_scatter_y"] = leg("pjds_scatter_y", lambda: M.spmv(x_dev, ys_, y_permuted=False), ys_)
            extra["pjds_xcd_remap"] = leg("pjds_xcd_remap", lambda: M.spmv(x_dev, ys_, y_permuted=True, xcd_remap=True),
                                          ys_, perm_dev=perm)
            del ys_
        # many right-hand sides on the same matrix: the tile shape and XCD renumbering tuned
        # per k on two sort windows (256 keeps shared rows of X close; 4096 with renumbering lets
        # each XCD's L2 keep them), and X staged in LDS on windows of 256; effective GFLOP/s vs
        # the headline single-vector product
        log("SpMMV leg")
        spmmv = {"plain_gflops": round(gflops, 2)}
        from paper_1112_5588_amd import autotune as _at
        rows_k = rows[::4]
        for sw_k in (256, 4096):
            Mk = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=sw_k)
            for k in (4, 8, 16, 32):
                (t, vpl, rmp), _ = _at.tune_spmmv(Mk, k, reps=3)
                X_np = synth.dense_x(A.n_cols, 4, k=k).reshape(A.n_cols, k)
                X = torch.from_numpy(X_np).to("cuda", tdt)
                Y = torch.empty((n, k), dtype=tdt, device="cuda")
                ref_k = reference_rows(A, X_np, rows_k)
                bk = (vbytes + 4) * nnz + 2 * vbytes * n * k
                r = leg(f"spmmv_k{k}_w{sw_k}", lambda: Mk.spmmv(X, Y, vectors_per_tile=t, vectors_per_lane=vpl,
                                                                y_permuted=True, xcd_remap=rmp),
                        Y, perm_dev=Mk.d["perm"], b=bk, flops=2 * k * nnz, ref=ref_k, rws=rows_k)
                r.update({"sort_window": sw_k, "tile": t, "vectors_per_lane": vpl, "xcd_remap": rmp,
                          "x_path": "caches", "over_plain": round(r["gflops"] / gflops, 2)})
                if f"k{k}" not in spmmv or r["ms"] < spmmv[f"k{k}"]["ms"]:
                    spmmv[f"k{k}"] = r
                if sw_k == 256:
                    # X staged in LDS (pjds_spmmv_xlds): one vector tile of up to 8 vectors, since
                    # 64 KiB holds 1024 rows of 8 FP64 values (512-row tiles) or 2048 rows of 4
                    t_s = min(k, 8)
                    tile_s = 1024 if t_s * vbytes <= 32 else 512
                    r = leg(f"spmmv_k{k}_lds", lambda: Mk.spmmv_xlds(X, Y, vectors_per_tile=t_s, vectors_per_lane=4,
                                                                     x_halo=512, tile_rows=tile_s, y_permuted=True),
                            Y, perm_dev=Mk.d["perm"], b=bk, flops=2 * k * nnz, ref=ref_k, rws=rows_k)
                    r.update({"sort_window": sw_k, "tile": t_s, "vectors_per_lane": 4, "tile_rows": tile_s,
                              "x_halo": 512, "x_path": "lds", "over_plain": round(r["gflops"] / gflops, 2)})
                    spmmv[f"k{k}_x_in_lds"] = r
                    if r["ms"] < spmmv[f"k{k}"]["ms"]:
                        spmmv[f"k{k}"] = r
                del X, Y
            del Mk
        extra["spmmv"] = spmmv
        # the small case (128 x 128 Laplacian): one SpMMV launch against k single products,
        # launched one by one and replayed from a captured graph (launch-bound: warm timing)
        L1 = synth.laplacian_2d(128)
        M1 = PjdsMatrix.from_csr(L1, block_height=64)
        small = {}
        for k in (1, 4, 8, 16, 32):
            X1 = synth.dense_x(L1.n_cols, 4, k=k).reshape(L1.n_cols, k)
            Xk = torch.from_numpy(X1).cuda()
            Yk = torch.empty((L1.n_rows, k), dtype=torch.float64, device="cuda")
            (t, vpl, rmp), _ = _at.tune_spmmv(M1, k, reps=5)
            ms_mm = time_launches(lambda: M1.spmmv(Xk, Yk, vectors_per_tile=t, vectors_per_lane=vpl, y_permuted=False,
                                                   xcd_remap=rmp), 200, 20)
            checks[f"laplacian_spmmv_k{k}"] = rel_err(Yk.cpu().numpy(), reference_rows(L1, X1, np.arange(L1.n_rows)))
            xs = [Xk[:, v].contiguous() for v in range(k)]
            ys = [torch.empty(L1.n_rows, dtype=torch.float64, device="cuda") for _ in range(k)]

            def singles():
                for v in range(k):
                    M1.spmv(xs[v], ys[v], y_permuted=True)
            ms_sep = time_launches(singles, 200, 20)
            g1 = torch.cuda.CUDAGraph()
            cs1 = torch.cuda.Stream()
            cs1.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cs1):
                with torch.cuda.graph(g1, stream=cs1):
                    singles()
            torch.cuda.current_stream().wait_stream(cs1)
            ms_gr = time_launches(g1.replay, 200, 20)
            f = 2 * k * L1.nnz / 1e6
            small[f"k{k}"] = {"spmmv_ms": round(ms_mm, 5), "spmmv_gflops": round(f / ms_mm, 2),
                              "singles_ms": round(ms_sep, 5), "singles_gflops": round(f / ms_sep, 2),
                              "singles_graph_ms": round(ms_gr, 5), "singles_graph_gflops": round(f / ms_gr, 2),
                              "tile": t, "vectors_per_lane": vpl, "rel_err": checks[f"laplacian_spmmv_k{k}"]}
            del g1
        extra["spmmv_laplacian_128"] = small
        # exhaustive autotuner on this matrix: every catalog configuration, plus x in LDS
        from paper_1112_5588_amd import autotune
        log("autotuner leg")
        t0_at = time.perf_counter()
        t_cat = autotune.time_all(A, x=x_orig)
        exhaustive_s = time.perf_counter() - t0_at
        # the learned tuner on the same matrix: features on the host, one network inference, and
        # on a near tie the timing of its three best candidates (the rule of tuner.decide)
        from paper_1112_5588_amd import tuner as _tn
        t0_at = time.perf_counter()
        feats = _lib.pjds_features(A.n_rows, A.n_cols, np.ascontiguousarray(A.row_ptr, np.int64),
                                   np.ascontiguousarray(A.col, np.int32))
        model = _tn.Model.load(os.path.join(ROOT, "paper_1112_5588_amd", "tuner_data", "model.json"))
        Xf = np.asarray(feats, np.float64)[None, :]
        runnable = autotune.runnable_mask(A.n_rows, A.n_cols, vbytes,
                                          bool(_tn.ellr_fits(Xf, np.array([float(nnz)]))[0]))[None, :]
        mode, cand = _tn.decide(_tn.predict_scores(model, Xf), runnable, Xf, model)
        mode = str(mode[0])
        if mode == "net":
            learned_pick = autotune.CONFIG_NAMES[int(cand[0, 0])]
        else:
            cfgs = autotune.CATALOG if mode == "full" else [autotune.CATALOG[int(c)] for c in cand[0]]
            t_k = autotune.time_all(A, x=x_orig, configs=cfgs)
            learned_pick = min(t_k, key=t_k.get)
        learned_s = time.perf_counter() - t0_at
        lds = {}
        for sw, halo, tile in ((512, 1024, 512), (1024, 1024, 1024)):   # LDS forms outside the catalog
            Mw = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=sw)
            yw = torch.empty(n, dtype=tdt, device="cuda")
            lds[f"pjds_b64_w{sw}_lds{halo}_t{tile}"] = autotune.time_median(
                lambda: Mw.spmv_xlds(x_orig, yw, x_halo=halo, tile_rows=tile, y_permuted=True), 20, 3)
            checks[f"autotune_w{sw}_lds"] = rel_err(rows_in_original_order(torch, yw, rows, Mw.d["perm"]), ref_rows)
            del Mw
        t_all = {**t_cat, **lds}
        best = min(t_all, key=t_all.get)
        plain = t_all[autotune.CONFIG_NAMES[autotune.DEFAULT]]
        # the product inside a solver: Lanczos steps in the permuted basis (symmetric conversion)
        if args.dtype == "f64" and A.n_rows == A.n_cols:
            log("Lanczos leg")
            Ms = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=args.sort_window, symmetric=True)
            v0 = torch.from_numpy(x_np).to("cuda", torch.float64)[Ms.d["perm"].long()].contiguous()
            steps = 20
            bufs = Ms.lanczos_buffers()
            al = torch.empty(steps, dtype=torch.float64, device="cuda")
            be = torch.empty(steps + 1, dtype=torch.float64, device="cuda")
            ms_l = time_launches(lambda: Ms.lanczos(v0, steps, x_halo=args.x_halo, tile_rows=args.tile_rows,
                                                    alpha=al, beta=be, buffers=bufs), 5, 1)
            g = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cs):
                with torch.cuda.graph(g, stream=cs):
                    Ms.lanczos(v0, steps, x_halo=args.x_halo, tile_rows=args.tile_rows, alpha=al, beta=be,
                               buffers=bufs)
            torch.cuda.current_stream().wait_stream(cs)
            ms_g = time_launches(g.replay, 5, 1)
            ys = torch.empty(n, dtype=torch.float64, device="cuda")
            # the product as the Lanczos step runs it (one-byte row lengths when every row fits)
            ms_p = time_launches(lambda: Ms.spmv_xlds(v0, ys, x_halo=args.x_halo, tile_rows=args.tile_rows,
                                                      y_permuted=True, two_rows=True), 50, 5)
            # vector passes besides the product's x and y: z read, w and u_j read and w written by
            # the update; w and u_j read once more for alpha when x is not staged in LDS
            passes = 4 if args.x_halo >= 0 else 6
            extra["lanczos"] = {"steps": steps, "ms_per_step_eager": round(ms_l / steps, 5),
                                "ms_per_step_graph": round(ms_g / steps, 5), "ms_product_alone": round(ms_p, 5),
                                "step_over_product": round(ms_g / steps / ms_p, 3),
                                "vector_passes_per_step": passes,
                                "GBps_alg_per_step": round((b_alg + passes * 8 * n) / (ms_g / steps) / 1e6, 1)}
            del Ms, bufs, g
        # host link (eq. 2-4): x to the device, the product on that copy, y back, from pinned
        # host memory
        xh = torch.from_numpy(x_np).to(tdt).pin_memory()
        yh = torch.empty(n, dtype=tdt).pin_memory()
        xd2 = torch.empty_like(x_dev)
        if args.mode == "symmetric":
            xh = xh[perm.cpu().long()].contiguous().pin_memory()

        def h2d():
            xd2.copy_(xh, non_blocking=True)

        def d2h():
            yh.copy_(y_dev, non_blocking=True)
        ms_h2d = time_launches(h2d, 20, 3)
        ms_d2h = time_launches(d2h, 20, 3)

        def with_link():
            xd2.copy_(xh, non_blocking=True)
            product(xd2, y_dev)
            yh.copy_(y_dev, non_blocking=True)
        ms_link = time_launches(with_link, 20, 3)
        torch.cuda.synchronize()
        yl = yh.double().numpy()
        # y in the permuted basis: original row r sits at the inverse permutation's slot r
        checks["host_link"] = rel_err(yl[np.argsort(ref_idx)][rows] if y_perm else yl[rows], ref_rows)
        from paper_1112_5588_amd import model as pmodel
        # eq. (2): B_GPU is the device's streaming bandwidth (the read probe), B_PCI the measured
        # round trip of x and y over the host link; alpha at its minimum 1/N_nzr
        nnzr = nnz / n
        b_gpu = result["hbm_probe"]["read_GBps"] * 1e9
        b_pci = 2 * vbytes * n / ((ms_h2d + ms_d2h) * 1e-3)
        ratio = b_gpu / b_pci
        t_mvm_model = pmodel.t_mvm(n, nnzr, 1.0 / nnzr, b_gpu)
        t_pci_model = pmodel.t_pci(n, b_pci)
        extra["host_link"] = {
            "h2d_GBps": round(vbytes * n / ms_h2d / 1e6, 1), "d2h_GBps": round(vbytes * n / ms_d2h / 1e6, 1),
            "B_gpu_over_B_pci": round(ratio, 2), "n_nzr": round(nnzr, 2),
            "ms_product": round(ms_warm, 5), "ms_product_eq2": round(t_mvm_model * 1e3, 5),
            "ms_transfers_eq2": round(t_pci_model * 1e3, 5), "ms_with_transfers": round(ms_link, 5),
            "transfer_share_measured": round(1 - ms_warm / ms_link, 4),
            "transfer_share_eq2": round(t_pci_model / (t_pci_model + t_mvm_model), 4),
            "eq3_nnzr_max_half_penalty": {"alpha0": round(pmodel.nnzr_bound_half_penalty(ratio, 0.0), 1),
                                          "alpha1": round(pmodel.nnzr_bound_half_penalty(ratio, 1.0), 1)},
            "eq4_nnzr_min_tenth_penalty": {"alpha0": round(pmodel.nnzr_bound_tenth_penalty(ratio, 0.0), 1),
                                           "alpha1": round(pmodel.nnzr_bound_tenth_penalty(ratio, 1.0), 1)},
            "rel_err_sampled": checks["host_link"]}
        del xh, yh, xd2
        # T lanes per row (block layout, same sort window, x through the caches) on this matrix,
        # and the sliced formats the outlook names: rows sorted only inside each 64-row slice
        # (sliced ELLPACK's padding; with T lanes, sliced ELLR-T's)
        lanes_leg = {}
        for T, sw_l in ((2, args.sort_window), (4, args.sort_window), (8, args.sort_window), (1, 64), (4, 64)):
            Ml = PjdsMatrix.from_csr(A, layout="block", sort_window=sw_l, lanes=T)
            yl_ = torch.empty(n, dtype=tdt, device="cuda")
            key = f"T{T}" if sw_l == args.sort_window else f"sliced_w{sw_l}_T{T}"
            lanes_leg[key] = leg(f"lanes_{key}", lambda: Ml.spmv(x_orig, yl_, y_permuted=True), yl_, perm_dev=Ml.d["perm"])
            lanes_leg[key]["nnz_stored"] = Ml.info.nnz_stored
            del Ml
        extra["lanes_per_row"] = lanes_leg
        # local/non-local split (vector mode with overlap): y written, then read and written again
        from paper_1112_5588_amd.matrix import split_columns
        loc, nl = split_columns(A, 0, A.n_cols // 2)
        ML, MN = PjdsMatrix.from_csr(loc), PjdsMatrix.from_csr(nl)
        M1 = PjdsMatrix.from_csr(A)
        yo = torch.empty(n, dtype=tdt, device="cuda")

        def split_step():
            ML.spmv(x_orig, yo)
            MN.spmv_axpby(x_orig, yo, alpha=1.0, beta=1.0, z=yo)
        split_r = leg("split_local_nonlocal", split_step, yo, hook=False)
        one_r = leg("split_reference_single", lambda: M1.spmv(x_orig, yo), yo, hook=False)   # like for like
        nnzr = nnz / n
        extra["split_local_nonlocal"] = {
            "ms_split": split_r["ms"], "ms_single": one_r["ms"],
            "penalty": round(split_r["ms"] / one_r["ms"] - 1, 4),
            "model_penalty_eq1": round((8.0 / nnzr) / pmodel.code_balance_dp(1.0 / nnzr, nnzr), 4),
            "rel_err_sampled": split_r["rel_err_sampled"]}
        del ML, MN, M1, loc, nl
        extra["autotune"] = {"ms": {k: round(v, 5) for k, v in t_all.items()}, "best": best,
                             "best_GBps_alg": round(b_alg / t_all[best] / 1e6, 1),
                             "plain_GBps_alg": round(b_alg / plain / 1e6, 1),
                             "tuned_over_plain": round(plain / t_all[best], 3),
                             "exhaustive_search_s": round(exhaustive_s, 2),
                             "learned": {"pick": learned_pick, "mode": mode,
                                         "candidates": [autotune.CONFIG_NAMES[int(c)] for c in cand[0]],
                                         "pick_ms": round(t_cat[learned_pick], 5),
                                         "regret_vs_catalog_best": round(t_cat[learned_pick] / min(t_cat.values()) - 1, 4),
                                         "over_plain": round(plain / t_cat[learned_pick], 3),
                                         "tuning_s": round(learned_s, 3)}}
        # the same matrix with FP32 values (values rounded to nearest), headline configuration
        if args.dtype == "f64":
            A32 = A.astype(np.float32)
            M32 = PjdsMatrix.from_csr(A32, block_height=args.block_height, layout=args.layout,
                                      sort_window=args.sort_window)
            x32_np = x_np.astype(np.float32)
            x32 = torch.from_numpy(x32_np).to("cuda")
            y32 = torch.empty(n, dtype=torch.float32, device="cuda")
            b32 = 8 * nnz + 8 * n
            ref32 = reference_rows(A32, x32_np.astype(np.float64), rows)
            if args.x_halo >= 0:
                fn32 = lambda: M32.spmv_xlds(x32, y32, x_halo=args.x_halo, tile_rows=args.tile_rows,  # noqa: E731
                                             y_permuted=True, two_rows=args.two_rows)
            else:
                fn32 = lambda: M32.spmv(x32, y32, y_permuted=True)  # noqa: E731
            r = leg("fp32", fn32, y32, perm_dev=M32.d["perm"], b=b32, ref=ref32)
            tol_of["fp32"] = TOL["f32"]
            r["alg_bytes"] = b32
            extra["fp32"] = r
            del A32, M32, x32, y32
        # the skewed-row workload: global sort vs sort windows 2^10..2^16 (padding and time),
        # several lanes per row, and ELLPACK-R's padded size (planned, not allocated)
        log("power-law leg")
        del M, x_dev, y_dev, x_orig
        torch.cuda.empty_cache()
        P, _ = make_workload("powerlaw", args.dtype)
        xp_np = synth.dense_x(P.n_cols, 3)
        if args.dtype == "f32":
            xp_np = xp_np.astype(np.float32).astype(np.float64)
        xp = torch.from_numpy(xp_np).to("cuda", tdt)
        yp_ = torch.empty(P.n_rows, dtype=tdt, device="cuda")
        bp = (vbytes + 4) * P.nnz + 2 * vbytes * P.n_rows
        rows_p = sample_rows(P.n_rows, 93)
        pl = {"nnz": P.nnz, "ellpack_r_stored": EllrMatrix.plan(P).nnz_stored}
        for label, kw in (("global_split512", dict(layout="block", split_len=512)),
                          ("global_nosplit", dict(layout="block", split_len=-1)),
                          ("w1024", dict(layout="block", sort_window=1024, split_len=512)),
                          ("w4096", dict(layout="block", sort_window=4096, split_len=512)),
                          ("w16384", dict(layout="block", sort_window=16384, split_len=512)),
                          ("w65536", dict(layout="block", sort_window=65536, split_len=512)),
                          ("global_lanes4", dict(layout="block", lanes=4)),
                          # rows sorted only inside each 64-row slice: the padding of sliced
                          # ELLPACK, and with 4 lanes per row that of sliced ELLR-T
                          ("sliced_ellpack_w64", dict(layout="block", sort_window=64, split_len=512)),
                          ("sliced_ellr_t4_w64", dict(layout="block", sort_window=64, lanes=4))):
            Mp = PjdsMatrix.from_csr(P, keep_host=True, **kw)
            if label == "global_split512":
                # the longest rows (split into work items) join the sampled rows
                rows_p = np.unique(np.concatenate([rows_p, Mp.host["perm"][:2048].astype(np.int64)]))
                ref_p = reference_rows(P, xp_np, rows_p)
            r = leg(f"powerlaw_{label}", lambda: Mp.spmv(xp, yp_, y_permuted=True), yp_, perm_dev=Mp.d["perm"],
                    b=bp, flops=2 * P.nnz, ref=ref_p, rws=rows_p)
            r.update({"nnz_stored": Mp.info.nnz_stored, "padding": round(Mp.info.nnz_stored / P.nnz - 1, 4)})
            pl[label] = r
            del Mp
        extra["powerlaw"] = pl
        del P, xp, yp_
        result["extra"] = extra
    if not args.no_batch:
        torch.cuda.empty_cache()
        result["batch"] = batch_leg(torch, checks)

    result["checks"] = {"tolerance": tol, "tolerance_per_leg": tol_of,
                        "rel_err": {k: float(f"{v:.3e}") for k, v in checks.items()}}
    bad = [k for k, v in checks.items() if not v <= tol_of.get(k, tol)]
    if bad:
        result["error"] = f"outside the relative-error tolerance: {', '.join(bad)}"
        result["value"] = None
        print(json.dumps(result), flush=True)
        return 1
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
