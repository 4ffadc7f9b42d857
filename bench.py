#!/usr/bin/env python3
"""Benchmark: pJDS sparse matrix-vector product on one MI355X.

Default workload: the Holstein-Hubbard-like matrix (N = 2^22 rows, banded symmetric pattern
with contiguous off-diagonals, row lengths 5..20, N(0,1) values), FP64.  Default kernel
configuration: the tuned pJDS form -- block height 64, rows sorted inside windows of 256
(per-block layout), x staged in LDS per 1024-row tile with a halo of 768, two adjacent rows
per lane, y written in the permuted basis (Listing 2).  The paper's plain configuration (global sort, jagged-diagonal
layout) is timed beside it in `extra.autotune`.  One step is one product y = A x with the
matrix and x already resident in HBM.

Prints ONE JSON line.  `value` is the achieved bandwidth by the algorithmic byte count of
the product, 12 B per non-zero (value + column index) plus 8 B per row for x and 8 B per
row for y, divided by the measured time per product.

    python bench.py [--steps K] [--warmup W] [--workload hh_like|laplacian|powerlaw]
                    [--dtype f64|f32] [--sort-window W] [--x-halo H] [--tile-rows T] [--one-row]
                    [--lanes T] [--xcd-remap] [--no-cpu] [--no-extra] [--no-batch]

Besides the headline line's own fields, `extra` holds the comparison legs (cold Infinity Cache,
ELLPACK-R, CSR, SpMMV with X through the caches or staged in LDS, the 128 x 128 Laplacian's
SpMMV against single products, the exhaustive and learned tuners, Lanczos steps, the host-link
model, lanes per row, the local/non-local split, FP32 and the power-law matrix) and `batch` the
512-matrix leg (persistent kernel with x through the caches or staged in LDS, per-member graph,
direct launches).
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


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_1112_5588_amd", "csrc", "spmv.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(workload_key: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it was taken
    on the kernel source that is built now; otherwise None."""
    p = os.path.join(ROOT, "profiles", "pjds_spmv_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    e = d.get(workload_key)
    if not e or e.get("kernel_source_sha256_16") != kernel_source_hash():
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
    """Average ms per call of `fn` over `steps` calls, bracketed by events on the stream the
    kernels are launched on (torch's current stream)."""
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


def cpu_baseline(A, x, budget_s: float = 12.0):
    """The oracle's serial CSR product timed on this host (1 core)."""
    import oracle
    t0 = time.perf_counter()
    y = oracle.csr_spmv(A, x)
    first = time.perf_counter() - t0
    reps = max(1, min(200, int(budget_s / max(first, 1e-4))))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.csr_spmv(A, x)
    dt = (time.perf_counter() - t0) / reps
    return y, dt, reps


def batch_leg(torch) -> dict:
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
        for name, mode, halo in (("persistent_graph", _lib.PJDS_BATCH_PERSISTENT, None),
                                 ("persistent_graph_x_in_lds", _lib.PJDS_BATCH_PERSISTENT, 4096),
                                 ("per_member_graph", _lib.PJDS_BATCH_GRAPH, None),
                                 ("direct_launches", _lib.PJDS_BATCH_DIRECT, None)):
            B = PjdsBatch(mats, xs, ys, mode=mode, y_permuted=True, x_halo=halo)
            ms = time_launches(B.launch, 10, 2)
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
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="hh_like", choices=["hh_like", "laplacian", "powerlaw"])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--block-height", type=int, default=64)
    ap.add_argument("--layout", default="block", choices=["jd", "block"])
    ap.add_argument("--mode", default="y_permuted", choices=["y_permuted", "scatter", "symmetric"])
    ap.add_argument("--split-len", type=int, default=0)
    ap.add_argument("--sort-window", type=int, default=256, help="0 = global sort")
    ap.add_argument("--xcd-remap", action="store_true")
    ap.add_argument("--x-halo", type=int, default=768,
                    help=">= 0: stage x in LDS with this halo (block layout, window % 256 == 0); -1: x through the caches")
    ap.add_argument("--tile-rows", type=int, default=1024, help="rows per workgroup of the LDS path")
    ap.add_argument("--one-row", dest="two_rows", action="store_false",
                    help="LDS path: one row per lane (default: two adjacent rows per lane, 2-wide loads)")
    ap.add_argument("--lanes", type=int, default=1,
                    help="lanes per row (power of two up to 64, block layout, x through the caches)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip comparison legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-matrix batch leg")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU path "
                                   "of the paper is not built (one GPU per process, --gpus 1)"}))
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

    if args.x_halo >= 0:
        def step():
            M.spmv_xlds(x_dev, y_dev, x_halo=args.x_halo, tile_rows=args.tile_rows, y_permuted=y_perm,
                        xcd_remap=args.xcd_remap, two_rows=args.two_rows)
    else:
        def step():
            M.spmv(x_dev, y_dev, y_permuted=y_perm, xcd_remap=args.xcd_remap)

    log("timing")
    ms = time_launches(step, args.steps, args.warmup)
    # algorithmic bytes: value + index per non-zero, x once, y once (write)
    b_alg = (vbytes + 4) * nnz + 2 * vbytes * n
    if args.mode == "scatter":
        b_alg += 4 * n               # the permutation read to scatter y
    gbs = b_alg / (ms * 1e-3) / 1e9
    gflops = 2 * nnz / (ms * 1e-3) / 1e9

    # correctness gate on the full vector: the oracle's serial product
    out: dict = {}
    cpu = None
    y = y_dev.double().cpu().numpy()
    if y_perm:
        ref_idx = M.d["perm"].cpu().numpy()
    if not args.no_cpu:
        log("CPU oracle baseline")
        y_ref, dt_cpu, reps = cpu_baseline(A, x_np)
        cpu = {"value": round(b_alg / dt_cpu / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"full matrix, {reps} serial CSR products (binary64, no FMA), median-free mean over {reps*dt_cpu:.1f}s",
               "gflops": round(2 * nnz / dt_cpu / 1e9, 3), "ms_per_product": round(dt_cpu * 1e3, 3)}
        yr = y_ref[ref_idx] if y_perm else y_ref
        import oracle
        out["rel_err_vs_oracle"] = oracle.rel_l2(y, yr)

    lanes_key = f"_T{args.lanes}" if args.lanes > 1 else ""
    if args.x_halo >= 0 and args.two_rows:
        lanes_key += "_2rows"
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
                   "split_len": M.info.split_len, "n_chunks": M.info.n_chunks},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": ("pjds_spmv_lds2_kernel" if args.two_rows else "pjds_spmv_lds_kernel") if args.x_halo >= 0 else
                               ("pjds_lanes_kernel" if args.lanes > 1 else "pjds_spmv_kernel"),
                     "alg_bytes_per_launch": b_alg},
        "cpu_baseline": cpu,
        "gflops": round(gflops, 2),
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "conversion_s": round(t_conv, 3),
        "footprint_bytes": {"pjds": M.footprint_bytes()},
        "kernel_source_sha256_16": kernel_source_hash(),
    }
    result.update(out)

    # achievable ceiling: read-only and copy probes over 2 GiB (the copy kernel of known
    # size also calibrates the byte counters of a profiling run)
    nprobe = 1 << 28
    a = torch.empty(nprobe, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty(nprobe, dtype=torch.float64, device="cuda")
    r = torch.empty(4096, dtype=torch.float64, device="cuda")
    ms_r = time_launches(lambda: _lib.pjds_probe(0, a, r, nprobe), 10, 2)
    ms_c = time_launches(lambda: _lib.pjds_probe(1, a, b, nprobe), 10, 2)
    result["hbm_probe"] = {"bytes_read": 8 * nprobe, "read_GBps": round(8 * nprobe / ms_r / 1e6, 1),
                           "copy_bytes": 16 * nprobe, "copy_GBps": round(16 * nprobe / ms_c / 1e6, 1)}
    result["pct_of_probe_read"] = round(100 * gbs / result["hbm_probe"]["read_GBps"], 2)
    del a, b, r

    if not args.no_extra:
        extra = {}
        # cold Infinity Cache: the median of single products, each after a 1 GiB streaming
        # pass over another buffer evicts the matrix and x from the 256 MB MALL
        flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        flush.fill_(1.0)

        def cold_median(fn, reps: int = 20) -> float:
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps + 1)]
            for s0, s1 in ev:
                flush.mul_(1.0)
                s0.record()
                fn()
                s1.record()
            torch.cuda.synchronize()
            cold = sorted(s0.elapsed_time(s1) for s0, s1 in ev[1:])
            return cold[len(cold) // 2]

        ms_cold = cold_median(step)
        extra["cold_mall"] = {"reps": 20, "median_ms": round(ms_cold, 5),
                              "GBps_alg": round(b_alg / ms_cold / 1e6, 1)}
        # same matrix in the comparison formats
        log("ELLPACK-R and CSR legs")
        info_e = EllrMatrix.plan(A)
        ebytes = info_e.nnz_stored * (vbytes + 4) + info_e.n_pad * 4
        result["footprint_bytes"]["ellpack_r"] = ebytes
        result["footprint_bytes"]["csr"] = nnz * (vbytes + 4) + (n + 1) * 8
        if ebytes < 64 * 2 ** 30:
            E = EllrMatrix.from_csr(A)
            xo = torch.from_numpy(x_np).to("cuda", tdt)
            ye = torch.empty(n, dtype=tdt, device="cuda")
            ms_e = time_launches(lambda: E.spmv(xo, ye), 50, 5)
            extra["ellpack_r"] = {"ms": round(ms_e, 5), "GBps_alg": round(((vbytes + 4) * nnz + 2 * vbytes * n) / ms_e / 1e6, 1),
                                  "gflops": round(2 * nnz / ms_e / 1e6, 2)}
            del E
        C = CsrMatrix.from_csr(A)
        xo = torch.from_numpy(x_np).to("cuda", tdt)
        yc = torch.empty(n, dtype=tdt, device="cuda")
        for v in (1, 4, 16):
            ms_c = time_launches(lambda: C.spmv(xo, yc, variant=v), 50, 5)
            extra[f"csr_v{v}"] = {"ms": round(ms_c, 5), "GBps_alg": round(((vbytes + 4) * nnz + 2 * vbytes * n) / ms_c / 1e6, 1),
                                  "gflops": round(2 * nnz / ms_c / 1e6, 2)}
        del C
        # scatter-y and XCD-renumbering variants of the headline kernel
        ms_s = time_launches(lambda: M.spmv(x_dev, y_dev, y_permuted=False), 50, 5)
        ms_nr = time_launches(lambda: M.spmv(x_dev, y_dev, y_permuted=y_perm, xcd_remap=True), 50, 5)
        extra["pjds_scatter_y"] = {"ms": round(ms_s, 5)}
        extra["pjds_xcd_remap"] = {"ms": round(ms_nr, 5)}
        # many right-hand sides on the same matrix: the tile shape and XCD renumbering tuned
        # per k on two sort windows (256 keeps shared rows of X close; 4096 with renumbering lets
        # each XCD's L2 keep them), and X staged in LDS on windows of 256; effective GFLOP/s vs
        # the headline single-vector product
        spmmv = {"plain_gflops": round(gflops, 2)}
        from paper_1112_5588_amd import autotune as _at
        for sw_k in (256, 4096):
            Mk = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=sw_k)
            for k in (4, 8, 16, 32):
                (t, vpl, rmp), _ = _at.tune_spmmv(Mk, k, reps=3)
                X = torch.from_numpy(synth.dense_x(A.n_cols, 4, k=k).reshape(A.n_cols, k)).to("cuda", tdt)
                Y = torch.empty((n, k), dtype=tdt, device="cuda")
                ms_k = time_launches(lambda: Mk.spmmv(X, Y, vectors_per_tile=t, vectors_per_lane=vpl,
                                                      y_permuted=True, xcd_remap=rmp), 20, 3)
                if f"k{k}" not in spmmv or ms_k < spmmv[f"k{k}"]["ms"]:
                    spmmv[f"k{k}"] = {"sort_window": sw_k, "tile": t, "vectors_per_lane": vpl, "xcd_remap": rmp,
                                      "x_path": "caches",
                                      "ms": round(ms_k, 5), "gflops": round(2 * k * nnz / ms_k / 1e6, 2),
                                      "over_plain": round(2 * k * nnz / ms_k / 1e6 / gflops, 2)}
                if sw_k == 256:
                    # X staged in LDS (pjds_spmmv_xlds): one vector tile of up to 8 vectors, since
                    # 64 KiB holds 1024 rows of 8 FP64 values (512-row tiles) or 2048 rows of 4
                    t_s = min(k, 8)
                    tile_s = 1024 if t_s * vbytes <= 32 else 512
                    ms_s = time_launches(lambda: Mk.spmmv_xlds(X, Y, vectors_per_tile=t_s, vectors_per_lane=4,
                                                               x_halo=512, tile_rows=tile_s, y_permuted=True), 20, 3)
                    spmmv[f"k{k}_x_in_lds"] = {"tile": t_s, "tile_rows": tile_s, "x_halo": 512, "ms": round(ms_s, 5),
                                               "gflops": round(2 * k * nnz / ms_s / 1e6, 2)}
                    if ms_s < spmmv[f"k{k}"]["ms"]:
                        spmmv[f"k{k}"] = {"sort_window": sw_k, "tile": t_s, "vectors_per_lane": 4, "xcd_remap": False,
                                          "x_path": "lds", "tile_rows": tile_s, "x_halo": 512,
                                          "ms": round(ms_s, 5), "gflops": round(2 * k * nnz / ms_s / 1e6, 2),
                                          "over_plain": round(2 * k * nnz / ms_s / 1e6 / gflops, 2)}
                del X, Y
            del Mk
        extra["spmmv"] = spmmv
        # the small case (128 x 128 Laplacian): one SpMMV launch against k single products,
        # launched one by one and replayed from a captured graph
        L1 = synth.laplacian_2d(128)
        M1 = PjdsMatrix.from_csr(L1, block_height=64)
        small = {}
        for k in (1, 4, 8, 16, 32):
            Xk = torch.from_numpy(synth.dense_x(L1.n_cols, 4, k=k).reshape(L1.n_cols, k)).cuda()
            Yk = torch.empty((L1.n_rows, k), dtype=torch.float64, device="cuda")
            (t, vpl, rmp), _ = _at.tune_spmmv(M1, k, reps=5)
            ms_mm = time_launches(lambda: M1.spmmv(Xk, Yk, vectors_per_tile=t, vectors_per_lane=vpl, y_permuted=True,
                                                   xcd_remap=rmp), 200, 20)
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
                              "tile": t, "vectors_per_lane": vpl}
            del g1
        extra["spmmv_laplacian_128"] = small
        # exhaustive autotuner on this matrix: every catalog configuration, plus x in LDS
        from paper_1112_5588_amd import autotune
        log("autotuner leg")
        xo = torch.from_numpy(x_np).to("cuda", tdt)
        t0_at = time.perf_counter()
        t_cat = autotune.time_all(A, x=xo)
        exhaustive_s = time.perf_counter() - t0_at
        # the learned tuner on the same matrix: features on the host, one network inference
        from paper_1112_5588_amd import tuner as _tn
        t0_at = time.perf_counter()
        feats = _lib.pjds_features(A.n_rows, A.n_cols, np.ascontiguousarray(A.row_ptr, np.int64),
                                   np.ascontiguousarray(A.col, np.int32))
        model = _tn.Model.load(os.path.join(ROOT, "paper_1112_5588_amd", "tuner_data", "model.json"))
        pick_i, pick_margin = _tn.predict_matrices(model, np.asarray(feats, np.float64)[None, :],
                                                   np.array([float(nnz)]))
        learned_s = time.perf_counter() - t0_at
        learned_pick = autotune.CONFIG_NAMES[int(pick_i[0])]
        lds = {}
        for sw, halo, tile in ((512, 1024, 512), (1024, 1024, 1024)):   # LDS forms outside the catalog
            Mw = PjdsMatrix.from_csr(A, block_height=64, layout="block", sort_window=sw)
            yw = torch.empty(n, dtype=tdt, device="cuda")
            lds[f"pjds_b64_w{sw}_lds{halo}_t{tile}"] = autotune.time_median(
                lambda: Mw.spmv_xlds(xo, yw, x_halo=halo, tile_rows=tile, y_permuted=True), 20, 3)
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
            ms_p = time_launches(lambda: Ms.spmv_xlds(v0, ys, x_halo=args.x_halo, tile_rows=args.tile_rows,
                                                      y_permuted=True, two_rows=True), 50, 5)
            extra["lanczos"] = {"steps": steps, "ms_per_step_eager": round(ms_l / steps, 5),
                                "ms_per_step_graph": round(ms_g / steps, 5), "ms_product_alone": round(ms_p, 5),
                                "vector_passes_per_step": 6,
                                "GBps_alg_per_step": round((b_alg + 6 * 8 * n) / (ms_g / steps) / 1e6, 1)}
            del Ms, bufs, g
        # host link (eq. 2-4): x to the device, the product, y back, from pinned host memory
        xh = torch.from_numpy(x_np).to(tdt).pin_memory()
        yh = torch.empty(n, dtype=tdt).pin_memory()
        xd2 = torch.empty(n, dtype=tdt, device="cuda")

        def h2d():
            xd2.copy_(xh, non_blocking=True)

        def d2h():
            yh.copy_(y_dev, non_blocking=True)
        ms_h2d = time_launches(h2d, 20, 3)
        ms_d2h = time_launches(d2h, 20, 3)

        def with_link():
            xd2.copy_(xh, non_blocking=True)
            step()
            yh.copy_(y_dev, non_blocking=True)
        ms_link = time_launches(with_link, 20, 3)
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
            "ms_product": round(ms, 5), "ms_product_eq2": round(t_mvm_model * 1e3, 5),
            "ms_transfers_eq2": round(t_pci_model * 1e3, 5), "ms_with_transfers": round(ms_link, 5),
            "transfer_share_measured": round(1 - ms / ms_link, 4),
            "transfer_share_eq2": round(t_pci_model / (t_pci_model + t_mvm_model), 4),
            "eq3_nnzr_max_half_penalty": {"alpha0": round(pmodel.nnzr_bound_half_penalty(ratio, 0.0), 1),
                                          "alpha1": round(pmodel.nnzr_bound_half_penalty(ratio, 1.0), 1)},
            "eq4_nnzr_min_tenth_penalty": {"alpha0": round(pmodel.nnzr_bound_tenth_penalty(ratio, 0.0), 1),
                                           "alpha1": round(pmodel.nnzr_bound_tenth_penalty(ratio, 1.0), 1)}}
        del xh, yh, xd2
        # T lanes per row (block layout, same sort window, x through the caches) on this matrix,
        # and the sliced formats the outlook names: rows sorted only inside each 64-row slice
        # (sliced ELLPACK's padding; with T lanes, sliced ELLR-T's)
        lanes_leg = {}
        for T, sw_l in ((2, args.sort_window), (4, args.sort_window), (8, args.sort_window), (1, 64), (4, 64)):
            Ml = PjdsMatrix.from_csr(A, layout="block", sort_window=sw_l, lanes=T)
            xo = torch.from_numpy(x_np).to("cuda", tdt)
            yl = torch.empty(n, dtype=tdt, device="cuda")
            ms_t = time_launches(lambda: Ml.spmv(xo, yl, y_permuted=True), 50, 5)
            lanes_leg[f"T{T}" if sw_l == args.sort_window else f"sliced_w{sw_l}_T{T}"] = {
                "ms": round(ms_t, 5), "GBps_alg": round(b_alg / ms_t / 1e6, 1), "nnz_stored": Ml.info.nnz_stored}
            del Ml
        extra["lanes_per_row"] = lanes_leg
        # local/non-local split (vector mode with overlap): y written, then read and written again
        from paper_1112_5588_amd.matrix import split_columns
        loc, nl = split_columns(A, 0, A.n_cols // 2)
        ML, MN = PjdsMatrix.from_csr(loc), PjdsMatrix.from_csr(nl)
        M1 = PjdsMatrix.from_csr(A)
        xo = torch.from_numpy(x_np).to("cuda", tdt)
        yo = torch.empty(n, dtype=tdt, device="cuda")

        def split_step():
            ML.spmv(xo, yo)
            MN.spmv_axpby(xo, yo, alpha=1.0, beta=1.0, z=yo)
        ms_split = time_launches(split_step, 30, 3)
        ms_one = time_launches(lambda: M1.spmv(xo, yo), 30, 3)
        from paper_1112_5588_amd import model as pmodel
        nnzr = nnz / n
        extra["split_local_nonlocal"] = {
            "ms_split": round(ms_split, 5), "ms_single": round(ms_one, 5),
            "penalty": round(ms_split / ms_one - 1, 4),
            "model_penalty_eq1": round((8.0 / nnzr) / pmodel.code_balance_dp(1.0 / nnzr, nnzr), 4)}
        del ML, MN, M1
        extra["autotune"] = {"ms": {k: round(v, 5) for k, v in t_all.items()}, "best": best,
                             "best_GBps_alg": round(b_alg / t_all[best] / 1e6, 1),
                             "plain_GBps_alg": round(b_alg / plain / 1e6, 1),
                             "tuned_over_plain": round(plain / t_all[best], 3),
                             "exhaustive_search_s": round(exhaustive_s, 2),
                             "learned": {"pick": learned_pick, "margin": round(float(pick_margin[0]), 4),
                                         "pick_ms": round(t_cat[learned_pick], 5),
                                         "regret_vs_catalog_best": round(t_cat[learned_pick] / min(t_cat.values()) - 1, 4),
                                         "over_plain": round(plain / t_cat[learned_pick], 3),
                                         "tuning_s": round(learned_s, 3)}}
        # the same matrix with FP32 values (values rounded to nearest), headline configuration
        if args.dtype == "f64":
            A32 = A.astype(np.float32)
            M32 = PjdsMatrix.from_csr(A32, block_height=args.block_height, layout=args.layout,
                                      sort_window=args.sort_window)
            x32 = torch.from_numpy(x_np).to("cuda", torch.float32)
            y32 = torch.empty(n, dtype=torch.float32, device="cuda")
            if args.x_halo >= 0:
                ms32 = time_launches(lambda: M32.spmv_xlds(x32, y32, x_halo=args.x_halo, tile_rows=args.tile_rows,
                                                           y_permuted=True, two_rows=args.two_rows), 100, 10)
            else:
                ms32 = time_launches(lambda: M32.spmv(x32, y32, y_permuted=True), 100, 10)
            b32 = 8 * nnz + 8 * n
            extra["fp32"] = {"ms": round(ms32, 5), "GBps_alg": round(b32 / ms32 / 1e6, 1),
                             "gflops": round(2 * nnz / ms32 / 1e6, 2), "alg_bytes": b32}
            del A32, M32, x32, y32
        # the skewed-row workload: global sort vs sort windows 2^10..2^16 (padding and time),
        # several lanes per row, and ELLPACK-R's padded size (planned, not allocated)
        log("power-law leg")
        del M, x_dev, y_dev
        torch.cuda.empty_cache()
        P, _ = make_workload("powerlaw", args.dtype)
        xp = torch.from_numpy(synth.dense_x(P.n_cols, 3)).to("cuda", tdt)
        yp_ = torch.empty(P.n_rows, dtype=tdt, device="cuda")
        bp = (vbytes + 4) * P.nnz + 2 * vbytes * P.n_rows
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
            Mp = PjdsMatrix.from_csr(P, **kw)
            ms_p = time_launches(lambda: Mp.spmv(xp, yp_, y_permuted=True), 20, 3)
            pl[label] = {"ms": round(ms_p, 5), "GBps_alg": round(bp / ms_p / 1e6, 1),
                         "nnz_stored": Mp.info.nnz_stored,
                         "padding": round(Mp.info.nnz_stored / P.nnz - 1, 4)}
            if label == "global_split512":        # cold-cache protocol: x (64 MB) evicted too
                ms_c = cold_median(lambda: Mp.spmv(xp, yp_, y_permuted=True))
                pl[label]["cold_mall_median_ms"] = round(ms_c, 5)
                pl[label]["cold_mall_GBps_alg"] = round(bp / ms_c / 1e6, 1)
            del Mp
        extra["powerlaw"] = pl
        del P, xp, yp_, flush
        result["extra"] = extra
    if not args.no_batch:
        torch.cuda.empty_cache()
        result["batch"] = batch_leg(torch)

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
