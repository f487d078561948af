"""Throughput of the Q-adic transform path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
coefficient bytes in HBM -> DQT pack -> exact FP64 MFMA contraction with
REDQ at K-block boundaries -> REDQ + L/H unpack -> coefficient bytes in HBM.
The default workload is the batch of 4096 uneven GEMMs over GF(3^4)
(X^4+2X^3+2, M, N, K uniform in 16..256, seed 3) in one persistent launch
replayed from a captured hipGraph; `value` is the packed FP64 path, the INT8
path and the plain per-product comparator sit beside it in `paths`.

Prints ONE JSON line.  Before timing, the output is checked bit-exactly:
sampled entries against the CPU oracle, and the whole output against the
other paths (the plain comparator unless --no-plain).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GF(p^k) field mul-adds/sec at bit-exact output, batched FQT vs plain; % roofline"
PEAK_FP64 = 78.6e12      # MI355X dense FP64 (matrix and vector), FLOP/s
PEAK_HBM = 8.0e12        # bytes/s
PEAK_INT8 = 5.0e15       # dense INT8 MFMA, OP/s
PEAK_I32_VALU = 157.3e12 / 2  # 32-bit integer vector ops per second (one per lane per clock)
INFINITY_CACHE_BYTES = 256 << 20  # MI355X's memory-side cache in front of HBM


# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by a plain-copy calibration (profiles/ holds the summary).
# Keyed by (workload, path, tile); valid only for the kernel version profiled.
MEASURED_TRAFFIC = {
    ("gemm-gf7^2-1024", "packed", 7): {
        "bytes": 15_269_888,  # FETCH 6432 KiB x 2.000 + WRITE 2048 KiB x 1.000
        "source": "profiles/gemm_direct_gf7-2_1024.md"},
    ("gemm-gf7^2-1024", "packed", 12): {
        "bytes": 14_993_408,  # FETCH 6297 KiB x 2.000 + WRITE 2048 KiB x 1.000
        "source": "profiles/gemm_direct_gf7-2_1024.md"},
    ("polymul-gf5-k3-2^24", "polymul", "polymul_w32_kernel"): {
        "bytes": 184_602_803,  # FETCH 49178.1 KiB x 2.000 + WRITE 81920.0 KiB x 1.000
        "source": "profiles/polymul_gf5_k3_2-24.md"},
    ("transforms-gf5^3-2^24", "unpack_poly", "unpack_w_kernel<5, 5, false>"): {
        "bytes": 218_159_124,  # FETCH 65562.99 KiB x 2.000 + WRITE 81920.04 KiB x 1.000
        "source": "profiles/transforms_gf5-3_2-24.md"},
    ("dfqt-gf3-n500-d4", "dfqt", 4, 1): {
        "bytes": 34_188_339,  # FETCH 8629.5 KiB x 2.000 + WRITE 16128 KiB x 1.000
        "source": "profiles/dfqt_gf3_n500_d4.md"},
    ("dfqt-gf3-n500-d4", "dfqt", 4, 0): {
        "bytes": 34_159_616,  # FETCH 8615.5 KiB x 2.000 + WRITE 16128 KiB x 1.000
        "source": "profiles/dfqt_gf3_n500_d4.md"},
    ("batched-gf3^4-4096", "packed", 15): {
        "bytes": 1_256_045_087,  # FETCH 454595.3 KiB x 2.000 + WRITE 317415.9 KiB x 1.000
        "source": "profiles/batched_gf3-4_4096.md"},
    ("batched-gf3^4-4096", "int8", 11): {
        "bytes": 1_028_396_073,  # FETCH 330734.4 KiB x 2.000 + WRITE 342824.3 KiB x 1.000
        "source": "profiles/batched_gf3-4_4096.md"},
}


def hbm_rate(alg_bytes, ms, traffic=None):
    """Achieved HBM rates of one step: algorithmic bytes (inputs read once,
    outputs written once) and, where counters were taken, measured bytes."""
    out = {"algorithmic_bytes": int(alg_bytes),
           "algorithmic_GBps": alg_bytes / (ms * 1e-3) / 1e9,
           "measured_bytes": traffic,
           "measured_GBps": traffic / (ms * 1e-3) / 1e9 if traffic else None}
    return out


def poly_str(P_low):
    k = len(P_low)
    terms = [f"X^{k}"]
    for i in range(k - 1, -1, -1):
        c = P_low[i]
        if c:
            terms.append(("" if c == 1 and i else str(c)) + (f"X^{i}" if i > 1 else ("X" if i == 1 else "")))
    return "+".join(terms)


# Default step counts are sized from the step's own duration: the GPU clock
# settles over some milliseconds of sustained load, so a short timed region of
# a ~40 us kernel reads a few per cent slow.
TIMED_MS, WARMUP_MS = 40.0, 20.0


def size_counts(fn, args, torch):
    """Fill in --steps / --warmup when not given: at least 50 timed steps
    covering TIMED_MS and at least 10 warmup steps covering WARMUP_MS."""
    if args.steps is not None and args.warmup is not None:
        return
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    ms = max((time.perf_counter() - t0) * 1e3 / 3, 1e-3)
    if args.steps is None:
        args.steps = int(min(5000, max(50, -(-TIMED_MS // ms))))
    if args.warmup is None:
        args.warmup = int(min(5000, max(10, -(-WARMUP_MS // ms))))


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per step


def host_info():
    """The host the CPU legs ran on: nproc (CPUs this process may use), the
    machine's CPU count and lscpu's model line."""
    info = {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Socket(s)"):
                info["lscpu " + key.strip()] = val.strip()
    except Exception as e:  # lscpu missing: say so rather than guess
        info["lscpu"] = f"unavailable ({type(e).__name__})"
    return info


def cpu_baseline_gemm(w, A, B, gf, target_s=15.0):
    """The oracle as it stands, on a bounded row sample of the same product."""
    rows = 16
    t0 = time.time()
    gf.gemm_gfpk_planes(A[:rows], B, w.p, w.P_low)
    dt = time.time() - t0
    rows = int(max(16, min(A.shape[0], rows * target_s / max(dt, 1e-3))))
    t0 = time.time()
    gf.gemm_gfpk_planes(A[:rows], B, w.p, w.P_low)
    dt = time.time() - t0
    rate = rows * B.shape[1] * A.shape[1] / dt
    return {"value": rate, "unit": "field mul-adds/s", "cores": 1, "kind": "oracle",
            "sample": f"first {rows} rows of A times all of B ({rows}x{B.shape[1]}x{A.shape[1]}), "
                      f"numpy int64 plane products, {dt:.1f} s"}


def _sized_run(fn, units_total, first, target_s, cum=None):
    """Time fn(n) on a bounded prefix: a first run on `first` units sizes a
    second one to about target_s seconds (never more than units_total).
    cum[i], when given, is the work of the first i + 1 units."""
    n = min(first, units_total)
    t0 = time.time()
    fn(n)
    dt = max(time.time() - t0, 1e-3)
    if cum is None:
        n = int(max(n, min(units_total, n * target_s / dt)))
    else:
        want = cum[n - 1] * target_s / dt
        n = int(max(n, min(units_total, np.searchsorted(cum, want) + 1)))
    t0 = time.time()
    out = fn(n)
    return n, time.time() - t0, out


def cpu_plain_gemm(w, A, B, Rh, target_s):
    """The multi-core C schoolbook comparator (oracle/plain_gf.c) on a row
    prefix of the same product; its rows are checked against the GPU's."""
    from oracle import plain_c
    rows, dt, C = _sized_run(lambda r: plain_c.gemm(A[:r], B, w.p, w.P_low), A.shape[0], 16,
                             target_s)
    return {"value": rows * B.shape[1] * A.shape[1] / dt, "unit": "field mul-adds/s",
            "cores": plain_c.threads_used(), "kind": "plain schoolbook, C + OpenMP",
            "sample": f"first {rows} rows of A times all of B, {dt:.1f} s",
            "identical_to_gpu_rows": bool(np.array_equal(C, Rh[:rows]))}


def cpu_batched(w, As, Bs, mnk, gf, target_s):
    """The oracle and the C comparator on a prefix of the batch's products."""
    from oracle import plain_c
    cum = np.cumsum(mnk[:, 0] * mnk[:, 1] * mnk[:, 2])
    out = {}
    n, dt, _ = _sized_run(lambda c: [gf.gemm_gfpk_planes(a, b, w.p, w.P_low)
                                     for a, b in zip(As[:c], Bs[:c])], len(As), 8, target_s,
                          cum)
    out["cpu_baseline"] = {"value": float(cum[n - 1]) / dt, "unit": "field mul-adds/s",
                           "cores": 1, "kind": "oracle",
                           "sample": f"first {n} of the {len(As)} products, numpy int64 plane "
                                     f"products, {dt:.1f} s"}
    n, dt, _ = _sized_run(lambda c: plain_c.gemm_batched(As[:c], Bs[:c], w.p, w.P_low),
                          len(As), 64, min(target_s, 8.0), cum)
    out["cpu_plain"] = {"value": float(cum[n - 1]) / dt, "unit": "field mul-adds/s",
                        "cores": plain_c.threads_used(), "kind": "plain schoolbook, C + OpenMP",
                        "sample": f"first {n} of the {len(As)} products, {dt:.1f} s"}
    return out


# Kernel that carries a packed step, by tile id (1..6 LDS-staged, 7..12 direct).
def packed_kernel_name(tile):
    if tile == 15:
        return ("gemm_wave_batched_kernel, tile 15 (wave-persistent 32 x 32 tiles: DQT by byte "
                "dot products into MFMA registers + FP64 MFMA + digit-sum block steps + L/H)")
    if tile and tile >= 13:
        return (f"gemm_split_kernel, tile {tile} (2-coefficient chunks at q = 2^17, three "
                "FP64 MFMA chunk-pair sums + REDQ_3 + L/H)")
    if tile and tile >= 7:
        return (f"gemm_direct_kernel, tile {tile} (DQT on load into MFMA registers + "
                "FP64 MFMA + REDQ + L/H)")
    return f"gemm_packed_kernel, tile {tile} (DQT into LDS + FP64 MFMA + REDQ + L/H)"


def roofline_for(path, k, work, ms, tile=0):
    """Algorithmic work of one step over its measured time, against the
    published MI355X peak of the unit the path runs on."""
    if path == "int8":
        ops = 2.0 * k * k * work          # k^2 INT8 multiply-adds per field mul-add
        ach = ops / (ms * 1e-3)
        return {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_INT8 / 1e12,
                "unit": "TOP/s", "frac": ach / PEAK_INT8, "traffic": None,
                "kernel": ("gemm_i8cs_batched_kernel, tile 11 (strips of 16 outputs over all "
                           "rows, B' of each K-tile built once in LDS)" if tile == 11 else
                           "gemm_i8f_kernel (B' built in LDS)" if tile >= 4 else
                           "gemm_i8_kernel (+ expand_b_kernel in the step)"),
                "algorithmic": "2 k^2 int8 ops per field mul-add"}
    if path == "plain":
        ops = 2.0 * k * k * work
        ach = ops / (ms * 1e-3)
        return {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_I32_VALU / 1e12,
                "unit": "TOP/s", "frac": ach / PEAK_I32_VALU, "traffic": None,
                "kernel": "gemm_plain_kernel",
                "algorithmic": "2 k^2 integer ops per field mul-add (reductions not counted)"}
    if tile and 13 <= tile <= 14:
        # d-split: three chunk-pair products per field mul-add
        ach = 6.0 * work / (ms * 1e-3)
        return {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP64, "traffic": None,
                "kernel": packed_kernel_name(tile),
                "algorithmic": "6 flop per field mul-add (three FP64 FMAs on packed chunks)"}
    flops = 2.0 * work
    ach = flops / (ms * 1e-3)
    return {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": ach / PEAK_FP64, "traffic": None,
            "kernel": packed_kernel_name(tile),
            "algorithmic": "2 flop per field mul-add (one FP64 FMA on packed values)"}


def bench_gemm(w, args, torch, fqt, gf):
    from paper_0710_0510_amd import workloads as W
    A_h, B_h = W.gemm_inputs(w)
    f = fqt.Field(w.p, w.k, w.P_low)
    A = torch.from_numpy(A_h).cuda()
    B = torch.from_numpy(B_h).cuda()
    q, nqmax = fqt.params(w.p, w.k, 1)
    work = w.M * w.N * w.K

    # reference output of the plain comparator, checked on sampled entries
    Cref = torch.empty((w.M, w.N, w.k), dtype=torch.uint8, device="cuda")
    fqt.gemm(f, A, B, Cref, path="plain")
    torch.cuda.synchronize()
    rng = np.random.default_rng(1234)
    idx = rng.integers(0, [w.M, w.N], size=(args.samples, 2))
    Rh = Cref.cpu().numpy()
    bad = sum(gf.gemm_entry(A_h[i], B_h[:, j], w.p, w.P_low) != Rh[i, j].tolist()
              for i, j in idx.tolist())
    if bad:
        raise SystemExit(f"parity failure: plain path differs from the oracle on {bad} entries")

    paths = [args.path] + [p for p in ("packed", "int8", "plain") if p != args.path and args.all_paths]
    results = {}
    tuned = {}
    def run_path(path, C, opts):
        if path == "winograd":
            return fqt.gemm_winograd(f, A, B, C, levels=args.levels, path="packed", opts=opts)
        return fqt.gemm(f, A, B, C, path=path, opts=opts)

    for path in paths:
        opts = {"tile": args.tile} if (args.tile and path == args.path) else None
        C = torch.empty_like(Cref)
        if path == "winograd" and opts is None:
            # tune the packed path on the block shape of the last level
            m, n, kk = w.M >> args.levels, w.N >> args.levels, w.K >> args.levels
            Cs = torch.empty((m, n, w.k), dtype=torch.uint8, device="cuda")
            opts = fqt.autotune(f, fqt.make_descs(f, [A[:m, :kk]], [B[:kk, :n]], [Cs]),
                                only="packed")[1]
            tuned["winograd_blocks"] = opts
        elif opts is None and path != "plain":
            # autotune this path once, outside the timed region; later calls
            # with opts=None use the tuned (q, tile)
            tuned[path] = fqt.autotune(f, fqt.make_descs(f, [A], [B], [C]), only=path)[1]
        run_path(path, C, opts)
        torch.cuda.synchronize()
        if not torch.equal(C, Cref):
            raise SystemExit(f"parity failure: path {path} differs from the plain path")
        size_counts(lambda: run_path(path, C, opts), args, torch)
        steps = args.steps if path != "plain" else max(3, args.steps // 10)
        ms = time_steps(lambda: run_path(path, C, opts), steps,
                        args.warmup if path != "plain" else 2, torch)
        tile = (opts or tuned.get(path) or {}).get("tile", 0)
        rl = roofline_for("packed" if path == "winograd" else path, w.k, work, ms, tile)
        results[path] = {"value": work / (ms * 1e-3), "ms_per_step": ms, "steps": steps,
                         "tile": tile, "roofline": rl}
        if path == "winograd":
            results[path]["levels"] = args.levels
            rl["kernel"] = (f"Winograd, {args.levels} level(s): 7^{args.levels} products on tile "
                            f"{tile} + block additions (classical flop count)")

    if args.all_paths:
        # the same product on discrete-log codes (Alg. 4's representation):
        # conversions outside the timed region, every log tile that admits K
        Al, Bl, Rl = fqt.to_log(f, A), fqt.to_log(f, B), fqt.to_log(f, Cref)
        Cl = torch.empty_like(Rl)
        best = None
        for tile in (7, 9, 11):
            try:
                fqt.gemm_log(f, Al, Bl, Cl, opts={"tile": tile})
            except fqt.FqtError:
                continue
            torch.cuda.synchronize()
            if not torch.equal(Cl, Rl):
                raise SystemExit(f"parity failure: log tile {tile} differs from the plain path")
            ms = time_steps(lambda: fqt.gemm_log(f, Al, Bl, Cl, opts={"tile": tile}), args.steps,
                            args.warmup, torch)
            if best is None or ms < best[1]:
                best = (tile, ms)
        if best:
            tile, ms = best
            rl = roofline_for("packed", w.k, work, ms, tile)
            rl["kernel"] = f"gemm_direct_kernel on codes, tile {tile} (pack-table lookup + FP64 MFMA + REDQ + L/H codes + Zech)"
            results["log"] = {"value": work / (ms * 1e-3), "ms_per_step": ms, "steps": args.steps,
                              "tile": tile, "roofline": rl}

    if args.all_paths and "packed" in results and "winograd" not in results:
        # Winograd's recursion (the setting of the paper's Fig. 3): 1 and 2
        # levels over the packed path with its tuned tile
        popts = {"tile": results["packed"]["tile"]} if results["packed"]["tile"] else None
        Cw = torch.empty_like(Cref)
        best = None
        for levels in (1, 2):
            fqt.gemm_winograd(f, A, B, Cw, levels=levels, path="packed", opts=popts)
            torch.cuda.synchronize()
            if not torch.equal(Cw, Cref):
                raise SystemExit(f"parity failure: Winograd with {levels} levels differs")
            ms = time_steps(lambda: fqt.gemm_winograd(f, A, B, Cw, levels=levels, path="packed",
                                                      opts=popts),
                            max(3, args.steps // 2), args.warmup, torch)
            if best is None or ms < best[1]:
                best = (levels, ms)
        levels, ms = best
        rl = roofline_for("packed", w.k, work, ms, results["packed"]["tile"])
        rl["kernel"] = (f"Winograd, {levels} level(s): 7^{levels} products on tile "
                        f"{results['packed']['tile']} + block additions (classical flop count)")
        results["winograd"] = {"value": work / (ms * 1e-3), "ms_per_step": ms, "steps": args.steps,
                               "tile": results["packed"]["tile"], "levels": levels, "roofline": rl}

    main_r = results[args.path]
    tr = MEASURED_TRAFFIC.get((w.name, args.path, main_r["tile"]))
    if tr:
        main_r["roofline"]["traffic"] = tr["bytes"]
        main_r["roofline"]["traffic_source"] = tr["source"]
        main_r["roofline"]["algorithmic_bytes"] = (w.M * w.K + w.K * w.N + w.M * w.N) * w.k
    out = {
        "metric": METRIC, "value": main_r["value"], "unit": "field mul-adds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"packed": "f64", "int8": "int8", "plain": "int32", "winograd": "f64"}[args.path],
        "data": "synthetic",
        "config": {"workload": w.name, "field": f"GF({w.p}^{w.k})", "P": poly_str(w.P_low),
                   "M": w.M, "N": w.N, "K": w.K, "seed": w.seed, "path": args.path,
                   "q": q, "n_q_max": nqmax, "tile": args.tile or "autotuned",
                   "tuned": tuned},
        "roofline": main_r["roofline"],
        "paths": {p: {"value": r["value"], "ms_per_step": r["ms_per_step"],
                      "roofline_frac": r["roofline"]["frac"], "unit": "field mul-adds/s",
                      "tile": r["tile"], **({"levels": r["levels"]} if "levels" in r else {})}
                  for p, r in results.items()},
        "parity": {"sampled_entries_vs_oracle": args.samples, "sampled_mismatches": bad,
                   "every_path_identical_to_plain": True},
    }
    if "plain" in results and args.path != "plain":
        out["speedup_vs_plain"] = results["plain"]["ms_per_step"] / main_r["ms_per_step"]
    out["hbm"] = hbm_rate((w.M * w.K + w.K * w.N + w.M * w.N) * w.k, main_r["ms_per_step"],
                          main_r["roofline"].get("traffic"))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_gemm(w, A_h, B_h, gf, target_s=args.cpu_seconds)
        out["cpu_plain"] = cpu_plain_gemm(w, A_h, B_h, Rh, target_s=min(args.cpu_seconds, 8.0))
        out["cpu_baseline"]["host"] = out["cpu_plain"]["host"] = host_info()
    return out


def _aligned_views(torch, arrays, align=256):
    """Pack a list of uint8 arrays into one device buffer; return (buffer,
    list of (offset, shape))."""
    offs, total = [], 0
    for a in arrays:
        offs.append(total)
        total += (a.nbytes + align - 1) // align * align
    host = np.zeros(max(total, 1), dtype=np.uint8)
    for a, o in zip(arrays, offs):
        host[o:o + a.nbytes] = a.reshape(-1)
    return torch.from_numpy(host).cuda(), offs


def bench_batched(w, args, torch, fqt, gf):
    """The metric's workload: 4096 uneven GEMMs in one persistent launch per
    path, replayed from a captured hipGraph.  Checks, before any timing: the
    packed output against the oracle on sampled entries of sampled products,
    and every other path byte for byte against the packed output."""
    from paper_0710_0510_amd import workloads as W
    mnk, As, Bs = W.batched_inputs(w)
    f = fqt.Field(w.p, w.k, w.P_low)
    k = w.k
    dA, offA = _aligned_views(torch, As)
    dB, offB = _aligned_views(torch, Bs)
    Cshapes = [np.zeros((M, N, k), dtype=np.uint8) for (M, N, K) in mnk.tolist()]
    dC, offC = _aligned_views(torch, Cshapes)

    def descs_for(out):
        arr = (fqt.GemmDesc * len(As))()
        for i, (M, N, K) in enumerate(mnk.tolist()):
            arr[i] = fqt.GemmDesc(M, N, K, K, N, N, dA.data_ptr() + offA[i],
                                  dB.data_ptr() + offB[i], out.data_ptr() + offC[i])
        return arr

    dC_descs = descs_for(dC)
    work = int((mnk[:, 0] * mnk[:, 1] * mnk[:, 2]).sum())

    # packed FP64 path: autotuned outside the timed region (or given options)
    tuned = {}
    if args.opts:
        popts = json.loads(args.opts)
    elif args.tile:
        popts = {"tile": args.tile}
    else:
        popts = fqt.autotune(f, dC_descs, only="packed")[1]
    tuned["packed"] = popts
    fqt.gemm_batched(f, dC_descs, path="packed", opts=popts)
    torch.cuda.synchronize()
    Ch = dC.cpu().numpy()
    rng = np.random.default_rng(99)
    bad = 0
    picks = rng.integers(0, len(As), size=args.samples // 4 + 1)
    for g in picks.tolist():
        M, N, K = mnk[g]
        C_g = Ch[offC[g]:offC[g] + M * N * k].reshape(M, N, k)
        for i, j in rng.integers(0, [M, N], size=(4, 2)).tolist():
            bad += gf.gemm_entry(As[g][i], Bs[g][:, j], w.p, w.P_low) != C_g[i, j].tolist()
    if bad:
        raise SystemExit(f"parity failure: batched packed path differs from the oracle on {bad} "
                         "sampled entries")
    size_counts(lambda: fqt.gemm_batched(f, dC_descs, path="packed", opts=popts), args, torch)
    ms = time_steps(lambda: fqt.gemm_batched(f, dC_descs, path="packed", opts=popts),
                    args.steps, args.warmup, torch)
    tile = int(popts.get("tile", 0))

    paths = {"packed": {"value": work / (ms * 1e-3), "ms_per_step": ms, "tile": tile,
                        "roofline_frac": roofline_for("packed", k, work, ms, tile)["frac"]}}
    identical = []
    if "int8" in args.paths:
        # INT8 coefficient-wise path, autotuned, byte-identical to the packed output
        dI = torch.zeros_like(dC)
        dI_descs = descs_for(dI)
        iopts = (json.loads(args.int8_opts) if args.int8_opts
                 else fqt.autotune(f, dI_descs, only="int8")[1])
        tuned["int8"] = iopts
        fqt.gemm_batched(f, dI_descs, path="int8", opts=iopts)
        torch.cuda.synchronize()
        if not torch.equal(dI, dC):
            raise SystemExit("parity failure: batched INT8 path differs from the packed path")
        i8_ms = time_steps(lambda: fqt.gemm_batched(f, dI_descs, path="int8", opts=iopts),
                           args.steps, args.warmup, torch)
        del dI
        paths["int8"] = {"value": work / (i8_ms * 1e-3), "ms_per_step": i8_ms,
                         "tile": int(iopts.get("tile", 0)),
                         "roofline_frac": roofline_for("int8", k, work, i8_ms,
                                                       int(iopts.get("tile", 0)))["frac"]}
        tr8 = MEASURED_TRAFFIC.get((w.name, "int8", int(iopts.get("tile", 0))))
        if tr8:
            paths["int8"]["traffic"] = tr8["bytes"]
            paths["int8"]["traffic_source"] = tr8["source"]
        identical.append("int8")
    if "plain" in args.paths and not args.no_plain:
        # the plain comparator: one launch per product, as the metric asks
        dR = torch.zeros_like(dC)
        dR_descs = descs_for(dR)
        fqt.gemm_batched(f, dR_descs, path="plain")
        torch.cuda.synchronize()
        if not torch.equal(dR, dC):
            raise SystemExit("parity failure: the plain comparator differs from the packed path")
        identical.append("plain")
        plain_ms = time_steps(lambda: fqt.gemm_batched(f, dR_descs, path="plain"),
                              max(2, args.steps // 10), 1, torch)
        paths["plain"] = {"value": work / (plain_ms * 1e-3), "ms_per_step": plain_ms,
                          "launches_per_step": len(As),
                          "roofline_frac": roofline_for("plain", k, work, plain_ms)["frac"]}
    q, nqmax = fqt.params(w.p, w.k, 1)
    rl = roofline_for("packed", k, work, ms, tile)
    rl["kernel"] = "persistent batched " + rl["kernel"]
    alg_bytes = int(((mnk[:, 0] * mnk[:, 2] + mnk[:, 2] * mnk[:, 1]
                      + mnk[:, 0] * mnk[:, 1]) * k).sum())
    tr = MEASURED_TRAFFIC.get((w.name, "packed", tile))
    if tr:
        rl["traffic"] = tr["bytes"]
        rl["traffic_source"] = tr["source"]
        rl["algorithmic_bytes"] = alg_bytes
    out = {
        "metric": METRIC, "value": work / (ms * 1e-3), "unit": "field mul-adds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "field": f"GF({w.p}^{w.k})", "P": poly_str(w.P_low),
                   "count": len(As), "MNK_range": [w.lo, w.hi], "sum_MNK": work, "seed": w.seed,
                   "path": "packed (persistent, hipGraph replay)", "q_max": q, "n_q_max": nqmax,
                   "tile": args.tile or ("given" if args.opts else "autotuned"),
                   "tuned": tuned},
        "roofline": rl,
        "paths": paths,
        "parity": {"sampled_entries_vs_oracle": int(len(picks) * 4), "sampled_mismatches": bad,
                   "identical_to_packed": identical},
    }
    if "plain" in paths:
        out["speedup_vs_plain"] = paths["plain"]["ms_per_step"] / ms
    out["hbm"] = hbm_rate(alg_bytes, ms, rl.get("traffic"))
    if not args.no_cpu:
        out.update(cpu_batched(w, As, Bs, mnk, gf, args.cpu_seconds))
        out["cpu_baseline"]["host"] = out["cpu_plain"]["host"] = host_info()
    return out


def bench_polymul(w, args, torch, fqt, gf):
    from paper_0710_0510_amd import workloads as W
    a_h, b_h = W.polymul_inputs(w)
    a, b = torch.from_numpy(a_h).cuda(), torch.from_numpy(b_h).cuda()
    c = fqt.polymul_batch(w.p, w.k, w.q, a, b)
    torch.cuda.synchronize()
    want = gf.polymul_batch(a_h, b_h, w.p)
    if not np.array_equal(c.cpu().numpy(), want):
        raise SystemExit("parity failure: polymul differs from the oracle")
    nbytes = w.n * (2 * w.k + 2 * w.k - 1)
    # One step's buffers (185 MB at 2^24 pairs) fit in the 256 MB Infinity
    # Cache behind L2, so replaying one set would time cache hits: the timed
    # steps cycle through enough sets (copies of the same inputs) that the
    # cache cannot hold them; the one-set time is reported beside it.
    sets = rotating_sets(
        lambda i: (a, b, c) if i == 0 else (a.clone(), b.clone(), torch.empty_like(c)), nbytes,
        args)
    nsets = len(sets)
    ms, ms_one_set = time_rotating(
        lambda x, y, z: fqt.polymul_batch(w.p, w.k, w.q, x, y, out=z), sets, args, torch)
    torch.cuda.synchronize()
    for x, y, z in sets[1:]:
        if not torch.equal(z, c):
            raise SystemExit("parity failure: polymul output differs between buffer sets")
    work = w.n * w.k * w.k
    ach = nbytes / (ms * 1e-3)
    # the launcher's choice: whole 32-bit words when q = 2^b, (2k-1) b <= 32
    # and every buffer is word-aligned (torch allocations are)
    b_q = w.q.bit_length() - 1
    kern = ("polymul_w32_kernel" if w.q == 1 << b_q and (2 * w.k - 1) * b_q <= 32
            else "polymul_k_kernel")
    cpu = {}
    if not args.no_cpu:
        from oracle import plain_c
        t0 = time.time()
        gf.polymul_batch(a_h, b_h, w.p)
        dt = max(time.time() - t0, 1e-6)
        cpu["cpu_baseline"] = {"value": work / dt, "unit": "GF(p) mul-adds/s", "cores": 1,
                               "kind": "oracle", "sample": f"all {w.n} products, numpy int64, "
                                                           f"{dt:.3f} s"}
        t0 = time.time()
        cp = plain_c.polymul_batch(a_h, b_h, w.p)
        dt = max(time.time() - t0, 1e-6)
        cpu["cpu_plain"] = {"value": work / dt, "unit": "GF(p) mul-adds/s",
                            "cores": plain_c.threads_used(), "kind": "plain schoolbook, C + OpenMP",
                            "sample": f"all {w.n} products, {dt:.3f} s",
                            "identical_to_gpu": bool(np.array_equal(cp, c.cpu().numpy()))}
    return {
        "metric": METRIC, "value": work / (ms * 1e-3), "unit": "GF(p) mul-adds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "p": w.p, "k": w.k, "q": w.q, "n": w.n, "seed": w.seed},
        "products_per_s": w.n / (ms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": ach / PEAK_HBM,
                     "traffic": (MEASURED_TRAFFIC.get((w.name, "polymul", kern)) or {}).get("bytes"),
                     "kernel": f"{kern}<{w.k}>",
                     "algorithmic": f"{2 * w.k} B in + {2 * w.k - 1} B out per product"},
        "buffer_sets": nsets,
        "one_set_ms_per_step": ms_one_set,
        "parity": {"full_output_vs_oracle": True},
        **cpu,
    }


def rotating_sets(make, nbytes, args):
    """Buffer sets for a streaming leg: enough copies that the timed steps
    cycle through more than four times the Infinity Cache (one step's
    buffers would otherwise be served partly from that cache), at most 64:
    a step small enough to need more is bound by its launch, not by HBM."""
    nsets = args.rotate or min(64, max(2, -(-4 * INFINITY_CACHE_BYTES // nbytes)))
    return [make(i) for i in range(nsets)]


def time_rotating(call, sets, args, torch):
    """ms per step over the buffer sets in turn, and over the first set alone."""
    turn = [0]

    def step():
        call(*sets[turn[0]])
        turn[0] = (turn[0] + 1) % len(sets)

    for _ in range(len(sets)):  # every set's output written before the timed steps
        step()
    size_counts(step, args, torch)
    ms = time_steps(step, args.steps, args.warmup, torch)
    ms_one = time_steps(lambda: call(*sets[0]), args.steps, args.warmup, torch)
    return ms, ms_one


def bench_transforms(w, args, torch, fqt, gf):
    """The boundary's standalone transforms on n elements: REDQ unpack of
    binary64 values with 2k-1 base-q digits to polynomial digits (Alg. 2 and
    the Q_d correction; `value`), the same values to field elements (L + H,
    Thm. 3), and the DQT pack of coefficient bytes (eq. (1)).  Bytes per
    element: 8 in + 2k-1 out, 8 in + k out, k in + 8 out."""
    from paper_0710_0510_amd import workloads as W
    c_h, r_h = W.transform_inputs(w)
    f = fqt.Field(w.p, w.k, w.P_low)
    nd = 2 * w.k - 1
    c, r = torch.from_numpy(c_h).cuda(), torch.from_numpy(r_h).cuda()
    poly = fqt.unpack_redq(f, w.q, r, nd, fqt.UNPACK_POLY)
    field = fqt.unpack_redq(f, w.q, r, nd, fqt.UNPACK_FIELD)
    packed = fqt.pack(f, w.q, c)
    torch.cuda.synchronize()
    # parity on a sample of every leg against the oracle's definitions
    rng = np.random.default_rng(99)
    idx = rng.integers(0, w.n, size=max(64, 16 * args.samples))
    idx[:2] = [0, w.n - 1]
    poly_h, field_h, packed_h = poly.cpu().numpy(), field.cpu().numpy(), packed.cpu().numpy()
    bad = 0
    for i in idx.tolist():
        dg = gf.dqt_inverse(int(r_h[i]), w.q, nd, w.p)
        bad += poly_h[i].tolist() != dg
        bad += field_h[i].tolist() != gf.poly_rem(dg, w.P_low, w.p)
        bad += float(packed_h[i]) != float(gf.dqt(c_h[i].tolist(), w.q))
    if bad:
        raise SystemExit(f"parity failure: {bad} sampled transform outputs differ from the oracle")
    b_q = w.q.bit_length() - 1
    pow2 = w.q == 1 << b_q
    legs = {
        "unpack_poly": (8 + nd, r, poly,
                        lambda x, y: fqt.unpack_redq(f, w.q, x, nd, fqt.UNPACK_POLY, out=y),
                        f"unpack_w_kernel<{nd}, {nd}, false>" if pow2 else "unpack_kernel<false>"),
        "unpack_field": (8 + w.k, r, field,
                         lambda x, y: fqt.unpack_redq(f, w.q, x, nd, fqt.UNPACK_FIELD, out=y),
                         f"unpack_w_kernel<{nd}, {w.k}, true>" if pow2 else "unpack_kernel<false>"),
        "pack": (w.k + 8, c, packed, lambda x, y: fqt.pack(f, w.q, x, out=y),
                 f"pack_w_kernel<{w.k}>" if pow2 else "pack_kernel"),
    }
    res = {}
    for name, (eb, x0, y0, call, kern) in legs.items():
        sets = rotating_sets(lambda i: (x0, y0) if i == 0 else (x0.clone(), torch.empty_like(y0)),
                             w.n * eb, args)
        ms, ms_one = time_rotating(call, sets, args, torch)
        torch.cuda.synchronize()
        for x, y in sets[1:]:
            if not torch.equal(y, y0):
                raise SystemExit(f"parity failure: {name} output differs between buffer sets")
        gbps = w.n * eb / (ms * 1e-3) / 1e9
        res[name] = {"ms_per_step": ms, "values_per_s": w.n / (ms * 1e-3), "GBps": gbps,
                     "roofline_frac": gbps * 1e9 / PEAK_HBM, "bytes_per_value": eb,
                     "buffer_sets": len(sets), "one_set_ms_per_step": ms_one, "kernel": kern}
        del sets
    main_r = res.pop("unpack_poly")
    ms = main_r["ms_per_step"]
    ach = w.n * (8 + nd) / (ms * 1e-3)
    kern = main_r["kernel"]
    return {
        "metric": "REDQ unpack values/s (boundary transform, binary64 in, 2k-1 digits out)",
        "value": w.n / (ms * 1e-3), "unit": "values/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "p": w.p, "k": w.k, "q": w.q, "n": w.n, "seed": w.seed,
                   "ndigits": nd},
        "roofline": {"bound": "hbm", "achieved": ach / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": ach / PEAK_HBM,
                     "traffic": (MEASURED_TRAFFIC.get((w.name, "unpack_poly", kern)) or {}).get(
                         "bytes"),
                     "kernel": kern,
                     "algorithmic": f"8 B in + {nd} B out per value"},
        "buffer_sets": main_r["buffer_sets"],
        "one_set_ms_per_step": main_r["one_set_ms_per_step"],
        "paths": res,
        "parity": {"sampled_values_vs_oracle": int(len(idx)), "legs": 3},
    }


def bench_dfqt(w, args, torch, fqt, gf):
    """d-FQT products of long polynomials (Section 6) against the classical
    product with delayed reduction (eq. (3)); work = count * len^2 GF(p)
    mul-adds (the classical count, the same for every method)."""
    from paper_0710_0510_amd import workloads as W
    a_h, b_h = W.poly_long_inputs(w)
    a, b = torch.from_numpy(a_h).cuda(), torch.from_numpy(b_h).cuda()
    ref = fqt.polymul_delayed(w.p, a, b)
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    picks = rng.integers(0, w.count, size=max(4, args.samples // 16))
    ref_h = ref.cpu().numpy()
    bad = sum(gf.polymul_long(a_h[i].tolist(), b_h[i].tolist(), w.p) != ref_h[i].tolist()
              for i in picks.tolist())
    if bad:
        raise SystemExit(f"parity failure: the delayed comparator differs from the oracle on {bad}")
    work = w.count * w.length * w.length
    variants = {}
    for d in sorted({w.d, 1, 2, 3}):
        for cen in ((0, 1) if w.p % 2 else (0,)):
            out = fqt.polymul_dfqt(w.p, d, a, b, centered=cen)
            torch.cuda.synchronize()
            if not torch.equal(out, ref):
                raise SystemExit(f"parity failure: d-FQT with d = {d}, centered = {cen} differs "
                                 "from the comparator")
            size_counts(lambda: fqt.polymul_dfqt(w.p, d, a, b, out=out, centered=cen), args,
                        torch)
            ms = time_steps(lambda: fqt.polymul_dfqt(w.p, d, a, b, out=out, centered=cen),
                            args.steps, args.warmup, torch)
            nch = -(-w.length // (d + 1))
            fl = 2.0 * w.count * nch * nch / (ms * 1e-3)  # one FP64 FMA per chunk product
            q, nq = gf.max_pow2_q(w.p, d + 1)
            if cen:
                nq = gf.centred_nq_max(w.p, d + 1, q)
            variants[(d, cen)] = {"value": work / (ms * 1e-3), "ms_per_step": ms, "q": q,
                                  "n_q": nq, "chunks": nch, "fp64_tflops": fl / 1e12,
                                  "centered": cen}
    dms = time_steps(lambda: fqt.polymul_delayed(w.p, a, b, out=ref), args.steps, args.warmup,
                     torch)
    # the workload's d, with the faster of the two chunk representations
    main_key = min((key for key in variants if key[0] == w.d),
                   key=lambda key: variants[key]["ms_per_step"])
    main_v = variants[main_key]
    out = {
        "metric": METRIC, "value": main_v["value"], "unit": "GF(p) mul-adds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_v["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "p": w.p, "degree": w.length - 1, "d": w.d,
                   "count": w.count, "seed": w.seed, "q": main_v["q"], "n_q": main_v["n_q"],
                   "centered": main_v["centered"]},
        "products_per_s": w.count / (main_v["ms_per_step"] * 1e-3),
        "roofline": {"bound": "alu", "achieved": main_v["fp64_tflops"], "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": main_v["fp64_tflops"] * 1e12 / PEAK_FP64,
                     "traffic": None, "kernel": "dfqt_kernel (DQT + FP64 FMA convolution + "
                     "block digits + overlap-add)",
                     "algorithmic": "2 flop per product of packed chunks, ceil(len/(d+1))^2 "
                                    "per polynomial product"},
        "paths": {f"dfqt_d{d}" + ("_centred" if cen else ""):
                  {"value": v["value"], "ms_per_step": v["ms_per_step"], "q": v["q"],
                   "n_q": v["n_q"]} for (d, cen), v in variants.items()},
        "comparator": {"kind": "classical, delayed reduction (eq. (3))",
                       "value": work / (dms * 1e-3), "ms_per_step": dms},
        "speedup_vs_delayed": dms / main_v["ms_per_step"],
        "parity": {"sampled_products_vs_oracle": int(len(picks)), "sampled_mismatches": bad,
                   "every_d_identical_to_comparator": True},
    }
    tr = MEASURED_TRAFFIC.get((w.name, "dfqt", w.d, main_v["centered"]))
    if tr:
        out["roofline"]["traffic"] = tr["bytes"]
        out["roofline"]["traffic_source"] = tr["source"]
        out["roofline"]["algorithmic_bytes"] = w.count * (2 * w.length + 2 * w.length - 1)
    out["hbm"] = hbm_rate(w.count * (2 * w.length + 2 * w.length - 1), main_v["ms_per_step"],
                          out["roofline"].get("traffic"))
    if not args.no_cpu:
        n = 4
        t0 = time.time()
        for i in range(n):
            gf.polymul_long(a_h[i].tolist(), b_h[i].tolist(), w.p)
        dt = max(time.time() - t0, 1e-6)
        n = int(max(4, min(w.count, n * args.cpu_seconds / dt)))
        t0 = time.time()
        for i in range(n):
            gf.polymul_long(a_h[i].tolist(), b_h[i].tolist(), w.p)
        dt = time.time() - t0
        out["cpu_baseline"] = {"value": n * w.length * w.length / dt, "unit": "GF(p) mul-adds/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"first {n} of the {w.count} products, numpy int64 "
                                         f"convolution, {dt:.1f} s"}
    return out


def bench_dfqt_batched(w, args, torch, fqt, gf):
    """d-FQT over a batch of uneven pairs (Section 6) in one persistent
    launch replayed from a captured graph; work = sum of la lb GF(p)
    mul-adds (the classical count).  Beside it, the same pairs padded to the
    longest length through the equal-length d-FQT and through the classical
    product with delayed reduction (eq. (3)), the comparator."""
    from paper_0710_0510_amd import workloads as W
    lens, a_h, b_h = W.poly_uneven_inputs(w)
    la, lb = lens[:, 0], lens[:, 1]
    lc = la + lb - 1
    oa = np.concatenate(([0], np.cumsum(la)))
    ob = np.concatenate(([0], np.cumsum(lb)))
    oc = np.concatenate(([0], np.cumsum(lc)))
    a, b = torch.from_numpy(a_h).cuda(), torch.from_numpy(b_h).cuda()
    c = torch.empty(int(lc.sum()), dtype=torch.uint8, device="cuda")
    descs = fqt.poly_descs_flat(a, b, c, lens)
    work = int((la * lb).sum())
    hi = int(lens.max())
    # the padded comparator's operands, built on the host by index arrays
    rows_a, rows_b = np.repeat(np.arange(w.count), la), np.repeat(np.arange(w.count), lb)
    A = np.zeros((w.count, hi), np.uint8)
    B = np.zeros((w.count, hi), np.uint8)
    A[rows_a, np.arange(len(a_h)) - np.repeat(oa[:-1], la)] = a_h
    B[rows_b, np.arange(len(b_h)) - np.repeat(ob[:-1], lb)] = b_h
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = fqt.polymul_delayed(w.p, Ad, Bd)
    # positions of every batch output inside the padded rows
    gather = torch.from_numpy(np.repeat(np.arange(w.count) * (2 * hi - 1) - oc[:-1], lc)
                              + np.arange(int(lc.sum()))).cuda()
    ref_flat = ref.view(-1)[gather]
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    picks = rng.integers(0, w.count, size=max(4, args.samples // 16)).tolist()
    ref_h = ref_flat.cpu().numpy()
    bad = sum(gf.polymul_long(a_h[oa[i]:oa[i + 1]].tolist(), b_h[ob[i]:ob[i + 1]].tolist(), w.p)
              != ref_h[oc[i]:oc[i + 1]].tolist() for i in picks)
    if bad:
        raise SystemExit(f"parity failure: the delayed comparator differs from the oracle on {bad}")

    def chunk_products(d):
        ke = d + 1
        return int((((la + ke - 1) // ke) * ((lb + ke - 1) // ke)).sum())

    variants = {}
    for d in range(8):
        for cen in ((0, 1) if w.p % 2 else (0,)):
            fn = lambda: fqt.polymul_dfqt_batched(w.p, d, descs, centered=cen)
            c.fill_(0xEE)
            try:
                fn()
            except fqt.FqtError as e:  # eq. (2) admits no q for this chunk length
                if e.name in ("FQT_ERR_BOUNDS", "FQT_ERR_UNSUPPORTED"):
                    continue
                raise
            torch.cuda.synchronize()
            if not torch.equal(c, ref_flat):
                raise SystemExit(f"parity failure: batched d-FQT with d = {d}, centered = {cen} "
                                 "differs from the comparator")
            size_counts(fn, args, torch)
            ms = time_steps(fn, args.steps, args.warmup, torch)
            fl = 2.0 * chunk_products(d) / (ms * 1e-3)
            variants[(d, cen)] = {"value": work / (ms * 1e-3), "ms_per_step": ms,
                                  "fp64_tflops": fl / 1e12, "centered": cen}
    tuned = fqt.autotune_polymul(w.p, descs)
    # the padded equal-length d-FQT and the comparator, at the workload's d
    cen_w = min((key for key in variants if key[0] == w.d),
                key=lambda key: variants[key]["ms_per_step"])[1]
    pad_out = fqt.polymul_dfqt(w.p, w.d, Ad, Bd, centered=cen_w)
    torch.cuda.synchronize()
    if not torch.equal(pad_out, ref):
        raise SystemExit("parity failure: padded d-FQT differs from the comparator")
    pms = time_steps(lambda: fqt.polymul_dfqt(w.p, w.d, Ad, Bd, out=pad_out, centered=cen_w),
                     args.steps, args.warmup, torch)
    dms = time_steps(lambda: fqt.polymul_delayed(w.p, Ad, Bd, out=ref), args.steps, args.warmup,
                     torch)
    # the autotuner's choice, timed as it was chosen (its block-boundary mode too)
    main_key = (tuned["d"], tuned["centered"])
    fn = lambda: fqt.polymul_dfqt_batched(w.p, main_key[0], descs, centered=main_key[1],
                                          boundary=tuned["boundary"])
    c.fill_(0xEE)
    fn()
    torch.cuda.synchronize()
    if not torch.equal(c, ref_flat):
        raise SystemExit(f"parity failure: batched d-FQT {tuned} differs")
    ms = time_steps(fn, args.steps, args.warmup, torch)
    main_v = {"value": work / (ms * 1e-3), "ms_per_step": ms,
              "fp64_tflops": 2.0 * chunk_products(main_key[0]) / (ms * 1e-3) / 1e12,
              "centered": main_key[1]}
    out = {
        "metric": METRIC, "value": main_v["value"], "unit": "GF(p) mul-adds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_v["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "p": w.p, "count": w.count, "lengths": f"{w.lo}..{w.hi}",
                   "seed": w.seed, "d": main_key[0], "centered": main_key[1],
                   "boundary": tuned["boundary"], "autotuned": True},
        "products_per_s": w.count / (main_v["ms_per_step"] * 1e-3),
        "roofline": {"bound": "alu", "achieved": main_v["fp64_tflops"], "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": main_v["fp64_tflops"] * 1e12 / PEAK_FP64,
                     "traffic": None, "kernel": "dfqt_batched_kernel (queue of uneven pairs: "
                     "DQT + FP64 FMA convolution + block digits + overlap-add)",
                     "algorithmic": "2 flop per product of packed chunks, "
                                    "ceil(la/(d+1)) ceil(lb/(d+1)) per pair"},
        "paths": {**{f"dfqt_batched_d{d}" + ("_centred" if cen else ""):
                     {"value": v["value"], "ms_per_step": v["ms_per_step"]}
                     for (d, cen), v in variants.items()},
                  f"dfqt_padded_d{w.d}": {"value": work / (pms * 1e-3), "ms_per_step": pms,
                                         "padded_to": hi},
                  "delayed_padded": {"value": work / (dms * 1e-3), "ms_per_step": dms,
                                     "padded_to": hi}},
        "comparator": {"kind": "classical, delayed reduction (eq. (3)), pairs padded to "
                               f"{hi} coefficients", "value": work / (dms * 1e-3),
                       "ms_per_step": dms},
        "speedup_vs_delayed": dms / main_v["ms_per_step"],
        "speedup_vs_padded_dfqt": pms / main_v["ms_per_step"],
        "parity": {"sampled_products_vs_oracle": len(picks), "sampled_mismatches": bad,
                   "every_variant_identical_to_comparator": True},
    }
    out["hbm"] = hbm_rate(int(la.sum() + lb.sum() + lc.sum()), main_v["ms_per_step"], None)
    if not args.no_cpu:
        n = 16
        t0 = time.time()
        for i in range(n):
            gf.polymul_long(a_h[oa[i]:oa[i + 1]].tolist(), b_h[ob[i]:ob[i + 1]].tolist(), w.p)
        dt = max(time.time() - t0, 1e-6)
        n = int(max(16, min(w.count, n * args.cpu_seconds / dt)))
        t0 = time.time()
        for i in range(n):
            gf.polymul_long(a_h[oa[i]:oa[i + 1]].tolist(), b_h[ob[i]:ob[i + 1]].tolist(), w.p)
        dt = time.time() - t0
        out["cpu_baseline"] = {"value": int((la[:n] * lb[:n]).sum()) / dt,
                               "unit": "GF(p) mul-adds/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {n} of the {w.count} pairs, numpy int64 "
                                         f"convolution, {dt:.1f} s", "host": host_info()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: >= 50, covering %g ms)" % TIMED_MS)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warmup steps (default: >= 10, covering %g ms)" % WARMUP_MS)
    ap.add_argument("--workload", default="batched-gf3^4-4096")
    ap.add_argument("--path", default="packed", choices=["packed", "int8", "plain", "winograd"])
    ap.add_argument("--levels", type=int, default=2,
                    help="levels of Winograd's recursion for --path winograd")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--all-paths", type=int, default=1, help="also time the other paths")
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched: leave out the plain per-product comparator (4096 launches), "
                         "e.g. under a counter-collecting profiler")
    ap.add_argument("--paths", default="packed,int8,plain",
                    help="batched: the paths to run beside the packed one (comma list of "
                         "int8, plain)")
    ap.add_argument("--opts", default=None,
                    help="batched: JSON options of the packed path instead of autotuning")
    ap.add_argument("--int8-opts", default=None,
                    help="batched: JSON options of the INT8 path instead of autotuning")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--rotate", type=int, default=0, metavar="SETS",
                    help="streaming workloads (polymul, transforms): buffer sets cycled by the timed steps "
                         "(0: enough to exceed 4x the Infinity Cache)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a "
                                   "design note, not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from oracle import gf  # the CPU-baseline leg and the parity check
    from paper_0710_0510_amd import fqt
    from paper_0710_0510_amd import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)
        return
    fqt.lib()
    w = W.WORKLOADS[args.workload]
    if w.kind == "gemm":
        out = bench_gemm(w, args, torch, fqt, gf)
    elif w.kind == "dfqt":
        out = bench_dfqt(w, args, torch, fqt, gf)
    elif w.kind == "dfqt_batched":
        out = bench_dfqt_batched(w, args, torch, fqt, gf)
    elif w.kind == "batched":
        out = bench_batched(w, args, torch, fqt, gf)
    elif w.kind == "transforms":
        out = bench_transforms(w, args, torch, fqt, gf)
    else:
        out = bench_polymul(w, args, torch, fqt, gf)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
