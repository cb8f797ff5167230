#!/usr/bin/env python3
"""Throughput of the TDB in situ compressor on one MI355X.

Workload (default): the reactive-flow-shaped stream, a 512 x 256 x 8 FP32 tensor
(3 advected plumes with reaction fronts, 8 Arrhenius-scaled variables, 1e-6 noise),
dt 5e-4, adaptive ranks from the rank rule with error threshold 1e-4 and caps
(64, 64, 8). One step = one snapshot ingested: two Heun stages of the projection
pass, the small FP64 work, the re-orthonormalisation, the weighted error pass and
the controller (with any HOSVD reinitialisation it triggers).

All snapshots of the run are generated on the device before timing (a ring far
larger than the 256 MB last-level cache), so every stage pass streams its snapshot
pair from HBM at least once. Prints one JSON line.

Besides the headline line, the same JSON carries: the same stream with the stage
pass in BF16-split products ("bf16_split"); the batched ensemble of independent
Fourier-mode streams of uneven grids ("ensemble", 256 streams by default, one batch
step = one snapshot of every stream); the plain FP64 GPU path; and the CPU oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
# HBM bytes per stage-pass launch from hardware counters (FETCH_SIZE / WRITE_SIZE,
# calibrated against a copy of known size); ignored once the kernel's sources change.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage_pass_plume512x256x8_fp32.txt")
PROFILE_EVERY = 8          # pass timing sampled on every 8th step of the timed run
ENSEMBLE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ensemble256_fp32.txt")
METRIC = "snapshots/s ingested + HBM GB/s vs plain FP64 GPU at <=1e-6 rel err"


def _workload(args):
    from streams import plume_spec
    sp = plume_spec(steps=args.warmup + args.steps + 1)
    desc = {"workload": "plume-512x256x8-fp32 (reactive-flow-shaped stream)",
            "dims": list(sp.dims), "dt": sp.dt, "eps_th": sp.eps_th, "rank_max": [64, 64, 8],
            "adaptive": True, "snapshot_storage": "f32", "noise": 1e-6}
    return sp, desc


def _make_snapshots(sp, n, device):
    import torch
    out = []
    for k in range(n):
        out.append(sp.snapshot(k, device=device))
    torch.cuda.synchronize()
    return out


def _run_gpu(sp, snaps, warmup, steps, precision, path, profile=True):
    import torch
    from paper_2201_06958_amd import Compressor
    cmp = Compressor(sp.dims, sp.dt, rank_max=(64, 64, 8), weights=sp.weights, data_dtype="f32",
                     precision=precision, path=path, adaptive=True, snapshot_mode="borrow",
                     eps_th=sp.eps_th)
    cmp.init(snaps[0])
    for k in range(1, warmup + 1):
        cmp.ingest(snaps[k])
    cmp.flush()
    torch.cuda.synchronize()
    if profile:
        # the dispatch-stamped events cost time on the stream: the passes of every
        # PROFILE_EVERY-th step are timed (a sample spread over the timed region)
        cmp.profile_enable(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        cmp.ingest(snaps[k])
    cmp.flush()   # the last step's decision is acted on inside the timed region
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = cmp.stats()
    prof = {}
    if profile:
        prof = {"project": cmp.profile_read("project"), "error": cmp.profile_read("error")}
    cmp.close()
    return t1 - t0, st, prof


def _run_ensemble(n, warmup, steps, precision="f32"):
    """The batched ensemble: n Fourier-mode streams of grids from {128,192,256}^2 x 4,
    caps 24, threshold 1e-5, one batch step per snapshot of every stream."""
    import torch
    from streams import fourier_ensemble_specs
    from paper_2201_06958_amd import Batch
    specs = fourier_ensemble_specs(n_streams=n, steps=warmup + steps + 1)
    snaps = [[sp.snapshot(k, device="cuda") for sp in specs] for k in range(warmup + steps + 1)]
    torch.cuda.synchronize()
    elems = sum(sp.dims[0] * sp.dims[1] * sp.dims[2] for sp in specs)
    cfgs = [dict(dims=sp.dims, dt=sp.dt, rank_max=sp.rank_max, weights=sp.weights, data_dtype="f32",
                 precision=precision, adaptive=True, eps_th=sp.eps_th, snapshot_mode="borrow") for sp in specs]
    b = Batch(cfgs).init(snaps[0])
    for k in range(1, warmup + 1):
        b.ingest(snaps[k])
    torch.cuda.synchronize()
    b.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        b.ingest(snaps[k])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pj, er = b.profile_read("project"), b.profile_read("error")
    pav = pj["total_ms"] / max(pj["launches"], 1) * 1e-3
    eav = er["total_ms"] / max(er["launches"], 1) * 1e-3
    ranks = [b.streams[i].ranks() for i in range(n)]
    b.close()
    step_bytes = 5.0 * 4.0 * elems   # two stage passes over two snapshots, one error pass
    traffic = None
    if precision == "f32" and n == 256:
        from paper_2201_06958_amd.profsum import read_pass_traffic
        traffic = read_pass_traffic(ENSEMBLE_TRAFFIC_FILE, "kb_mpass<float, 1>")
    return {"workload": f"fourier-ensemble-{n}x{{128,192,256}}^2x4-fp32", "streams": n, "steps": steps,
            "precision": precision, "elements_per_step": elems,
            "value": n * steps / el, "unit": "snapshots/s", "ms_per_step": 1e3 * el / steps,
            "step_hbm_frac": step_bytes / (el / steps) / (HBM_PEAK_GBS * 1e9),
            "pass": {"avg_launch_us": pav * 1e6, "achieved_GBs": pj["bytes_per_launch"] / pav / 1e9,
                     "frac": pj["bytes_per_launch"] / pav / 1e9 / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": pj["bytes_per_launch"],
                     "traffic": traffic["traffic_bytes"] if traffic else None,
                     "traffic_read_write": [traffic["read_bytes"], traffic["write_bytes"]] if traffic else None},
            "error_pass": {"avg_launch_us": eav * 1e6, "achieved_GBs": er["bytes_per_launch"] / eav / 1e9},
            "max_ranks": [max(r[i] for r in ranks) for i in range(3)]}


def _cpu_baseline(sp, start, budget_s=15.0, max_steps=60):
    """The FP64 numpy oracle on the host: init at snapshot `start`, then as many
    steps as fit in the budget (bounded sample of the same workload)."""
    import numpy as np
    from oracle import tdb_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(64, 64, 8),
                         rank_init=None, adaptive=True, eps_th=sp.eps_th)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(start).astype(np.float64), t0=sp.time(start))
    n = 0
    t0 = time.perf_counter()
    while n < max_steps and time.perf_counter() - t0 < budget_s:
        o.ingest(sp.snapshot_np(start + 1 + n).astype(np.float64))
        n += 1
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "snapshots/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} consecutive steps of the same stream after an HOSVD init at step {start} "
                      f"(FP64 numpy oracle, {el:.1f} s, snapshot generation excluded)"}


def _scaling_sweep(sizes, steps, reps=5):
    """TDB step against HOSVD as N grows (N x N x N cubes of the five-term analytic
    stream, FP32 storage, ranks fixed at (5, 5, 5)): the cost of one fused TDB step
    (pipelined ingest, averaged over `steps`) and of one HOSVD of a snapshot (Grams,
    eigenpairs, core projection: what a per-snapshot HOSVD would cost; the median
    over `reps` fresh initialisations), and the log-log slopes of both against S."""
    import torch
    from streams import analytic_cp5_spec
    from paper_2201_06958_amd import Compressor
    rows = []
    for n in sizes:
        sp = analytic_cp5_spec(n=n, steps=steps + 2)
        snaps = [sp.snapshot(k, device="cuda").to(torch.float32) for k in range(steps + 2)]
        torch.cuda.synchronize()
        ts = []
        for rep in range(reps + 1):
            c = Compressor(sp.dims, sp.dt, rank_max=sp.rank_max, rank_init=sp.rank_init, weights=sp.weights,
                           data_dtype="f32", precision="f32", adaptive=False, eps_th=1.0, snapshot_mode="borrow")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.init(snaps[0])
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            if rep < reps:
                c.close()
        hosvd = sorted(ts[1:])[len(ts[1:]) // 2]      # the first initialisation loads code
        c.ingest(snaps[1])
        c.flush()
        torch.cuda.synchronize()
        c.profile_enable(True)
        t0 = time.perf_counter()
        for k in range(2, steps + 2):
            c.ingest(snaps[k])
        c.flush()
        torch.cuda.synchronize()
        step = (time.perf_counter() - t0) / steps
        pj = c.profile_read("project")
        c.close()
        rows.append({"N": n, "S": n ** 3, "hosvd_ms": 1e3 * hosvd, "tdb_step_us": 1e6 * step,
                     "hosvd_over_step": hosvd / step, "pass_launches": pj["launches"],
                     "pass_avg_us": 1e3 * pj["total_ms"] / max(pj["launches"], 1)})
        print(f"[bench] sweep N={n}: HOSVD {1e3 * hosvd:.3f} ms, TDB step {1e6 * step:.1f} us, "
              f"stage pass {rows[-1]['pass_avg_us']:.1f} us x {rows[-1]['pass_launches']}",
              file=sys.stderr, flush=True)

    def slope(key):
        xs = [math.log(r["S"]) for r in rows]
        ys = [math.log(r[key]) for r in rows]
        mx, my = sum(xs) / len(xs), sum(ys) / len(ys)
        return sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sum((x - mx) ** 2 for x in xs)

    return {"sweep": "tdb-vs-hosvd", "data": "synthetic", "stream": "analytic five-term, FP32, ranks (5,5,5)",
            "rows": rows, "slope_tdb_step_vs_S": slope("tdb_step_us"), "slope_hosvd_vs_S": slope("hosvd_ms")}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--path", default="auto", choices=["auto", "plain", "fused"])
    ap.add_argument("--plain-steps", type=int, default=200,
                    help="steps of the plain FP64 GPU path timed for comparison (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ensemble-streams", type=int, default=256,
                    help="streams of the batched ensemble measurement (0 = skip)")
    ap.add_argument("--ensemble-steps", type=int, default=20)
    ap.add_argument("--bf16-steps", type=int, default=300,
                    help="steps of the BF16-split form of the headline stream (0 = skip)")
    ap.add_argument("--scaling-sweep", type=str, default="",
                    help="comma-separated cube sizes N: time a TDB step against an HOSVD of an "
                         "N x N x N snapshot for each (prints one JSON line and nothing else)")
    ap.add_argument("--sweep-steps", type=int, default=50, help="TDB steps timed per size of the sweep")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (a known-size reference for "
                         "hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the design notes, "
              "'How the path would shard').", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.scaling_sweep:
        sizes = [int(x) for x in args.scaling_sweep.split(",") if x.strip()]
        print(json.dumps(_scaling_sweep(sizes, max(args.sweep_steps, 10))), flush=True)
        return
    sp, desc = _workload(args)
    print(f"[bench] generating {args.warmup + args.steps + 1} snapshots on the device", file=sys.stderr,
          flush=True)
    snaps = _make_snapshots(sp, args.warmup + args.steps + 1, "cuda")
    if args.calibrate_copy:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    print("[bench] timed run", file=sys.stderr, flush=True)
    el, st, prof = _run_gpu(sp, snaps, args.warmup, args.steps, args.precision, args.path)
    value = args.steps / el
    pj = prof["project"]
    avg_s = pj["total_ms"] / max(pj["launches"], 1) * 1e-3
    achieved = pj["bytes_per_launch"] / avg_s / 1e9 if avg_s > 0 else 0.0
    er = prof["error"]
    er_avg_s = er["total_ms"] / max(er["launches"], 1) * 1e-3
    traffic = None
    if args.precision == "f32" and args.path != "plain":
        from paper_2201_06958_amd.profsum import read_pass_traffic
        traffic = read_pass_traffic(TRAFFIC_FILE, "k_mpass_w16<float, 1>")
    plain = None
    if args.plain_steps > 0:
        print("[bench] plain FP64 GPU path", file=sys.stderr, flush=True)
        n_pl = min(args.plain_steps, args.steps)
        el_p, st_p, _ = _run_gpu(sp, snaps, args.warmup, n_pl, "f64", "plain", profile=False)
        plain = {"value": n_pl / el_p, "unit": "snapshots/s", "steps": n_pl,
                 "speedup": value / (n_pl / el_p)}
    bf16 = None
    if args.bf16_steps > 0 and args.precision == "f32":
        print("[bench] BF16-split stage pass", file=sys.stderr, flush=True)
        n_b = min(args.bf16_steps, args.steps)
        el_b, st_b, pr_b = _run_gpu(sp, snaps, args.warmup, n_b, "bf16s", args.path)
        pb = pr_b["project"]
        pbav = pb["total_ms"] / max(pb["launches"], 1) * 1e-3
        bf16 = {"value": n_b / el_b, "unit": "snapshots/s", "steps": n_b, "pass_avg_launch_us": pbav * 1e6,
                "pass_achieved_GBs": pb["bytes_per_launch"] / pbav / 1e9, "final_eps": st_b["eps"],
                "final_ranks": st_b["ranks"]}
    ens = None
    if args.ensemble_streams > 0:
        del snaps
        torch.cuda.empty_cache()
        print(f"[bench] batched ensemble of {args.ensemble_streams} streams", file=sys.stderr, flush=True)
        ens = _run_ensemble(args.ensemble_streams, 3, args.ensemble_steps)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = _cpu_baseline(sp, args.warmup)
    line = {
        "metric": METRIC, "value": value, "unit": "snapshots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": dict(desc, path=args.path, precision=args.precision),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["traffic_bytes"] if traffic else None,
                     "traffic_unit": "bytes/launch",
                     "traffic_read_write": ([traffic["read_bytes"], traffic["write_bytes"]]
                                            if traffic else None),
                     "kernel": "stage projection pass (one Heun stage; k_mpass_w16, matrix cores)",
                     "avg_launch_us": avg_s * 1e6, "launches": pj["launches"],
                     "timed_every_nth_step": PROFILE_EVERY,
                     "algorithmic_bytes_per_launch": pj["bytes_per_launch"]},
        "error_pass": {"avg_launch_us": er_avg_s * 1e6,
                       "achieved_GBs": er["bytes_per_launch"] / er_avg_s / 1e9 if er_avg_s > 0 else 0.0},
        "final_stats": {"ranks": st["ranks"], "eps": st["eps"], "crbar": st["crbar"],
                        "n_add": st["n_add"], "n_reinit": st["n_reinit"], "n_remove": st["n_remove"]},
        "plain_fp64_gpu": plain,
        "bf16_split": bf16,
        "ensemble": ens,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
