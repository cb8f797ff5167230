#!/usr/bin/env python3
"""Throughput of the TDB in situ compressor on one MI355X.

Headline workload: the batched stochastic ensemble. 256 independent streams of 2-D
fields on grids drawn uniformly from {128,192,256}^2 with 4 variables (FP32
snapshots), each variable a sum of 16 random Fourier modes (amplitudes N(0,1)|k|^-5/6,
phases drifting at rates U(0.5, 2)); adaptive ranks capped at 24 per mode, error
threshold 1e-5. One step = one snapshot of every stream ingested (256 snapshots) by
the batched fused path: two Heun stages of the column-block projection pass, the
small FP64 work, the re-orthonormalisation, the weighted error pass and the
controller, pipelined (the host reads a step while the next one runs) and replayed
from HIP graphs.

All snapshots of the run are generated on the device before timing. One step's 256
snapshots hold 151 MB and a stage pass streams two steps' worth (302 MB), more than
the 256 MB last-level cache, so the passes read HBM. Prints one JSON line.

Besides the headline, the line carries: the same ensemble with BF16-split products;
the plain FP64 GPU path on a sample of its streams; the single reactive-flow-shaped
stream (512 x 256 x 8, FP32) with its own pass roofline; and the FP64 CPU oracle
timed on the host's cores at one thread and at all physical cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E peak
LLC_BYTES = 256 << 20      # MI355X last-level (Infinity) cache
PROFILE_EVERY = 8          # pass timing sampled on every 8th step of a timed run
# HBM bytes per launch from hardware counters (FETCH_SIZE / WRITE_SIZE, calibrated
# against a copy of known size); ignored once the kernel's sources change.
ENSEMBLE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ensemble256_fp32.txt")
PLUME_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stage_pass_plume512x256x8_fp32.txt")
def _pass_kernel_name(plan, flavor=1):
    """The stage-pass kernel a batch's plan runs (FP32 products: flavor 1; BF16-split: 2)."""
    if plan["pass"] == "matrix-core-columns":
        return f"kb_rpass<float, {flavor}, 4, true, {plan['pass_cols']}>"
    if plan["pass"] == "matrix-core-tiles":
        return f"kb_mpass<float, {flavor}>"
    return "kb_fpass<float, float>"
PLUME_PASS = "k_mpass_w16<float, 1>"
METRIC = "snapshots/s ingested + HBM GB/s vs plain FP64 GPU at <=1e-6 rel err"


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _ensemble_specs(n, steps):
    from streams import fourier_ensemble_specs
    return fourier_ensemble_specs(n_streams=n, steps=steps)


def _ensemble_desc(n, specs):
    grids = sorted({(sp.dims[0], sp.dims[1]) for sp in specs})
    return {"workload": f"fourier-ensemble-{n}x{{128,192,256}}^2x4-fp32 (batched stochastic ensemble)",
            "streams": n, "grids": [list(g) for g in grids], "variables": 4, "fourier_modes": 16,
            "rank_max": list(specs[0].rank_max), "eps_th": specs[0].eps_th, "dt": specs[0].dt,
            "adaptive": True, "snapshot_storage": "f32",
            "elements_per_step": sum(sp.dims[0] * sp.dims[1] * sp.dims[2] for sp in specs)}


def _run_ensemble(specs, snaps, warmup, steps, precision, profile_every):
    """The batched ensemble: warmup steps, then `steps` timed steps bracketed by a device
    synchronisation (the last step is read inside the timed region)."""
    import torch
    from paper_2201_06958_amd import Batch
    cfgs = [dict(dims=sp.dims, dt=sp.dt, rank_max=sp.rank_max, weights=sp.weights, data_dtype="f32",
                 precision=precision, adaptive=True, eps_th=sp.eps_th, snapshot_mode="borrow") for sp in specs]
    b = Batch(cfgs).init(snaps[0])
    for k in range(1, warmup + 1):
        b.ingest(snaps[k])
    b.flush()
    torch.cuda.synchronize()
    if profile_every:
        b.profile_enable(True, every=profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        b.ingest(snaps[k])
    b.flush()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = {}
    if profile_every:
        prof = {"project": b.profile_read("project"), "error": b.profile_read("error")}
    sts = [m.stats() for m in b.streams]
    plan = b.plan()
    b.close()
    return el, sts, dict(prof, plan=plan)


def _avg_s(p):
    return p["total_ms"] / max(p["launches"], 1) * 1e-3


def _run_plain(specs, snaps, steps):
    """The plain FP64 GPU path (unfused per-mode TTMs, FP64 products) on the given
    streams, one after another: one step of each after one warm-up step."""
    import torch
    from paper_2201_06958_amd import Compressor
    total = 0.0
    for i, sp in enumerate(specs):
        c = Compressor(sp.dims, sp.dt, rank_max=sp.rank_max, weights=sp.weights, data_dtype="f32",
                       precision="f64", path="plain", adaptive=True, eps_th=sp.eps_th, snapshot_mode="borrow")
        c.init(snaps[0][i])
        c.ingest(snaps[1][i])
        c.flush()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(2, steps + 2):
            c.ingest(snaps[k][i])
        c.flush()
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
        c.close()
    return len(specs) * steps / total


def _run_plume(warmup, steps):
    """The single reactive-flow-shaped stream (512 x 256 x 8, FP32, caps (64, 64, 8),
    threshold 1e-4), pipelined, passes timed on every PROFILE_EVERY-th step."""
    import torch
    from streams import plume_spec
    from paper_2201_06958_amd import Compressor
    sp = plume_spec(steps=warmup + steps + 1)
    snaps = [sp.snapshot(k, device="cuda") for k in range(warmup + steps + 1)]
    torch.cuda.synchronize()
    c = Compressor(sp.dims, sp.dt, rank_max=(64, 64, 8), weights=sp.weights, data_dtype="f32", precision="f32",
                   adaptive=True, snapshot_mode="borrow", eps_th=sp.eps_th)
    c.init(snaps[0])
    for k in range(1, warmup + 1):
        c.ingest(snaps[k])
    c.flush()
    torch.cuda.synchronize()
    c.profile_enable(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        c.ingest(snaps[k])
    c.flush()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = c.stats()
    pj, er = c.profile_read("project"), c.profile_read("error")
    c.close()
    ring = len(snaps) * snaps[0].numel() * 4
    pav, eav = _avg_s(pj), _avg_s(er)
    from paper_2201_06958_amd.profsum import read_pass_traffic
    traffic = read_pass_traffic(PLUME_TRAFFIC_FILE, PLUME_PASS)
    return {"workload": "plume-512x256x8-fp32 (reactive-flow-shaped stream)", "steps": steps,
            "value": steps / el, "unit": "snapshots/s", "ms_per_step": 1e3 * el / steps,
            "ring_bytes": ring, "cache_resident": ring <= LLC_BYTES,
            "pass": {"kernel_name": PLUME_PASS, "avg_launch_us": pav * 1e6, "launches": pj["launches"],
                     "algorithmic_bytes_per_launch": pj["bytes_per_launch"],
                     "achieved_GBs": pj["bytes_per_launch"] / pav / 1e9,
                     "frac": pj["bytes_per_launch"] / pav / 1e9 / HBM_PEAK_GBS,
                     "traffic": traffic["traffic_bytes"] if traffic else None},
            "error_pass": {"avg_launch_us": eav * 1e6, "achieved_GBs": er["bytes_per_launch"] / eav / 1e9},
            "final_stats": {"ranks": st["ranks"], "eps": st["eps"], "crbar": st["crbar"], "n_add": st["n_add"],
                            "n_reinit": st["n_reinit"], "n_remove": st["n_remove"]}}


def _tdb1_vs_tdb2(warmup, steps):
    """The reactive-flow-shaped stream compressed two ways at the same threshold
    (Sec. 3.2): TDB-1, third order (x1, x2, variables) with caps (64, 64, 8), and
    TDB-2, the DBO form of order 2 with x1 and x2 grouped into one mode of 131072 rows
    (row passes), caps (8, 8). Both adaptive from the HOSVD of the first snapshot;
    per-step eps and events from untimed runs, throughput of TDB-2 from a timed one.
    Storage counts the core and bases at the final ranks, as Sec. 3.2 writes it."""
    import torch
    from streams import plume_spec
    from paper_2201_06958_amd import Compressor
    sp = plume_spec(steps=warmup + steps + 1)
    n1, n2, nv = sp.dims
    snaps = [sp.snapshot(k, device="cuda") for k in range(warmup + steps + 1)]
    torch.cuda.synchronize()
    w12 = np.kron(sp.weights[0], sp.weights[1])
    out = {"workload": f"plume-{n1}x{n2}x{nv}-fp32, eps_th {sp.eps_th:g}", "steps": steps}
    for name in ("tdb1", "tdb2"):
        if name == "tdb1":
            mk = lambda: Compressor(sp.dims, sp.dt, rank_max=(64, 64, nv), weights=sp.weights, data_dtype="f32",
                                    precision="f32", adaptive=True, eps_th=sp.eps_th)
            view = lambda x: x
        else:
            mk = lambda: Compressor((n1 * n2, nv), sp.dt, rank_max=(nv, nv), weights=[w12, sp.weights[2]],
                                    data_dtype="f32", precision="f32", adaptive=True, eps_th=sp.eps_th)
            view = lambda x: x.view(n1 * n2, nv)
        c = mk()
        c.init(view(snaps[0]))
        eps, ranks = [], []
        for k in range(1, warmup + steps + 1):
            c.ingest(view(snaps[k]))
            st = c.stats()
            eps.append(st["eps"])
            ranks.append(st["ranks"])
        st = c.stats()
        c.close()
        r = st["ranks"]
        if name == "tdb1":
            storage = r[0] * n1 + r[1] * n2 + r[2] * nv + r[0] * r[1] * r[2]
        else:
            storage = r[0] * n1 * n2 + r[1] * nv + r[0] * r[1]
        # timed run (no statistics read between steps)
        c = mk()
        c.init(view(snaps[0]))
        for k in range(1, warmup + 1):
            c.ingest(view(snaps[k]))
        c.flush()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup + 1, warmup + steps + 1):
            c.ingest(view(snaps[k]))
        c.flush()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stt = c.stats()
        c.close()
        e = np.array(eps[warmup:])
        out[name] = {"value": steps / el, "unit": "snapshots/s", "ms_per_step": 1e3 * el / steps,
                     "path": stt["path_used"], "final_ranks": r, "crbar": st["crbar"],
                     "storage_floats": storage, "n_reinit": st["n_reinit"], "n_add": st["n_add"],
                     "n_remove": st["n_remove"], "eps_max": float(np.nanmax(e)), "eps_mean": float(np.nanmean(e)),
                     "max_rank_sum": int(max(sum(x) for x in ranks))}
    out["storage_ratio_tdb2_over_tdb1"] = out["tdb2"]["storage_floats"] / out["tdb1"]["storage_floats"]
    return out


def _samples_as_mode(warmup, steps, nx=128, ny=64, nv=8, s=(4, 4)):
    """Samples as a tensor mode (Sec. 3.3, eq. (UQ)) against independent streams: the
    s1 x s2 stochastic reactive-flow samples compressed as one order-4 tensor (sample
    mode first, product Gauss weights) and as a batch of independent third-order streams,
    both adaptive at the same threshold. The tensor's eps is the weighted RMS over the
    samples; the batch's is formed from its members' eps with the same weights.
    Compression counts the core and bases of each at every step (time-weighted)."""
    import torch
    from streams import stochastic_plume_spec
    from paper_2201_06958_amd import Compressor, Batch
    sp = stochastic_plume_spec(nx=nx, ny=ny, nv=nv, s=s, steps=warmup + steps + 1)
    S = sp.dims[0]
    snaps = [sp.snapshot(k, device="cuda") for k in range(warmup + steps + 1)]
    torch.cuda.synchronize()
    out = {"workload": f"stochastic-plume {S} samples x {nx}x{ny}x{nv} fp32, eps_th {sp.eps_th:g}", "steps": steps}
    # one tensor
    c = Compressor(sp.dims, sp.dt, rank_max=(S, 32, 32, nv), weights=sp.weights, data_dtype="f32",
                   precision="f32", adaptive=True, eps_th=sp.eps_th)
    c.init(snaps[0])
    eps = []
    for k in range(1, warmup + 1):
        c.ingest(snaps[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        c.ingest(snaps[k])
        eps.append(c.stats()["eps"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = c.stats()
    c.close()
    out["tensor"] = {"value": S * steps / el, "unit": "sample-snapshots/s", "ms_per_step": 1e3 * el / steps,
                     "path": st["path_used"], "final_ranks": st["ranks"], "crbar": st["crbar"],
                     "eps_mean": float(np.mean(eps)), "eps_max": float(np.max(eps)),
                     "events": {k: st[k] for k in ("n_add", "n_remove", "n_reinit")}}
    # independent streams
    specs = sp.meta["sample_specs"]
    b = Batch([dict(dims=q.dims, dt=q.dt, rank_max=(32, 32, nv), weights=q.weights, data_dtype="f32",
                    precision="f32", adaptive=True, snapshot_mode="borrow", eps_th=sp.eps_th) for q in specs])
    b.init([snaps[0][i] for i in range(S)])
    for k in range(1, warmup + 1):
        b.ingest([snaps[k][i] for i in range(S)])
    b.flush()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        b.ingest([snaps[k][i] for i in range(S)])
    b.flush()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sts = [m.stats() for m in b.streams]
    b.close()
    wq = sp.weights[0]
    elems = nx * ny * nv
    # aggregate compression: all samples' values over all members' stored floats (time-weighted
    # per member, combined as the sum of stored floats)
    stored = sum(elems / m["crbar"] for m in sts)
    out["independent"] = {"value": S * steps / el, "unit": "sample-snapshots/s", "ms_per_step": 1e3 * el / steps,
                          "max_ranks": [max(m["ranks"][i] for m in sts) for i in range(3)],
                          "crbar": S * elems / stored,
                          "eps_weighted_rms_end": float(np.sqrt(sum(w * m["eps"] ** 2 for w, m in zip(wq, sts)))),
                          "events": {k: sum(m[k] for m in sts) for k in ("n_add", "n_remove", "n_reinit")}}
    out["cr_ratio_tensor_over_independent"] = out["tensor"]["crbar"] / out["independent"]["crbar"]
    return out


def _run_c1(steps=200, warmup=5):
    """The plain single-stream case: the five-term analytic 64^3 stream in FP64, fixed
    ranks (5, 5, 5), Heun with the first-order difference, on the fused FP64 path and on
    the plain FP64 per-mode path; their final states agree to the stated 1e-6."""
    import torch
    from streams import analytic_cp5_spec
    from paper_2201_06958_amd import Compressor
    sp = analytic_cp5_spec(n=64, steps=warmup + steps)
    snaps = [sp.snapshot(k, device="cuda") for k in range(warmup + steps + 1)]
    torch.cuda.synchronize()
    out = {"workload": "analytic-64^3-fp64, ranks (5, 5, 5) fixed, dt 1e-3", "steps": steps}
    recs = {}
    for path in ("fused", "plain"):
        c = Compressor(sp.dims, sp.dt, rank_max=(5, 5, 5), rank_init=(5, 5, 5), weights=sp.weights, data_dtype="f64",
                       precision="f64", path=path, adaptive=False, eps_th=1.0)
        c.init(snaps[0])
        for k in range(1, warmup + 1):
            c.ingest(snaps[k])
        c.flush()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup + 1, warmup + steps + 1):
            c.ingest(snaps[k])
        c.flush()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = c.stats()
        rec = torch.empty_like(snaps[0])
        c.reconstruct(rec)
        torch.cuda.synchronize()
        recs[path] = rec
        c.close()
        out[path] = {"value": steps / el, "unit": "snapshots/s", "ms_per_step": 1e3 * el / steps,
                     "path_used": st["path_used"], "eps_over_nu": st["eps"] / st["nu"],
                     "achieved_GBs_step": 5 * sp.size * 8 / (el / steps) / 1e9}
    out["max_rel_diff_fused_vs_plain"] = float((recs["fused"] - recs["plain"]).abs().max() /
                                               recs["plain"].abs().max())
    out["speedup_fused_over_plain"] = out["fused"]["value"] / out["plain"]["value"]
    return out


def _run_c4(steps=30, warmup=5):
    """The channel-flow-shaped stream, 192 x 129 x 192 x 3 FP32, adaptive (caps (40, 40,
    40, 3), threshold 1e-3). Order 4 runs on the plain per-mode path; BF16-split
    products are not available for it, so precision_used reports FP32."""
    import torch
    from streams import channel_spec
    from paper_2201_06958_amd import Compressor
    sp = channel_spec(steps=warmup + steps)
    snaps = [sp.snapshot(k, device="cuda") for k in range(warmup + steps + 1)]
    torch.cuda.synchronize()
    c = Compressor(sp.dims, sp.dt, rank_max=sp.rank_max, weights=sp.weights, data_dtype="f32",
                   precision="bf16s", adaptive=True, eps_th=sp.eps_th)
    t0 = time.perf_counter()
    c.init(snaps[0])
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    for k in range(1, warmup + 1):
        c.ingest(snaps[k])
    c.flush()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup + 1, warmup + steps + 1):
        c.ingest(snaps[k])
    c.flush()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = c.stats()
    c.close()
    return {"workload": "channel-192x129x192x3-fp32, caps (40, 40, 40, 3), eps_th 1e-3", "steps": steps,
            "value": steps / el, "unit": "snapshots/s", "ms_per_step": 1e3 * el / steps,
            "init_hosvd_ms": 1e3 * t_init, "path_used": st["path_used"], "precision_used": st["precision_used"],
            "ranks": st["ranks"], "eps": st["eps"], "crbar": st["crbar"],
            "events": {k: st[k] for k in ("n_add", "n_remove", "n_reinit")},
            "achieved_GBs_step": 5 * sp.size * 4 / (el / steps) / 1e9}


def _run_c5(train_steps=150, eval_steps=30):
    """The learned error gate at a larger scale: trained on the histories of 48 held-out
    ensemble members and 16 reactive-flow streams of 256 x 128 x 8 (windows of 8 exact
    steps without a reinitialisation), evaluated on the 256-stream ensemble together
    with 64 reactive-flow streams of 512 x 256 x 8 (shifted plumes, their own noise
    seeds): skipped error passes, mis-decisions against the exact pass, decisions of
    the gated and exact runs, and snapshots/s gated against always exact."""
    from streams import fourier_ensemble_specs, plume_spec, gate_init_params
    from paper_2201_06958_amd import Gate
    from paper_2201_06958_amd import gate as GP

    def cfg(sp, caps):
        return dict(dims=sp.dims, dt=sp.dt, rank_max=caps, weights=sp.weights, data_dtype="f32",
                    precision="f32", adaptive=True, eps_th=sp.eps_th, snapshot_mode="copy")

    def streams(seed0, n_ens, n_plume, size, steps):
        specs = fourier_ensemble_specs(n_streams=n_ens, seed0=seed0, steps=steps + 1)
        cfgs = [cfg(q, q.rank_max) for q in specs]
        rng = np.random.default_rng(seed0)
        for j in range(n_plume):
            q = plume_spec(nx=size[0], ny=size[1], nv=8, steps=steps + 1, noise_seed=100 * seed0 + 17 * j,
                           centre_shift=(float(rng.uniform(0, 2)), float(rng.uniform(0, 1))))
            specs.append(q)
            cfgs.append(cfg(q, (32, 32, 8)))
        cache = {}

        def snapshot(k):
            if k not in cache:
                cache.clear()
                cache[k] = [q.snapshot(k, device="cuda") for q in specs]
            return cache[k]
        return specs, cfgs, snapshot

    specs, cfgs, snap = streams(5000, 48, 16, (256, 128), train_steps)
    t0 = time.perf_counter()
    h = GP.record_histories(cfgs, snap, train_steps)
    X, t = GP.make_samples(h)
    ms = GP.standardisation(X)
    g = Gate(max_batch=1024)
    g.set_params(gate_init_params(11))
    hist = GP.train(g, X, t, ms, epochs=30, batch=256, lr=1e-3)
    t_train = time.perf_counter() - t0
    specs2 = fourier_ensemble_specs(n_streams=256, seed0=1000, steps=eval_steps + 1)
    cfgs2 = [cfg(q, q.rank_max) for q in specs2]
    rng = np.random.default_rng(9000)
    for j in range(64):
        q = plume_spec(steps=eval_steps + 1, noise_seed=9000 + 17 * j,
                       centre_shift=(float(rng.uniform(0, 2)), float(rng.uniform(0, 1))))
        specs2.append(q)
        cfgs2.append(cfg(q, (32, 32, 8)))   # the stream's ranks stay near (15, 15, 4)
    import torch
    # every evaluation snapshot is generated before the runs, so that the timed loops
    # measure the compression only
    allsnaps = [[q.snapshot(k, device="cuda") for q in specs2] for k in range(eval_steps + 1)]
    torch.cuda.synchronize()
    ev = GP.evaluate(cfgs2, lambda k: allsnaps[k], eval_steps, g, ms, [q.eps_th for q in specs2])
    g.close()
    ev.update({"workload": "gate: trained on 48 ensemble + 16 reactive-flow (256x128x8) histories; evaluated on "
                           "the 256-stream ensemble + 64 reactive-flow streams (512x256x8)",
               "train_samples": int(X.shape[0]), "train_loss_first_last": [hist[0], hist[-1]],
               "train_wall_s": t_train, "eval_steps": eval_steps,
               "speedup_gated_over_exact": ev["snapshots_per_s_gated"] / ev["snapshots_per_s_exact"]})
    return ev


def _guarded(name, fn, *a):
    """An extra record: its failure is reported in the line, not raised."""
    try:
        return fn(*a)
    except Exception as e:  # noqa: BLE001 - the headline must still be printed
        _log(f"{name} failed: {e!r}")
        return {"error": repr(e)}


# ---------------------------------------------------------------- CPU oracle

def _physical_cores():
    """Physical cores from lscpu (cores per socket x sockets), capped by the CPUs this
    process may run on."""
    phys = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for ln in out.splitlines():
            if ":" in ln:
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
        phys = int(kv["Core(s) per socket"]) * int(kv.get("Socket(s)", "1"))
        model = kv.get("Model name", "")
    except Exception:
        model = ""
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return min(phys or avail, avail), phys, avail, model


def _cpu_worker(n_streams, warm, timed):
    """The FP64 numpy oracle on the first n_streams ensemble streams: per stream an
    HOSVD initialisation, `warm` steps, then `timed` timed steps; prints the median
    per-snapshot ingest time and the threads the BLAS pools hold."""
    import numpy as np
    from oracle import tdb_oracle as O
    specs = _ensemble_specs(256, warm + timed + 1)[:n_streams]
    times = []
    for sp in specs:
        snaps = [sp.snapshot_np(k).astype(np.float64) for k in range(warm + timed + 1)]
        o = O.OracleTDB(O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                                       rank_init=None, adaptive=True, eps_th=sp.eps_th)).init(snaps[0])
        for k in range(1, warm + 1):
            o.ingest(snaps[k])
        for k in range(warm + 1, warm + timed + 1):
            t0 = time.perf_counter()
            o.ingest(snaps[k])
            times.append(time.perf_counter() - t0)
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        pass
    times.sort()
    print(json.dumps({"median_s": times[len(times) // 2], "samples": len(times), "blas_threads": threads}))


def _cpu_baseline(n_streams=32, warm=5, timed=5):
    """The oracle in child processes (so the BLAS thread count is fixed before numpy
    loads): one thread, then all physical cores available to this process."""
    cores, phys, avail, model = _physical_cores()
    runs = {}
    for nt in (1, cores):
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
            env[k] = str(nt)
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-oracle-worker",
                              f"{n_streams},{warm},{timed}"], capture_output=True, text=True, env=env,
                             timeout=900)
        if out.returncode != 0:
            raise RuntimeError(out.stderr[-2000:])
        runs[nt] = json.loads(out.stdout.strip().splitlines()[-1])
    sample = (f"the FP64 numpy oracle on the first {n_streams} ensemble streams: per stream an HOSVD "
              f"initialisation and {warm} warm-up steps, then {timed} timed steps; median per-snapshot "
              f"ingest time (snapshot generation excluded) over {runs[cores]['samples']} snapshots")
    all_c = runs[cores]
    return {"value": 1.0 / all_c["median_s"], "unit": "snapshots/s", "cores": cores, "kind": "oracle",
            "sample": sample, "blas_threads": all_c["blas_threads"],
            "one_thread": {"value": 1.0 / runs[1]["median_s"], "unit": "snapshots/s", "cores": 1},
            "host": {"lscpu_physical_cores": phys, "cpus_available": avail, "model": model}}


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
        _log(f"sweep N={n}: HOSVD {1e3 * hosvd:.3f} ms, TDB step {1e6 * step:.1f} us, "
             f"stage pass {rows[-1]['pass_avg_us']:.1f} us x {rows[-1]['pass_launches']}")

    def slope(key):
        xs = [math.log(r["S"]) for r in rows]
        ys = [math.log(r[key]) for r in rows]
        mx, my = sum(xs) / len(xs), sum(ys) / len(ys)
        return sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sum((x - mx) ** 2 for x in xs)

    return {"sweep": "tdb-vs-hosvd", "data": "synthetic", "stream": "analytic five-term, FP32, ranks (5,5,5)",
            "rows": rows, "slope_tdb_step_vs_S": slope("tdb_step_us"), "slope_hosvd_vs_S": slope("hosvd_ms")}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed ensemble steps")
    ap.add_argument("--warmup", type=int, default=10, help="untimed ensemble steps first")
    ap.add_argument("--streams", type=int, default=256, help="streams of the ensemble")
    ap.add_argument("--no-extras", action="store_true",
                    help="the headline only (no BF16-split, plain FP64 GPU or reactive-flow records)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-streams", type=int, default=16,
                    help="ensemble streams the plain FP64 GPU path is timed on")
    ap.add_argument("--plume-steps", type=int, default=300, help="timed steps of the reactive-flow stream")
    ap.add_argument("--calibrate-traffic", action="store_true",
                    help="only run the traffic-counter calibration kernels (a 256 MiB copy, a 256 MiB "
                         "read-only sum, a gather of one float per 128-byte line) and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (a known-size reference for "
                         "hardware traffic counters)")
    ap.add_argument("--scaling-sweep", type=str, default="",
                    help="comma-separated cube sizes N: time a TDB step against an HOSVD of an "
                         "N x N x N snapshot for each (prints one JSON line and nothing else)")
    ap.add_argument("--sweep-steps", type=int, default=50, help="TDB steps timed per size of the sweep")
    ap.add_argument("--configs", type=str, default="",
                    help="only run the named configuration records (comma-separated: c1, c4, c5) and print "
                         "them as one JSON line")
    ap.add_argument("--samples-as-mode", action="store_true",
                    help="only compare 16 stochastic samples compressed as one order-4 tensor with the same "
                         "samples as independent streams over --plume-steps steps (prints one JSON line)")
    ap.add_argument("--plume-only", action="store_true",
                    help="only run the reactive-flow-shaped stream (512 x 256 x 8, FP32) over --plume-steps steps "
                         "(prints its record as one JSON line; with --calibrate-copy the 256 MiB copy first)")
    ap.add_argument("--tdb1-vs-tdb2", action="store_true",
                    help="only compare TDB-1 (third order) with TDB-2 (order 2, grouped spatial mode) on the "
                         "reactive-flow-shaped stream over --plume-steps steps (prints one JSON line)")
    ap.add_argument("--cpu-oracle-worker", type=str, default="", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_oracle_worker:
        n, w, t = (int(x) for x in args.cpu_oracle_worker.split(","))
        _cpu_worker(n, w, t)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the design notes say how the "
              "path would shard); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.plume_only:
        if args.calibrate_copy:
            x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
            y = torch.empty_like(x)
            for _ in range(3):
                y.copy_(x)
            torch.cuda.synchronize()
            del x, y
        print(json.dumps(_run_plume(20, args.plume_steps)), flush=True)
        return
    if args.configs:
        fns = {"c1": _run_c1, "c4": _run_c4, "c5": _run_c5}
        print(json.dumps({c: fns[c]() for c in args.configs.split(",") if c}), flush=True)
        return
    if args.samples_as_mode:
        print(json.dumps(_samples_as_mode(10, args.plume_steps)), flush=True)
        return
    if args.tdb1_vs_tdb2:
        print(json.dumps(_tdb1_vs_tdb2(10, args.plume_steps)), flush=True)
        return
    if args.calibrate_traffic:
        # known footprints for FETCH_SIZE / WRITE_SIZE: a copy reads and writes 256 MiB, the
        # sum reads 256 MiB and writes one value, the gather touches 2 Mi lines of 128 B and
        # writes 8 MiB
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
            _ = x.sum()
            _ = x.view(-1, 32)[:, 0].contiguous()
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy 268435456 B; sum 268435456 B; gather 2097152 lines of 128 B"}))
        return
    if args.scaling_sweep:
        sizes = [int(x) for x in args.scaling_sweep.split(",") if x.strip()]
        print(json.dumps(_scaling_sweep(sizes, max(args.sweep_steps, 10))), flush=True)
        return
    n = args.streams
    total = args.warmup + args.steps + 1
    specs = _ensemble_specs(n, total)
    desc = _ensemble_desc(n, specs)
    _log(f"generating {total} snapshots of each of {n} streams on the device")
    snaps = [[sp.snapshot(k, device="cuda") for sp in specs] for k in range(total)]
    torch.cuda.synchronize()
    if args.calibrate_copy:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    _log("timed run (FP32 products)")
    el, sts, prof = _run_ensemble(specs, snaps, args.warmup, args.steps, "f32", PROFILE_EVERY)
    value = n * args.steps / el
    pj, er = prof["project"], prof["error"]
    pav, eav = _avg_s(pj), _avg_s(er)
    achieved = pj["bytes_per_launch"] / pav / 1e9
    step_s = el / args.steps
    elems = desc["elements_per_step"]
    step_bytes = 5.0 * 4.0 * elems     # two stages x (V_k+1, V_k), one error pass
    from paper_2201_06958_amd.profsum import read_pass_traffic
    pass_name = _pass_kernel_name(prof["plan"])
    traffic = read_pass_traffic(ENSEMBLE_TRAFFIC_FILE, pass_name)
    ring = total * elems * 4
    extras = {}
    if not args.no_extras:
        _log("BF16-split products")
        n_b = max(10, args.steps // 2)
        el_b, sts_b, prof_b = _run_ensemble(specs, snaps, args.warmup, n_b, "bf16s", PROFILE_EVERY)
        pb = _avg_s(prof_b["project"])
        extras["ensemble_bf16_split"] = {
            "value": n * n_b / el_b, "unit": "snapshots/s", "steps": n_b, "ms_per_step": 1e3 * el_b / n_b,
            "pass_avg_launch_us": pb * 1e6, "pass_achieved_GBs": prof_b["project"]["bytes_per_launch"] / pb / 1e9,
            "max_ranks": [max(s["ranks"][i] for s in sts_b) for i in range(3)]}
        ns = min(args.plain_streams, n)
        _log(f"plain FP64 GPU path on {ns} streams")
        plain_v = _run_plain(specs[:ns], [row[:ns] for row in snaps[:5]], 3)
        extras["plain_fp64_gpu"] = {
            "value": plain_v, "unit": "snapshots/s",
            "sample": f"the first {ns} ensemble streams one after another (unfused per-mode TTMs, FP64 "
                      f"products), 3 steps each after one warm-up step",
            "speedup": value / plain_v}
        del snaps
        torch.cuda.empty_cache()
        _log("reactive-flow-shaped stream")
        extras["plume_c2"] = _guarded("plume", _run_plume, 20, args.plume_steps)
        _log("TDB-1 against TDB-2 (grouped spatial mode) on the reactive-flow-shaped stream")
        extras["tdb1_vs_tdb2"] = _guarded("tdb1_vs_tdb2", _tdb1_vs_tdb2, 10, args.plume_steps)
        _log("16 stochastic samples as one order-4 tensor against independent streams")
        extras["samples_as_mode"] = _guarded("samples_as_mode", _samples_as_mode, 10, 100)
        _log("analytic 64^3 FP64, fused against plain")
        extras["c1_analytic_fp64"] = _guarded("c1", _run_c1)
        _log("channel-flow-shaped stream (order 4)")
        extras["c4_channel"] = _guarded("c4", _run_c4)
        _log("learned error gate at scale")
        extras["c5_gate"] = _guarded("c5", _run_c5)
    else:
        del snaps
    cpu = None
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle, 1 thread and all physical cores)")
        cpu = _cpu_baseline()
    line = {
        "metric": METRIC, "value": value, "unit": "snapshots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * step_s, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(desc, precision="f32", path="fused-batched", ring_bytes=ring,
                       cache_resident=ring <= LLC_BYTES, kernel_plan=prof["plan"]),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["traffic_bytes"] if traffic else None,
                     "traffic_unit": "bytes/launch",
                     "traffic_read_write": ([traffic["read_bytes"], traffic["write_bytes"]]
                                            if traffic else None),
                     "kernel": "column-block stage projection pass, one Heun stage of all 256 streams "
                               "(matrix cores, FP32 products)",
                     "kernel_name": pass_name,
                     "avg_launch_us": pav * 1e6, "launches": pj["launches"],
                     "timed_every_nth_step": PROFILE_EVERY,
                     "algorithmic_bytes_per_launch": pj["bytes_per_launch"],
                     "step_algorithmic_bytes": step_bytes,
                     "step_frac": step_bytes / step_s / 1e9 / HBM_PEAK_GBS},
        "error_pass": {"kernel_name": "kb_ferr_mf<float, 24>", "avg_launch_us": eav * 1e6,
                       "algorithmic_bytes_per_launch": er["bytes_per_launch"],
                       "achieved_GBs": er["bytes_per_launch"] / eav / 1e9},
        "final_stats": {"max_ranks": [max(s["ranks"][i] for s in sts) for i in range(3)],
                        "max_eps_over_nu": max(s["eps"] / s["nu"] for s in sts),
                        "events": {k: sum(s[k] for s in sts) for k in ("n_add", "n_remove", "n_reinit")},
                        "graph_steps": sts[0]["graph_steps"]},
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
