"""Text summaries of rocprofv3 result databases for the library's kernels.

    python -m paper_2201_06958_amd.profsum stats DB --command CMD [--bench JSON] [--out FILE]
    python -m paper_2201_06958_amd.profsum pmc FETCH_DB WRITE_DB --command-fetch CMD
        --command-write CMD [--copy-bytes N] [--out FILE]
    python -m paper_2201_06958_amd.profsum counters DB --command CMD [--match NAME] [--out FILE]
    python -m paper_2201_06958_amd.profsum timeline DB --command CMD [--first NAME] [--out FILE]

`stats` tabulates per-kernel call counts and average durations from a
`rocprofv3 --kernel-trace --stats` run (and, given the JSON lines bench.py printed
with and without the profiler, the stage-pass launch duration bench.py measured itself
with dispatch-stamped HIP events, so the two clocks can be compared).

`timeline` splits a `--kernel-trace` run's library kernels into steps at each launch of
the step's first kernel (`--first`), and gives each of the last steps' span against the
time some kernel was running (the union of their intervals), then one step kernel by
kernel, start and end from the step's start.

`pmc` turns two counter runs (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`, each with
`--kernel-trace`) into HBM bytes per dispatch. The raw counters are scaled by what
they read for the largest device-to-device copy in the same run, whose size is known
(`bench.py --calibrate-copy` issues a 256 MiB copy): read scale = bytes / FETCH
reading, write scale = bytes / WRITE reading. The record line at the end of the
output carries the stage-pass figures and a digest of the sources that kernel is
built from, so a reader can tell when they no longer describe the current kernel.

Only the standard library is used; nothing here touches the GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# The stage-pass kernels and the sources each is built from.
_GENERIC = ("fused_pass.hip", "fused.h", "tdb_common.h", "tdb_kernels.h", "device_util.h")
_MATRIX = ("mfma_pass.hip", "fused.h", "tdb_common.h", "tdb_kernels.h")
PASS_KERNELS = {
    "k_mpass_w16<float, 1>": _MATRIX,    # matrix-core pass, FP32 products, one stream,
                                         # one 16-wave tile per compute unit
    "k_mpass_w16<float, 2>": _MATRIX,    # the same with BF16-split products
    "k_mpass<float, 1>": _MATRIX,        # eight-wave tiles, two per compute unit
    "k_mpass<float, 2>": _MATRIX,
    "k_mpass_w4<float, 1>": _MATRIX,     # four-wave tiles (larger grids)
    "kb_mpass<float, 1>": _MATRIX,       # four-wave tiles for a batch of streams
    "k_fpass<float, float>": _GENERIC,   # generic pass
    # column-block pass of batches (FP32 products; BF16-split), 4-entry fibers as float4,
    # column blocks of 64 or 32 (the batch's plan picks one at creation)
    "kb_rpass<float, 1, 4, true, 64>": ("rpass.hip", "mfma_util.h", "fused.h", "tdb_common.h", "tdb_kernels.h"),
    "kb_rpass<float, 1, 4, true, 32>": ("rpass.hip", "mfma_util.h", "fused.h", "tdb_common.h", "tdb_kernels.h"),
    "kb_rpass<float, 2, 4, true, 64>": ("rpass.hip", "mfma_util.h", "fused.h", "tdb_common.h", "tdb_kernels.h"),
    "kb_rpass<float, 2, 4, true, 32>": ("rpass.hip", "mfma_util.h", "fused.h", "tdb_common.h", "tdb_kernels.h"),
    # column-block error pass of batches (mode-1 rank cap 24; the reconstruction on the
    # matrix cores for FP32 compute, on the vector ALU otherwise)
    "kb_ferr_mf<float, 24>": ("fused_ops.hip", "fused.h", "tdb_common.h", "device_util.h"),
    "kb_ferr_cols<float, float, 24>": ("fused_ops.hip", "fused.h", "tdb_common.h", "device_util.h"),
}
PASS_KERNEL = "k_mpass_w16<float, 1>"     # the pass of the reactive-flow workload


def pass_source_digest(kernel: str = PASS_KERNEL) -> str:
    h = hashlib.sha256()
    for name in PASS_KERNELS[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("void ", "")
    cut = name.find("(")
    return name if cut < 0 else name[:cut]


def _bench_line(path: str) -> dict:
    with open(path) as f:
        line = [ln for ln in f.read().splitlines() if ln.startswith("{")][-1]
    return json.loads(line)


def stats_text(db: str, command: str, bench_json: str | None = None, bench_plain: str | None = None,
               top: int = 30) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels order by total_duration desc").fetchall()
    out = ["# rocprofv3 --kernel-trace --stats", "", "command:", f"    {command}", "",
           "durations in microseconds (top_kernels table of the result database)", "",
           f"{'kernel':60s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for name, calls, total, avg, pct in rows[:top]:
        out.append(f"{_short(name)[:60]:60s} {calls:7d} {avg:10.2f} {total / 1e3:10.3f} {pct:6.2f}")
    if bench_json:
        b = _bench_line(bench_json)
        rf = b["roofline"]
        kern = rf.get("kernel_name", PASS_KERNEL)
        prof = [r for r in rows if ("tdb::" + kern + "(") in r[0]]
        out += ["", "bench.py line printed by the profiled run:",
                f"    value {b['value']:.1f} {b['unit']}, ms_per_step {b['ms_per_step']:.4f}",
                f"    stage pass average launch (HIP events in bench.py): {rf['avg_launch_us']:.2f} us"
                f" over {rf['launches']} launches"]
        if prof:
            out.append(f"    stage pass average (this trace, all launches incl. warmup): {prof[0][3]:.2f} us"
                       f" over {prof[0][1]} launches")
        out.append("    (under the tracer the dispatch-stamped events include its per-dispatch overhead)")
    if bench_plain:
        b = _bench_line(bench_plain)
        rf = b["roofline"]
        out += ["", "bench.py without the profiler (same build, same workload):",
                f"    value {b['value']:.1f} {b['unit']} over {b['steps']} steps",
                f"    stage pass average launch (HIP events): {rf['avg_launch_us']:.2f} us over "
                f"{rf['launches']} launches -> {rf['achieved']:.1f} GB/s algorithmic"]
    return "\n".join(out) + "\n"


def _per_kernel(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, grid_size, value from counters_collection").fetchall()
    agg = defaultdict(list)
    for k, g, v in rows:
        agg[(k, g)].append(v)
    return agg


def _calibration(agg):
    copies = [(k, vals) for k, vals in agg.items() if "copyBuffer" in k[0]]
    if not copies:
        raise SystemExit("no copy kernel in the counter run: run bench.py with --calibrate-copy")
    k, vals = max(copies, key=lambda kv: max(kv[1]))
    return max(vals)


def pmc_text(fetch_db: str, write_db: str, cmd_f: str, cmd_w: str, copy_bytes: int):
    fa, wa = _per_kernel(fetch_db), _per_kernel(write_db)
    f_cal, w_cal = _calibration(fa), _calibration(wa)
    f_scale = copy_bytes / 1024.0 / f_cal
    w_scale = copy_bytes / 1024.0 / w_cal
    out = ["# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (HBM traffic per dispatch)", "",
           "commands:", f"    {cmd_f}", f"    {cmd_w}", "",
           f"calibration: a {copy_bytes} B device-to-device copy reads FETCH_SIZE {f_cal:.1f} KiB "
           f"and WRITE_SIZE {w_cal:.1f} KiB",
           f"    read scale {f_scale:.4f}, write scale {w_scale:.4f} (bytes = KiB reading x 1024 x scale)", "",
           f"{'kernel':48s} {'grid':>9s} {'n':>5s} {'read_KiB':>11s} {'write_KiB':>11s}"]
    records = {}
    keys = sorted(set(fa) | set(wa), key=lambda k: (-len(fa.get(k, [])), k))
    for k in keys:
        if "tdb::" not in k[0]:
            continue
        fv, wv = fa.get(k, [0.0]), wa.get(k, [0.0])
        rd = sum(fv) / len(fv) * f_scale
        wr = sum(wv) / len(wv) * w_scale
        out.append(f"{_short(k[0])[:48]:48s} {k[1]:9d} {len(fv):5d} {rd:11.1f} {wr:11.1f}")
        for kern in PASS_KERNELS:
            # a kernel seen only in a batch's plan timing (a few launches on its first
            # snapshots) gives no record: those launches do not stream a step's data
            if len(fv) < 8:
                continue
            if ("tdb::" + kern + "(") in k[0] and (kern not in records or len(fv) > records[kern]["dispatches"]):
                records[kern] = {"kernel": kern, "dispatches": len(fv), "read_bytes": rd * 1024.0,
                                 "write_bytes": wr * 1024.0, "traffic_bytes": (rd + wr) * 1024.0,
                                 "read_scale": f_scale, "write_scale": w_scale,
                                 "source_digest": pass_source_digest(kern)}
    if records:
        out.append("")
        out += ["record: " + json.dumps(r) for r in records.values()]
    return "\n".join(out) + "\n", records


def read_pass_traffic(path: str, kernel: str = PASS_KERNEL):
    """The record of `kernel` in a `pmc` summary, or None when the file or the record is
    missing or the kernel's sources have changed since the counters were taken."""
    try:
        with open(path) as f:
            lines = [ln for ln in f.read().splitlines() if ln.startswith("record: ")]
    except OSError:
        return None
    for ln in reversed(lines):   # the last record of a kernel is the current one
        rec = json.loads(ln[len("record: "):])
        if rec.get("kernel") == kernel:
            return rec if rec.get("source_digest") == pass_source_digest(kernel) else None
    return None


def calibration_text(fetch_db: str, write_db: str, cmd_f: str, cmd_w: str) -> str:
    """FETCH_SIZE and WRITE_SIZE of the calibration kernels of `bench.py
    --calibrate-traffic` against their known footprints: the scale each implies for
    whole-line streaming (copy, read-only sum) and what the one-float-per-128-byte-line
    gather reads per line at the copy's scale."""
    fa, wa = _per_kernel(fetch_db), _per_kernel(write_db)
    MiB = 1024.0 * 1024.0

    def pick(agg, word):
        ks = [k for k in agg if word in k[0]]
        if not ks:
            return None
        k = max(ks, key=lambda q: max(agg[q]))
        return max(agg[k])
    copy_f, copy_w = pick(fa, "copyBuffer"), pick(wa, "copyBuffer")
    sum_f = pick(fa, "reduce_kernel")
    # the gather is the element-wise kernel that reads (the buffer's fill only writes);
    # its write reading is taken for the same kernel and grid
    gk = [k for k in fa if "elementwise_kernel" in k[0]]
    gkey = max(gk, key=lambda q: max(fa[q])) if gk else None
    gat_f = max(fa[gkey]) if gkey else None
    gat_w = max(wa[gkey]) if gkey and gkey in wa else None
    out = ["# traffic-counter calibration (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, KiB per dispatch)", "",
           "commands:", f"    {cmd_f}", f"    {cmd_w}", ""]
    if copy_f:
        sc = 256 * MiB / 1024.0 / copy_f
        out.append(f"copy of 256 MiB:   FETCH {copy_f:12.1f} KiB -> read scale {sc:.4f}; "
                   f"WRITE {copy_w or 0:12.1f} KiB -> write scale {256 * 1024.0 / copy_w if copy_w else float('nan'):.4f}")
        if sum_f:
            out.append(f"sum of 256 MiB:    FETCH {sum_f:12.1f} KiB -> read scale {256 * 1024.0 / sum_f:.4f} "
                       f"(copy's scale gives {sum_f * sc / 1024.0:.1f} MiB for 256 MiB read)")
        if gat_f:
            per_line = gat_f * 1024.0 * sc / (2 * MiB)
            out.append(f"gather, 1 float per 128 B line (2 Mi lines): FETCH {gat_f:12.1f} KiB -> at the copy's scale "
                       f"{per_line:.1f} B per line read; WRITE {gat_w or 0:.1f} KiB (8 MiB written)")
    return "\n".join(out) + "\n"


def counters_text(db: str, command: str, match: str) -> str:
    """Per-dispatch averages of every counter of a `--pmc` run for the kernels whose
    name contains `match` (one row per kernel and counter)."""
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
    cands = [c for c in cols if c == "counter_name"] + [c for c in cols if "counter" in c and "name" in c]
    if not cands:
        raise SystemExit(f"no counter-name column among {cols}")
    name_col = cands[0]
    rows = con.execute(f"select kernel_name, {name_col}, value from counters_collection").fetchall()
    agg = defaultdict(list)
    for k, c, v in rows:
        if match in k:
            agg[(_short(k), c)].append(v)
    out = ["# rocprofv3 --pmc (counters per dispatch)", "", "command:", f"    {command}", "",
           f"{'kernel':40s} {'counter':34s} {'n':>5s} {'avg_per_dispatch':>18s}"]
    for (k, c), vals in sorted(agg.items()):
        out.append(f"{k[:40]:40s} {c[:34]:34s} {len(vals):5d} {sum(vals) / len(vals):18.1f}")
    return "\n".join(out) + "\n"


def step_timeline(rows, first):
    """rows: (name, start_ns, end_ns) in start order. Steps begin at each kernel whose name
    contains `first`; returns [(span_us, busy_us, kernels)] for the complete steps and the
    kernels of the last complete step as (name, start_us, end_us) from its start."""
    marks = [i for i, r in enumerate(rows) if first in r[0]]
    steps, last = [], []
    for a, b in zip(marks, marks[1:]):
        seg = rows[a:b]
        iv = sorted((st, en) for _, st, en in seg)
        busy, cs, ce = 0, iv[0][0], iv[0][1]
        for st, en in iv[1:]:
            if st > ce:
                busy += ce - cs
                cs, ce = st, en
            else:
                ce = max(ce, en)
        busy += ce - cs
        span = max(en for _, _, en in seg) - seg[0][1]
        steps.append((span / 1e3, busy / 1e3, len(seg)))
        t0 = seg[0][1]
        last = [(n, (st - t0) / 1e3, (en - t0) / 1e3) for n, st, en in seg]
    return steps, last


def timeline_text(db: str, command: str, first: str = "kb_fetch_ptrs", nsteps: int = 10) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    con.close()
    rows = [(_short(str(n)), int(st), int(en)) for n, st, en in rows if "tdb::" in str(n)]
    steps, last = step_timeline(rows, first)
    out = ["# rocprofv3 --kernel-trace: timeline of the library's kernels per step", "",
           "command:", "    " + command, "",
           f"steps start at each launch of {first}; the last {min(nsteps, len(steps))} complete steps "
           "(busy: time some kernel was running)", ""]
    for span, busy, k in steps[-nsteps:]:
        out.append(f"    span {span:8.1f} us   busy {busy:8.1f} us   kernels {k}")
    out += ["", "the last complete step (us from its first kernel's start):", "",
            f"{'start':>9} {'end':>9} {'length':>8}  kernel"]
    for n, st, en in last:
        out.append(f"{st:9.1f} {en:9.1f} {en - st:8.1f}  {n[:90]}")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    cb = sub.add_parser("calib")
    cb.add_argument("fetch_db")
    cb.add_argument("write_db")
    cb.add_argument("--command-fetch", required=True)
    cb.add_argument("--command-write", required=True)
    cb.add_argument("--out")
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--command", required=True)
    s.add_argument("--bench", help="stdout of the profiled bench.py run")
    s.add_argument("--bench-plain", help="JSON line of an unprofiled bench.py run of the same build")
    s.add_argument("--out")
    p = sub.add_parser("pmc")
    p.add_argument("fetch_db")
    p.add_argument("write_db")
    p.add_argument("--command-fetch", required=True)
    p.add_argument("--command-write", required=True)
    p.add_argument("--copy-bytes", type=int, default=256 * 1024 * 1024)
    p.add_argument("--out")
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("--command", required=True)
    c.add_argument("--match", default="tdb::")
    c.add_argument("--out")
    t = sub.add_parser("timeline")
    t.add_argument("db")
    t.add_argument("--command", required=True)
    t.add_argument("--first", default="kb_fetch_ptrs", help="the first kernel of a step")
    t.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "timeline":
        text = timeline_text(a.db, a.command, a.first)
    elif a.cmd == "stats":
        text = stats_text(a.db, a.command, a.bench, a.bench_plain)
    elif a.cmd == "counters":
        text = counters_text(a.db, a.command, a.match)
    elif a.cmd == "calib":
        text = calibration_text(a.fetch_db, a.write_db, a.command_fetch, a.command_write)
    else:
        text, _ = pmc_text(a.fetch_db, a.write_db, a.command_fetch, a.command_write, a.copy_bytes)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text, end="")


if __name__ == "__main__":
    main()
