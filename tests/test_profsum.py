"""Host logic of the rocprofv3 summary module (no GPU): counter calibration against a
copy of known size, the stage-pass record and its source-digest check."""
import json
import sqlite3

from paper_2201_06958_amd import profsum


def _counter_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, grid_size int, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()


def test_pmc_scaling_and_record(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    kpass = "void tdb::k_mpass_w16<float, 1>(tdb::FPassArgs)"
    # the copy of 1 MiB reads as 512 KiB on FETCH and 1024 KiB on WRITE -> scales 2 and 1
    f = tmp_path / "f.db"
    w = tmp_path / "w.db"
    # eight dispatches of the pass (a record), four of a batch pass seen only while a
    # plan was being timed (no record)
    ktune = "void tdb::kb_rpass<float, 1, 4, true, 32>(tdb::FPassArgs)"
    _counter_db(f, [(copy, 4096, 512.0), (copy, 64, 1.0)] + [(kpass, 1000, 100.0), (kpass, 1000, 110.0)] * 4
                + [(ktune, 500, 50.0)] * 4)
    _counter_db(w, [(copy, 4096, 1024.0), (copy, 64, 1.0)] + [(kpass, 1000, 20.0)] * 8 + [(ktune, 500, 5.0)] * 4)
    text, recs = profsum.pmc_text(str(f), str(w), "cmd f", "cmd w", 1024 * 1024)
    assert "kb_rpass<float, 1, 4, true, 32>" not in recs
    rec = recs["k_mpass_w16<float, 1>"]
    assert abs(rec["read_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert abs(rec["read_bytes"] - 105.0 * 2 * 1024) < 1e-6
    assert abs(rec["write_bytes"] - 20.0 * 1024) < 1e-6
    assert rec["source_digest"] == profsum.pass_source_digest("k_mpass_w16<float, 1>")
    out = tmp_path / "traffic.txt"
    out.write_text(text)
    assert profsum.read_pass_traffic(str(out))["traffic_bytes"] == rec["traffic_bytes"]
    # a record taken from other sources is ignored
    stale = dict(rec, source_digest="0" * 16)
    out.write_text(text + "record: " + json.dumps(stale) + "\n")
    assert profsum.read_pass_traffic(str(out)) is None
    assert profsum.read_pass_traffic(str(tmp_path / "missing.txt")) is None


def test_stats_text(tmp_path):
    db = tmp_path / "s.db"
    con = sqlite3.connect(db)
    con.execute("create table top_kernels (name text, total_calls int, total_duration real, "
                "average real, percentage real)")
    con.executemany("insert into top_kernels values (?, ?, ?, ?, ?)",
                    [("void tdb::k_mpass_w16<float, 1>(tdb::FPassArgs)", 10, 450.0, 45.0, 60.0),
                     ("tdb::k_fqr(tdb::FQrArgs, CtrlState*)", 5, 300.0, 60.0, 40.0)])
    con.commit()
    con.close()
    text = profsum.stats_text(str(db), "the command")
    assert "tdb::k_mpass_w16<float, 1>" in text and "the command" in text
    assert text.index("k_mpass") < text.index("k_fqr")


def test_counters_text(tmp_path):
    db = tmp_path / "c.db"
    con = sqlite3.connect(db)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)",
                    [("void tdb::kb_rpass<float, 1, 4, true>(x)", "SQ_INSTS_MFMA", 100.0),
                     ("void tdb::kb_rpass<float, 1, 4, true>(x)", "SQ_INSTS_MFMA", 300.0),
                     ("void other(x)", "SQ_INSTS_MFMA", 7.0)])
    con.commit()
    con.close()
    text = profsum.counters_text(str(db), "cmd", "kb_rpass")
    row = [ln for ln in text.splitlines() if "SQ_INSTS_MFMA" in ln]
    assert len(row) == 1 and row[0].split()[-1] == "200.0" and row[0].split()[-2] == "2"


def test_step_timeline(tmp_path):
    """Steps split at the first kernel; busy time is the union of overlapping kernels."""
    rows = [("tdb::kb_fetch_ptrs", 0, 5_000), ("tdb::kb_rpass<float>", 5_000, 105_000),
            ("tdb::kb_fpost<float, 1>", 110_000, 150_000), ("tdb::kb_fpost<float, 2>", 120_000, 200_000),
            ("tdb::kb_fetch_ptrs", 210_000, 215_000), ("tdb::kb_rpass<float>", 215_000, 300_000),
            ("tdb::kb_fetch_ptrs", 310_000, 311_000)]
    steps, last = profsum.step_timeline(rows, "kb_fetch_ptrs")
    assert len(steps) == 2
    span, busy, k = steps[0]
    assert abs(span - 200.0) < 1e-9 and abs(busy - 195.0) < 1e-9 and k == 4
    assert abs(steps[1][0] - 90.0) < 1e-9 and abs(steps[1][1] - 90.0) < 1e-9
    assert last[0][1] == 0.0 and abs(last[-1][2] - 90.0) < 1e-9
    db = tmp_path / "k.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int)")
    con.executemany("insert into kernels values (?, ?, ?)", [(f"void {n}(x)", a, b) for n, a, b in rows])
    con.commit()
    con.close()
    text = profsum.timeline_text(str(db), "the command")
    assert "the command" in text and "busy    195.0 us" in text
