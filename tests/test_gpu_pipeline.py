"""Pipelined ingest (borrowed snapshots, fused path): each call enqueues its step and
reads the previous step's decision afterwards. The result must be the synchronous
ingest's, bit for bit, including across add, removal and reinitialisation events, and
whichever calls happen to read the decisions."""
import math
import sys

import numpy as np
import pytest

from streams import plume_spec, switched_term_spec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_06958_amd import load_library
    load_library()


def _switched():
    t_on, t_peak, t_low, h_min = 0.05, 0.15, 0.35, 0.002

    def h(t):
        if t <= t_on:
            return 0.0
        if t <= t_peak:
            return 2.0 * (t - t_on)
        if t <= t_low:
            return 0.2 + (h_min - 0.2) * (t - t_peak) / (t_low - t_peak)
        return h_min

    return switched_term_spec(steps=140, profile=h, profile2=lambda t: 0.004 * math.exp(-t))


def _run(sp, snaps, mode, precision, read_every, rank_max=None):
    """Ingest every snapshot; read the statistics after every `read_every`-th call
    (0: only at the end). Returns (events seen, final stats, ranks, core, bases)."""
    from paper_2201_06958_amd import Compressor
    g = Compressor(sp.dims, sp.dt, rank_max=rank_max or sp.rank_max, rank_init=sp.rank_init, weights=sp.weights,
                   data_dtype=sp.storage, precision=precision, path="fused", adaptive=sp.adaptive,
                   eps_th=sp.eps_th if sp.eps_th > 0 else 1.0, snapshot_mode=mode)
    g.init(snaps[0])
    events = []
    for k in range(1, len(snaps)):
        g.ingest(snaps[k])
        if read_every and k % read_every == 0:
            st = g.stats()
            if st["event"]:
                events.append((k, st["event"], st["ranks"]))
    g.flush()
    st = g.stats()
    r, C, U = g.get_core_and_bases()
    g.close()
    return events, st, r, C, U


def _same(a, b):
    ea, sa, ra, Ca, Ua = a
    eb, sb, rb, Cb, Ub = b
    assert ra == rb
    assert np.array_equal(Ca, Cb)
    for x, y in zip(Ua, Ub):
        assert np.array_equal(x, y)
    for key in ("eps", "nu", "n_add", "n_remove", "n_reinit", "n_numeric", "crbar"):
        assert sa[key] == sb[key], key


def test_pipelined_switched_stream_matches_synchronous():
    sp = _switched()
    _say("case pipelined ingest, switched-term stream 140 steps, fused FP64")
    snaps = [torch.from_numpy(np.ascontiguousarray(sp.snapshot_np(k))).to("cuda") for k in range(sp.steps + 1)]
    torch.cuda.synchronize()
    sync_each = _run(sp, snaps, "copy", "f64", 1)
    assert sync_each[1]["n_add"] >= 1 and sync_each[1]["n_remove"] >= 1, "the stream must exercise both events"
    pipe_each = _run(sp, snaps, "borrow", "f64", 1)
    assert pipe_each[0] == sync_each[0]
    _same(pipe_each, sync_each)
    for every in (0, 7):
        _same(_run(sp, snaps, "borrow", "f64", every), sync_each)
    _say("  events", sync_each[0])


def test_pipelined_plume_fp32_matches_synchronous():
    sp = plume_spec(nx=128, ny=64, nv=8, steps=30)
    _say("case pipelined ingest, plume 128x64x8 FP32 30 steps")
    snaps = [torch.from_numpy(np.ascontiguousarray(sp.snapshot_np(k))).to("cuda") for k in range(sp.steps + 1)]
    torch.cuda.synchronize()
    ref = _run(sp, snaps, "copy", "f32", 1, rank_max=(32, 32, 8))
    _same(_run(sp, snaps, "borrow", "f32", 0, rank_max=(32, 32, 8)), ref)


def test_pass_timing_sampled_every_kth_step():
    """Pass timing of every k-th step: 2 projection launches and 1 error launch per
    timed step, none in between; every step timed with k = 1."""
    _say("case pass timing sampled")
    sp = plume_spec(nx=64, ny=32, nv=8, steps=13)
    snaps = [sp.snapshot(k, device="cuda") for k in range(13)]
    from paper_2201_06958_amd import Compressor
    for every, timed in ((1, 12), (4, 3), (5, 3)):
        g = Compressor(sp.dims, sp.dt, rank_max=(16, 16, 8), weights=sp.weights, data_dtype="f32",
                       precision="f32", adaptive=False, rank_init=(6, 6, 3), eps_th=1.0)
        g.init(snaps[0])
        g.profile_enable(True, every=every)
        for k in range(1, 13):
            g.ingest(snaps[k])
        g.flush()
        pj, er = g.profile_read("project"), g.profile_read("error")
        assert pj["launches"] == 2 * timed, (every, pj)
        assert er["launches"] == timed, (every, er)
        assert pj["total_ms"] > 0.0
        g.close()


# ---------------------------------------------------------------- batches

def _switched_at(t_on, t_peak, t_low, seed, dims):
    h_min = 0.002

    def h(t):
        if t <= t_on:
            return 0.0
        if t <= t_peak:
            return 2.0 * (t - t_on)
        if t <= t_low:
            return 0.2 + (h_min - 0.2) * (t - t_peak) / (t_low - t_peak)
        return h_min

    return switched_term_spec(dims=dims, steps=120, seed=seed, profile=h, profile2=lambda t: 0.004 * math.exp(-t))


def _run_batch(specs, snaps, mode, precision, read_every, env, rank_max=None):
    """Ingest every step of a batch; read every member's statistics after every
    `read_every`-th call (0: only at the end). Returns (events, per-member results)."""
    import os
    from paper_2201_06958_amd import Batch
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        cfgs = [dict(dims=sp.dims, dt=sp.dt, rank_max=rank_max or sp.rank_max, rank_init=sp.rank_init,
                     weights=sp.weights, data_dtype=sp.storage, precision=precision, adaptive=sp.adaptive,
                     eps_th=sp.eps_th if sp.eps_th > 0 else 1.0, snapshot_mode=mode) for sp in specs]
        b = Batch(cfgs).init([s[0] for s in snaps])
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    events = []
    steps = len(snaps[0]) - 1
    for k in range(1, steps + 1):
        b.ingest([s[k] for s in snaps])
        if read_every and k % read_every == 0:
            for i, m in enumerate(b.streams):
                st = m.stats()
                if st["event"]:
                    events.append((k, i, st["event"], st["ranks"]))
    b.flush()
    res = []
    for m in b.streams:
        st = m.stats()
        r, C, U = m.get_core_and_bases()
        res.append((events, st, r, C, U))
    b.close()
    return events, res


def _same_batch(a, b):
    for x, y in zip(a[1], b[1]):
        _same(x, y)


def test_batch_pipelined_and_graphs_match_synchronous():
    """Two switched-term streams whose add and removal steps differ (so a step runs again
    for one member while the other went on), FP64: the pipelined batch, with the step's
    launches replayed from graphs or issued one by one, and whichever calls read the
    decisions, equals the synchronous batch bit for bit."""
    specs = [_switched_at(0.05, 0.15, 0.35, 3, (16, 14, 6)), _switched_at(0.12, 0.2, 0.45, 5, (18, 12, 5))]
    _say("case pipelined batch, two switched-term streams 120 steps, FP64")
    snaps = [[torch.from_numpy(np.ascontiguousarray(sp.snapshot_np(k))).to("cuda") for k in range(sp.steps + 1)]
             for sp in specs]
    torch.cuda.synchronize()
    ref = _run_batch(specs, snaps, "copy", "f64", 1, {"TDB_GRAPH": "0"})
    ev = ref[0]
    assert {e[1] for e in ev if e[2] == "add"} == {0, 1}, ev      # both members add
    assert {e[1] for e in ev if e[2] == "remove"} == {0, 1}, ev   # and remove
    assert len({e[0] for e in ev}) == len(ev), ev                # never on the same step
    _say("  events", ev)
    for env in ({"TDB_GRAPH": "1"}, {"TDB_GRAPH": "0"}):
        for every in (1, 0, 5):
            _say("  borrow", env, "read every", every)
            got = _run_batch(specs, snaps, "borrow", "f64", every, env)
            if every == 1:
                assert got[0] == ev
            graphs = got[1][0][1]["graph_steps"]
            # every step and every run again for held members, all but the captures
            assert (graphs >= 100) if env["TDB_GRAPH"] == "1" else (graphs == 0), graphs
            _same_batch(got, ref)
    # the synchronous batch with graphs is the same too
    _same_batch(_run_batch(specs, snaps, "copy", "f64", 0, {"TDB_GRAPH": "1"}), ref)


def test_batch_pipelined_fp32_mixed_matches_synchronous():
    """A reactive-flow stream (8 variables) and two Fourier ensemble members (4
    variables) in one FP32 batch, adaptive ranks: pipelined with graphs against the
    synchronous batch, bit for bit."""
    from streams import fourier_ensemble_specs
    pl = plume_spec(nx=96, ny=64, nv=8, steps=24)
    fe = fourier_ensemble_specs(n_streams=2, steps=24, seed0=3000)
    specs = [pl] + fe
    _say("case pipelined batch FP32", [sp.dims for sp in specs])
    snaps = [[sp.snapshot(k, device="cuda") for k in range(25)] for sp in specs]
    torch.cuda.synchronize()
    ref = _run_batch(specs, snaps, "copy", "f32", 0, {"TDB_GRAPH": "0"}, rank_max=(24, 24, 4))
    got = _run_batch(specs, snaps, "borrow", "f32", 0, {"TDB_GRAPH": "1"}, rank_max=(24, 24, 4))
    assert got[1][0][1]["graph_steps"] >= 20
    _same_batch(got, ref)
