"""GPU parity of the batched path: several independent streams of uneven shapes and
ranks advanced by one set of launches per step, each stream checked against its own
FP64 CPU oracle run on the same snapshots.

Bars as for single streams: FP64 1e-9 relative on reconstructions and projectors
(the batch initialises by a device HOSVD), FP32 1e-6 relative; controller events
identical.
"""
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import fourier_ensemble_specs, plume_spec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_06958_amd import load_library
    load_library()


def _random_stream(dims, ranks, seed, steps):
    rng = np.random.default_rng(seed)
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = rng.normal(size=dims)
    snaps = [base + 0.005 * k * rng.normal(size=dims) for k in range(steps + 1)]
    return w, snaps


def test_batch_fp64_fixed_ranks_against_oracle():
    """Three FP64 streams (a ragged tile in both tiled modes, a full-rank third mode,
    non-uniform weights), fixed ranks: every stream's state vs its oracle per step."""
    cases = [((20, 17, 9), (3, 4, 2)), ((16, 12, 3), (4, 3, 3)), ((70, 130, 5), (6, 5, 4))]
    steps = 6
    from paper_2201_06958_amd import Batch
    data, cfgs, orcs = [], [], []
    for i, (dims, ranks) in enumerate(cases):
        w, snaps = _random_stream(dims, ranks, 100 + i, steps)
        data.append(snaps)
        cfgs.append(dict(dims=dims, dt=0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f64",
                         precision="f64", adaptive=False, eps_th=1.0))
        oc = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks, adaptive=False,
                            eps_th=1.0)
        orcs.append(O.OracleTDB(oc).init(snaps[0]))
    _say("case batch fp64", cases)
    b = Batch(cfgs).init([_dev(d[0]) for d in data])
    for k in range(1, steps + 1):
        snaps_k = [_dev(d[k]) for d in data]
        b.ingest(snaps_k)
        for i, o in enumerate(orcs):
            rec = o.ingest(data[i][k])
            st = b.streams[i].stats()
            assert st["eps"] == pytest.approx(rec.eps, rel=1e-9), (k, i)
    for i, o in enumerate(orcs):
        r, C, U = b.streams[i].get_core_and_bases()
        assert r == o.ranks
        assert _rel(O.reconstruct(C, U), o.reconstruct()) < 1e-9, i
        for n in range(3):
            w = cfgs[i]["weights"][n]
            Pg = U[n] @ U[n].T * w[None, :]
            Po = o.U[n] @ o.U[n].T * w[None, :]
            assert np.abs(Pg - Po).max() < 1e-9, (i, n)
    b.close()


def test_batch_fp32_adaptive_mixed_shapes_against_oracle():
    """FP32 data and passes: three ensemble members (uneven grids from {128,192,256}^2,
    4 variables, caps 24, threshold 1e-5) and a reactive-flow-shaped stream (8
    variables, threshold 1e-4) in one batch; adaptive ranks from the rank rule."""
    steps = 8
    specs = fourier_ensemble_specs(n_streams=3, steps=steps) + [plume_spec(nx=96, ny=48, nv=8, steps=steps)]
    rank_max = [sp.rank_max for sp in specs[:3]] + [(24, 24, 8)]
    _say("case batch fp32", [sp.dims for sp in specs])
    from paper_2201_06958_amd import Batch
    data = [[sp.snapshot_np(k) for k in range(steps + 1)] for sp in specs]
    cfgs, orcs = [], []
    for sp, rm, d in zip(specs, rank_max, data):
        cfgs.append(dict(dims=sp.dims, dt=sp.dt, rank_max=rm, weights=sp.weights, data_dtype="f32",
                         precision="f32", adaptive=True, eps_th=sp.eps_th))
        oc = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=rm, rank_init=None,
                            adaptive=True, eps_th=sp.eps_th)
        orcs.append(O.OracleTDB(oc).init(d[0].astype(np.float64)))
    b = Batch(cfgs).init([_dev(d[0]) for d in data])
    for i, o in enumerate(orcs):
        assert b.streams[i].ranks() == o.ranks, i
    for k in range(1, steps + 1):
        b.ingest([_dev(d[k]) for d in data])
        for i, o in enumerate(orcs):
            rec = o.ingest(data[i][k].astype(np.float64))
            st = b.streams[i].stats()
            assert st["event"] == rec.event, (k, i)
            assert abs(st["eps"] - rec.eps) <= 1e-6 * rec.nu, (k, i)
    for i, o in enumerate(orcs):
        st = b.streams[i].stats()
        r, C, U = b.streams[i].get_core_and_bases()
        rel = _rel(O.reconstruct(C, U), o.reconstruct())
        so = O.core_singular_values(o.C)
        sig_rel = max(abs(st["sigma"][n][j] - so[n][j]) / so[n][0] for n in range(3)
                      for j in range(min(len(st["sigma"][n]), 16)))
        _say(f"  stream {i} {specs[i].dims}: ranks {r}, reconstruction rel {rel:.2e}, sigma rel {sig_rel:.2e}")
        assert rel < 1e-6, i
        assert sig_rel < 1e-6, i
    b.close()


def test_batch_stream_handles_are_owned_by_the_batch():
    """A batch member cannot be advanced on its own, and destroying its handle is a
    no-op (the batch frees it)."""
    from paper_2201_06958_amd import Batch, TDBError
    sp = plume_spec(nx=32, ny=16, nv=4, steps=2)
    cfg = dict(dims=sp.dims, dt=sp.dt, rank_max=(8, 8, 4), weights=sp.weights, data_dtype="f32", precision="f32",
               adaptive=True, eps_th=sp.eps_th)
    b = Batch([cfg]).init([_dev(sp.snapshot_np(0))])
    with pytest.raises(TDBError):
        b.streams[0].ingest(_dev(sp.snapshot_np(1)))
    b.streams[0].lib.tdb_destroy(b.streams[0].h)
    b.ingest([_dev(sp.snapshot_np(1))])
    assert b.streams[0].stats()["step"] == 1
    b.close()


def _tucker_walk(dims, ranks, seed, steps, amp=0.005):
    """A Tucker tensor with a diagonally dominant core (every unfolding well conditioned)
    plus a small random walk, in FP32."""
    rng = np.random.default_rng(seed)
    C = 0.2 * rng.normal(size=ranks)
    for i in range(min(ranks)):
        C[(i,) * len(ranks)] += 1.0 - 0.1 * i
    X = C
    for k, (N, r) in enumerate(zip(dims, ranks)):
        X = np.moveaxis(np.tensordot(rng.normal(size=(N, r)), X, axes=([1], [k])), 0, k)
    snaps = [X]
    for _ in range(steps):
        snaps.append(snaps[-1] + amp * rng.normal(size=dims))
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    return w, [s.astype(np.float32) for s in snaps]


def test_batch_fp32_ragged_shapes_against_oracle():
    """FP32 data and passes at fixed ranks on shapes that leave ragged tails everywhere:
    mode-1 sizes that are not multiples of the 16-row blocks of the matrix-core error
    pass, column counts N2*N3 that are not multiples of its 64-column waves, ranks that
    are not multiples of 4, a full-rank third mode. eps per step within 1e-6 of nu and
    the final reconstruction at 1e-6 relative, against the FP64 oracle fed the same
    rounded snapshots."""
    cases = [((20, 17, 9), (3, 4, 2)), ((37, 29, 3), (5, 4, 3)), ((70, 45, 5), (6, 5, 4))]
    steps = 6
    from paper_2201_06958_amd import Batch
    data, cfgs, orcs = [], [], []
    for i, (dims, ranks) in enumerate(cases):
        w, snaps = _tucker_walk(dims, ranks, 300 + i, steps)
        data.append(snaps)
        cfgs.append(dict(dims=dims, dt=0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f32",
                         precision="f32", adaptive=False, eps_th=1.0))
        oc = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks, adaptive=False,
                            eps_th=1.0)
        orcs.append(O.OracleTDB(oc).init(snaps[0].astype(np.float64)))
    _say("case batch fp32 ragged", cases)
    b = Batch(cfgs).init([_dev(d[0]) for d in data])
    for k in range(1, steps + 1):
        b.ingest([_dev(d[k]) for d in data])
        for i, o in enumerate(orcs):
            rec = o.ingest(data[i][k].astype(np.float64))
            st = b.streams[i].stats()
            assert abs(st["eps"] - rec.eps) <= 1e-6 * rec.nu, (k, i, st["eps"], rec.eps)
    for i, o in enumerate(orcs):
        r, C, U = b.streams[i].get_core_and_bases()
        assert tuple(r[:3]) == tuple(o.ranks)
        assert _rel(O.reconstruct(C, U), o.reconstruct()) < 1e-6, i
    b.close()
