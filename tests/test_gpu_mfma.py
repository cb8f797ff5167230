"""GPU parity of the matrix-core stage pass in its two flavours: FP32 products
(bar 1e-6 relative, as every FP32 path) and BF16-split products (bar 1e-4 relative),
against the FP64 oracle on the same snapshots; the generic stage pass (TDB_MFMA=0)
on the same cases for comparison. Shapes cover ragged tiles in both tiled modes,
ranks on both sides of 16, third modes of 3 to 8 entries, full and deficient
third-mode ranks."""
import os
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import fourier_ensemble_specs, plume_spec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = {"f32": 1e-6, "bf16s": 1e-4}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _sigma_rel(sig_dev, sig_orc):
    """Largest difference of the leading (up to 16) core singular values per mode,
    relative to the mode's largest: the core compared through its invariants (after a
    reinitialisation the bases of two runs may differ by rotations within clusters of
    close singular values)."""
    worst = 0.0
    for sd, so in zip(sig_dev, sig_orc):
        k = min(len(sd), len(so), 16)
        worst = max(worst, float(np.abs(np.asarray(sd[:k]) - so[:k]).max() / so[0]))
    return worst


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_06958_amd import load_library
    load_library()


@pytest.fixture
def pass_kernel(request):
    old = os.environ.get("TDB_MFMA")
    os.environ["TDB_MFMA"] = "0" if request.param == "generic" else "1"
    yield request.param
    if old is None:
        os.environ.pop("TDB_MFMA", None)
    else:
        os.environ["TDB_MFMA"] = old


CASES = [((37, 70, 5), (17, 9, 3)), ((50, 130, 7), (32, 20, 7)), ((21, 65, 8), (8, 32, 4)),
         ((16, 64, 4), (16, 16, 4)), ((90, 40, 3), (24, 17, 2)),
         # one 16 x 32 tile per compute unit (sixteen waves): exact tiles with 16-byte
         # fiber loads; ragged tiles in both modes, a 6-entry third mode, ranks past 16;
         # 16 x 64 tiles (two fibers per loading thread) with a 4-entry third mode
         ((256, 512, 8), (15, 15, 4)), ((250, 500, 6), (20, 18, 4)), ((512, 512, 4), (12, 10, 3))]


def _mpass_waves(dims):
    """Waves per tile the library's single-stream plan gives a matrix-core pass: T2
    halves from 64 (not below 16) while there are fewer than 256 tiles of 16 x T2;
    sixteen waves for at most 256 tiles with T2 >= 32, eight for at most 512."""
    n1, n2 = dims[0], dims[1]
    t2 = 64
    while t2 > 16 and -(-n1 // 16) * -(-n2 // t2) < 256:
        t2 //= 2
    tiles = -(-n1 // 16) * -(-n2 // t2)
    return 16 if tiles <= 256 and t2 >= 32 else (8 if tiles <= 512 else 4)


def test_cases_cover_every_single_stream_tile_shape():
    assert {_mpass_waves(d) for d, _ in CASES} == {8, 16}


@pytest.mark.parametrize("pass_kernel,precision", [("mfma", "f32"), ("mfma", "bf16s"), ("generic", "f32")],
                         indirect=["pass_kernel"])
@pytest.mark.parametrize("dims,ranks", CASES)
def test_fixed_rank_random_streams(dims, ranks, pass_kernel, precision):
    """FP32 snapshots around a low-rank base with random weights, fixed ranks, started
    from the oracle's factors: reconstruction, core and eps against the oracle."""
    _say(f"case mfma-pass {pass_kernel} {precision} dims {dims} ranks {ranks} waves {_mpass_waves(dims)}")
    rng = np.random.default_rng(sum(dims) + 7)
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = rng.normal(size=dims)
    snaps = [(base + 0.002 * k * rng.normal(size=dims)).astype(np.float32) for k in range(7)]
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks, adaptive=False, eps_th=1.0)
    orc = O.OracleTDB(cfg).init(snaps[0].astype(np.float64))
    from paper_2201_06958_amd import Compressor
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f32", precision=precision,
                   adaptive=False, path="fused", eps_th=1.0)
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    bar = BAR[precision]
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k].astype(np.float64))
        g.ingest(_dev(snaps[k]))
        assert abs(g.stats()["eps"] - rec.eps) <= bar * rec.nu, k
    r, C, U = g.get_core_and_bases()
    rel = _rel(O.reconstruct(C, U), orc.reconstruct())
    relc = _rel(C, orc.C)
    _say(f"  reconstruction rel {rel:.2e}, core rel {relc:.2e}")
    # both runs start from the same factors and evolve by the same smooth equations,
    # so the core is compared as it is (same gauge), at the stated bar
    assert rel < bar and relc < bar
    g.close()


# Ranks above 32 (the reactive-flow stream's caps are (64, 64, 8)): the generic stage
# pass takes them, or the plain path where the fused step's small kernels do not fit
# in LDS; a BF16-split request there runs FP32 products. The statistics report which.
HIGH_RANK_CASES = [((150, 130, 8), (40, 36, 6)), ((200, 96, 8), (64, 48, 8)), ((97, 110, 6), (33, 40, 5))]


@pytest.mark.parametrize("precision", ["f32", "bf16s"])
@pytest.mark.parametrize("dims,ranks", HIGH_RANK_CASES)
def test_fixed_rank_high_ranks(dims, ranks, precision):
    _say(f"case high-rank {precision} dims {dims} ranks {ranks}")
    rng = np.random.default_rng(sum(dims) + sum(ranks))
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = np.zeros(dims)
    for q in range(max(ranks) + 8):
        a = [rng.normal(size=n) for n in dims]
        base += 0.9 ** q * np.einsum("i,j,k->ijk", *a)
    snaps = [(base + 0.002 * k * rng.normal(size=dims)).astype(np.float32) for k in range(6)]
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks, adaptive=False, eps_th=1.0)
    h = O.hosvd(snaps[0].astype(np.float64), w, ranks)
    C0, U0 = h.truncate(ranks)
    orc = O.OracleTDB(cfg).init_from_factors(snaps[0].astype(np.float64), C0, U0)
    from paper_2201_06958_amd import Compressor
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f32", precision=precision,
                   adaptive=False, path="fused", eps_th=1.0)
    g.init_from_factors(_dev(snaps[0]), C0, U0)
    bar = BAR[precision]
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k].astype(np.float64))
        g.ingest(_dev(snaps[k]))
        st = g.stats()
        assert abs(st["eps"] - rec.eps) <= bar * rec.nu, k
    r, C, U = g.get_core_and_bases()
    rel = _rel(O.reconstruct(C, U), orc.reconstruct())
    relc = _rel(C, orc.C)
    st = g.stats()
    _say(f"  ran {st['path_used']} {st['precision_used']}: reconstruction rel {rel:.2e}, core rel {relc:.2e}")
    assert st["path_used"] in ("fused", "plain")
    assert st["fused_steps"] + st["plain_steps"] == len(snaps) - 1
    assert st["precision_used"] in (("f32",) if precision == "f32" else ("f32", "bf16s"))
    assert rel < bar and relc < bar
    g.close()


@pytest.mark.parametrize("precision", ["f32", "bf16s"])
def test_plume_adaptive(precision):
    """Reactive-flow-shaped stream (8 variables: the third mode is not full rank, so
    the third-mode terms run too), adaptive ranks, matrix-core pass."""
    sp = plume_spec(nx=128, ny=64, nv=8, steps=20)
    _say(f"case mfma plume 128x64x8 {precision}")
    snaps = [sp.snapshot_np(k) for k in range(sp.steps + 1)]
    orc = O.OracleTDB(O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(32, 32, 8),
                                     rank_init=None, adaptive=True, eps_th=sp.eps_th)).init(snaps[0].astype(np.float64))
    from paper_2201_06958_amd import Compressor
    g = Compressor(sp.dims, sp.dt, rank_max=(32, 32, 8), weights=sp.weights, data_dtype="f32", precision=precision,
                   adaptive=True, eps_th=sp.eps_th)
    g.init(_dev(snaps[0]))
    bar = BAR[precision]
    for k in range(1, sp.steps + 1):
        rec = orc.ingest(snaps[k].astype(np.float64))
        g.ingest(_dev(snaps[k]))
        st = g.stats()
        assert st["event"] == rec.event, k
        assert abs(st["eps"] - rec.eps) <= bar * rec.nu, k
    r, C, U = g.get_core_and_bases()
    rel = _rel(O.reconstruct(C, U), orc.reconstruct())
    rels = _sigma_rel(g.stats()["sigma"], O.core_singular_values(orc.C))
    _say(f"  ranks {r}, reconstruction rel {rel:.2e}, core singular values rel {rels:.2e}")
    assert rel < bar and rels < bar
    g.close()


@pytest.mark.parametrize("precision", ["f32", "bf16s"])
def test_batch_ensemble(precision):
    """Three ensemble members in one batch on the matrix-core pass."""
    steps = 6
    specs = fourier_ensemble_specs(n_streams=3, steps=steps, seed0=2000)
    _say(f"case mfma batch {[sp.dims for sp in specs]} {precision}")
    from paper_2201_06958_amd import Batch
    data = [[sp.snapshot_np(k) for k in range(steps + 1)] for sp in specs]
    cfgs, orcs = [], []
    for sp, d in zip(specs, data):
        cfgs.append(dict(dims=sp.dims, dt=sp.dt, rank_max=sp.rank_max, weights=sp.weights, data_dtype="f32",
                         precision=precision, adaptive=True, eps_th=sp.eps_th))
        orcs.append(O.OracleTDB(O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                                               rank_init=None, adaptive=True, eps_th=sp.eps_th))
                    .init(d[0].astype(np.float64)))
    b = Batch(cfgs).init([_dev(d[0]) for d in data])
    bar = BAR[precision]
    for k in range(1, steps + 1):
        b.ingest([_dev(d[k]) for d in data])
        for i, o in enumerate(orcs):
            rec = o.ingest(data[i][k].astype(np.float64))
            st = b.streams[i].stats()
            assert st["event"] == rec.event, (k, i)
            assert abs(st["eps"] - rec.eps) <= bar * rec.nu, (k, i)
    for i, o in enumerate(orcs):
        r, C, U = b.streams[i].get_core_and_bases()
        rel = _rel(O.reconstruct(C, U), o.reconstruct())
        rels = _sigma_rel(b.streams[i].stats()["sigma"], O.core_singular_values(o.C))
        _say(f"  stream {i} {specs[i].dims} ranks {r}: reconstruction rel {rel:.2e}, sigma rel {rels:.2e}")
        assert rel < bar and rels < bar
    b.close()


@pytest.mark.parametrize("cols", [32, 64])
@pytest.mark.parametrize("precision", ["f32", "bf16s"])
def test_batch_ensemble_column_counts(cols, precision):
    """The column-block pass with 32 and with 64 columns of mode 2 per workgroup (the two
    shapes the batch's tuner chooses between for a mode-3 extent of 4), forced, against
    the oracle."""
    old = os.environ.get("TDB_RPASS_COLS")
    os.environ["TDB_RPASS_COLS"] = str(cols)
    try:
        steps = 5
        specs = fourier_ensemble_specs(n_streams=3, steps=steps, seed0=2100)
        _say(f"case column-block pass {cols} columns {precision} {[sp.dims for sp in specs]}")
        from paper_2201_06958_amd import Batch
        data = [[sp.snapshot_np(k) for k in range(steps + 1)] for sp in specs]
        cfgs, orcs = [], []
        for sp, d in zip(specs, data):
            cfgs.append(dict(dims=sp.dims, dt=sp.dt, rank_max=sp.rank_max, weights=sp.weights, data_dtype="f32",
                             precision=precision, adaptive=True, eps_th=sp.eps_th))
            orcs.append(O.OracleTDB(O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                                                   rank_init=None, adaptive=True, eps_th=sp.eps_th))
                        .init(d[0].astype(np.float64)))
        b = Batch(cfgs).init([_dev(d[0]) for d in data])
    finally:
        if old is None:
            os.environ.pop("TDB_RPASS_COLS", None)
        else:
            os.environ["TDB_RPASS_COLS"] = old
    pl = b.plan()
    assert pl["pass"] == "matrix-core-columns" and pl["pass_cols"] == cols and pl["source"] == "rule", pl
    bar = BAR[precision]
    for k in range(1, steps + 1):
        b.ingest([_dev(d[k]) for d in data])
        for i, o in enumerate(orcs):
            rec = o.ingest(data[i][k].astype(np.float64))
            st = b.streams[i].stats()
            assert st["event"] == rec.event, (k, i)
            assert abs(st["eps"] - rec.eps) <= bar * rec.nu, (k, i)
    for i, o in enumerate(orcs):
        r, C, U = b.streams[i].get_core_and_bases()
        rel = _rel(O.reconstruct(C, U), o.reconstruct())
        rels = _sigma_rel(b.streams[i].stats()["sigma"], O.core_singular_values(o.C))
        assert rel < bar and rels < bar, (i, rel, rels)
    b.close()


def test_batch_plan_tuned_then_cached():
    """The batch's plan: timed at the first creation for a shape class (two or more stage-
    pass candidates and both error passes timed), the same plan from the cache at the
    second, the fixed rule with TDB_AUTOTUNE=0."""
    specs = fourier_ensemble_specs(n_streams=4, steps=2, seed0=2200)
    from paper_2201_06958_amd import Batch

    def make():
        cfgs = [dict(dims=sp.dims, dt=sp.dt, rank_max=sp.rank_max, weights=sp.weights, data_dtype="f32",
                     precision="f32", adaptive=True, eps_th=sp.eps_th, snapshot_mode="borrow") for sp in specs]
        return Batch(cfgs).init([sp.snapshot(0, device="cuda") for sp in specs])

    _say("case batch plan tuner")
    b1 = make()
    p1 = b1.plan()
    _say("  ", p1)
    assert p1["source"] in ("timed", "cached"), p1
    if p1["source"] == "timed":
        assert sum(1 for x in p1["pass_us"] if x > 0) >= 2 and all(x > 0 for x in p1["err_us"]), p1
    b1.close()
    b2 = make()
    p2 = b2.plan()
    assert p2["source"] == "cached" and {k: p2[k] for k in ("pass", "pass_cols", "error_pass")} == \
        {k: p1[k] for k in ("pass", "pass_cols", "error_pass")}, (p1, p2)
    b2.close()
    old = os.environ.get("TDB_AUTOTUNE")
    os.environ["TDB_AUTOTUNE"] = "0"
    try:
        b3 = make()
    finally:
        if old is None:
            os.environ.pop("TDB_AUTOTUNE", None)
        else:
            os.environ["TDB_AUTOTUNE"] = old
    p3 = b3.plan()
    assert p3["source"] == "rule" and p3["pass"] == "matrix-core-columns" and p3["pass_cols"] == 64, p3
    b3.close()
