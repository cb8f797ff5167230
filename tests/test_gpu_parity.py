"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on the
same seeded snapshots.

Bars: FP64 plain path 1e-10 relative (core, bases, reconstruction, eps); FP32 path
1e-6 relative on the reconstruction and core (spec tolerance); decisions of
the controller identical unless the oracle's error sits inside the ambiguity band
around the threshold it was compared with.
"""
import math
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import (analytic_cp5_spec, fourier_ensemble_specs, lowrank_manifold_spec, plume_spec,
                     switched_term_spec)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _cmp_cfg(sp, **kw):
    from paper_2201_06958_amd import Compressor
    args = dict(dims=sp.dims, dt=sp.dt, rank_max=sp.rank_max, rank_init=sp.rank_init,
                weights=sp.weights, data_dtype=sp.storage, precision="f64", adaptive=sp.adaptive,
                eps_th=sp.eps_th if sp.eps_th > 0 else 1.0)
    args.update(kw)
    return Compressor(**args)


def _ocfg(sp, **kw):
    args = dict(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                rank_init=sp.rank_init, adaptive=sp.adaptive,
                eps_th=sp.eps_th if sp.eps_th > 0 else 1.0)
    args.update(kw)
    return O.OracleConfig(**args)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _sigma_rel(sig_dev, sig_orc):
    """Largest difference of the leading (up to 16) core singular values per mode,
    relative to the mode's largest (the core compared through its invariants)."""
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


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_analytic_fp64_full_run_from_identical_factors(path):
    """64^3 analytic stream, fixed ranks (5,5,5), 200 Heun steps: every core entry,
    basis entry and error matches the oracle to 1e-10 relative."""
    sp = analytic_cp5_spec()
    _say(f"case analytic-cp5 64^3 fp64 {path}, 200 steps")
    snaps = [sp.snapshot_np(k) for k in range(sp.steps + 1)]
    orc = O.OracleTDB(_ocfg(sp)).init(snaps[0])
    g = _cmp_cfg(sp, path=path)
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, sp.steps + 1):
        rec = orc.ingest(snaps[k])
        g.ingest(_dev(snaps[k]))
        if k % 25 == 0 or k == sp.steps:
            r, C, U = g.get_core_and_bases()
            st = g.stats()
            _say(f"  step {k}: eps gpu {st['eps']:.6e} oracle {rec.eps:.6e}")
            assert r == orc.ranks
            assert _rel(C, orc.C) < 1e-10
            for n in range(3):
                assert _rel(U[n], orc.U[n]) < 1e-10
            assert abs(st["eps"] - rec.eps) <= 1e-8 * rec.nu + 1e-10 * rec.eps
            assert st["nu"] == pytest.approx(rec.nu, rel=1e-12)
    g.close()


def test_hosvd_init_matches_oracle():
    """Device HOSVD (Gram, tridiagonal eigensolver, projection) against the oracle's
    LAPACK eigendecomposition: projectors, core singular values, eps0."""
    sp = analytic_cp5_spec(n=48)
    _say("case hosvd-init analytic 48^3")
    V0 = sp.snapshot_np(3)
    orc = O.OracleTDB(_ocfg(sp)).init(V0)
    g = _cmp_cfg(sp)
    g.init(_dev(V0))
    r, C, U = g.get_core_and_bases()
    assert r == orc.ranks
    for n in range(3):
        w = sp.weights[n]
        Pg = U[n] @ U[n].T * w[None, :]
        Po = orc.U[n] @ orc.U[n].T * w[None, :]
        assert np.abs(Pg - Po).max() < 1e-9
    sg = O.core_singular_values(C)
    so = O.core_singular_values(orc.C)
    for n in range(3):
        assert np.allclose(sg[n], so[n], rtol=1e-10)
    rec_g = O.reconstruct(C, U)
    rec_o = O.reconstruct(orc.C, orc.U)
    assert _rel(rec_g, rec_o) < 1e-9
    g.close()


@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("dims,ranks", [((20, 17, 9), (3, 4, 2)), ((33, 8), (3, 3)),
                                        ((9, 7, 6, 5), (2, 3, 2, 2)), ((16, 12, 3), (4, 3, 3)),
                                        ((70, 130, 5), (6, 5, 4))])
def test_random_weighted_streams_fp64(dims, ranks, path):
    """Random non-uniform weights, random snapshots around a low-rank base, orders 2
    to 4 (the fused path covers order 3; other orders run the plain path), a
    full-rank mode, ragged tiles in both tiled modes: raw state parity per step."""
    _say(f"case random fp64 dims {dims} ranks {ranks} {path}")
    rng = np.random.default_rng(sum(dims))
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = rng.normal(size=dims)
    snaps = [base + 0.05 * k * rng.normal(size=dims) * 0.1 for k in range(8)]
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks,
                         adaptive=False, eps_th=1.0)
    orc = O.OracleTDB(cfg).init(snaps[0])
    from paper_2201_06958_amd import Compressor
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f64",
                   precision="f64", adaptive=False, path=path, eps_th=1.0)
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, 8):
        rec = orc.ingest(snaps[k])
        g.ingest(_dev(snaps[k]))
        r, C, U = g.get_core_and_bases()
        assert _rel(C, orc.C) < 1e-10, k
        for n in range(len(dims)):
            assert _rel(U[n], orc.U[n]) < 1e-10, (k, n)
        assert g.stats()["eps"] == pytest.approx(rec.eps, rel=1e-9)
    g.close()


def test_reconstruct_and_rotation():
    sp = lowrank_manifold_spec(dims=(14, 11, 9), ranks=(3, 3, 2), seed=2)
    _say("case reconstruct+rotation")
    snaps = [sp.snapshot_np(k) for k in range(4)]
    orc = O.OracleTDB(_ocfg(sp)).init(snaps[0])
    g = _cmp_cfg(sp, path="plain")
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, 4):
        orc.ingest(snaps[k])
        g.ingest(_dev(snaps[k]))
    out = g.reconstruct().cpu().numpy()
    assert _rel(out, orc.reconstruct()) < 1e-10
    r, Cr, Ur = g.get_core_and_bases(rotate=True)
    Co, Uo = O.core_rotation(orc.C, orc.U)
    assert _rel(Cr, Co) < 1e-8
    for n in range(3):
        assert _rel(Ur[n], Uo[n]) < 1e-8
    g.close()


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_controller_add_and_remove_decisions_match(path):
    """Closed-form switched stream: the add fires on the same step as in the oracle,
    ranks grow to (4,4,4), then the removal fires on the same step."""
    t_on, t_peak, t_low, h_min = 0.05, 0.15, 0.35, 0.002

    def h(t):
        if t <= t_on:
            return 0.0
        if t <= t_peak:
            return 2.0 * (t - t_on)
        if t <= t_low:
            return 0.2 + (h_min - 0.2) * (t - t_peak) / (t_low - t_peak)
        return h_min

    def gfun(t):
        return 0.004 * math.exp(-t)

    sp = switched_term_spec(steps=140, profile=h, profile2=gfun)
    _say(f"case controller switched-term 140 steps {path}")
    snaps = [sp.snapshot_np(k) for k in range(sp.steps + 1)]
    orc = O.OracleTDB(_ocfg(sp)).init(snaps[0])
    g = _cmp_cfg(sp, path=path)
    g.init(_dev(snaps[0]))
    assert g.ranks() == orc.ranks
    ev_o, ev_g = [], []
    for k in range(1, sp.steps + 1):
        rec = orc.ingest(snaps[k])
        g.ingest(_dev(snaps[k]))
        st = g.stats()
        if rec.event:
            ev_o.append((k, rec.event, rec.ranks))
        if st["event"]:
            ev_g.append((k, st["event"], st["ranks"]))
        assert st["eps"] == pytest.approx(rec.eps, rel=1e-6, abs=1e-12), k
    _say("  oracle events", ev_o, "gpu events", ev_g)
    assert ev_g == ev_o
    g.close()


@pytest.mark.parametrize("path,nx,ny,steps", [("plain", 128, 64, 30), ("fused", 128, 64, 30),
                                              ("fused", 512, 256, 20)])
def test_plume_fp32_against_oracle(path, nx, ny, steps):
    """Reactive-flow-shaped stream (same generator; 512 x 256 x 8 is the full size),
    FP32 data and FP32 bulk passes, adaptive from the rank rule: reconstruction and
    eps vs the FP64 oracle within the 1e-6 FP32 bar."""
    sp = plume_spec(nx=nx, ny=ny, nv=8, steps=steps)
    _say(f"case plume {nx}x{ny}x8 fp32 adaptive {steps} steps {path}")
    snaps = [sp.snapshot_np(k) for k in range(sp.steps + 1)]
    orc = O.OracleTDB(_ocfg(sp, rank_max=(32, 32, 8))).init(snaps[0].astype(np.float64))
    g = _cmp_cfg(sp, precision="f32", rank_max=(32, 32, 8), path=path)
    g.init(_dev(snaps[0]))
    assert g.ranks() == orc.ranks
    worst = 0.0
    for k in range(1, sp.steps + 1):
        rec = orc.ingest(snaps[k].astype(np.float64))
        g.ingest(_dev(snaps[k]))
        st = g.stats()
        assert st["event"] == rec.event, k
        rel_eps = abs(st["eps"] - rec.eps) / rec.nu
        worst = max(worst, rel_eps)
    r, C, U = g.get_core_and_bases()
    rec_g = O.reconstruct(C, U)
    rel = _rel(rec_g, orc.reconstruct())
    rels = _sigma_rel(g.stats()["sigma"], O.core_singular_values(orc.C))
    _say(f"  fp32 plume: reconstruction rel diff {rel:.3e}, worst eps diff / nu {worst:.3e}, "
         f"core singular values rel {rels:.3e}")
    assert rel < 1e-6 and worst < 1e-6 and rels < 1e-6
    g.close()


@pytest.mark.parametrize("path", ["plain", "fused"])
def test_ensemble_member_fp32_against_oracle(path):
    """One stream of the batched ensemble (uneven grid, 4 variables, exactly low rank
    <= 17 per spatial mode, caps 24, threshold 1e-5): FP32 path vs FP64 oracle."""
    sp = fourier_ensemble_specs(n_streams=3, steps=12)[2]
    _say(f"case ensemble member {sp.dims} fp32 {path}")
    snaps = [sp.snapshot_np(k) for k in range(sp.steps + 1)]
    orc = O.OracleTDB(_ocfg(sp)).init(snaps[0].astype(np.float64))
    g = _cmp_cfg(sp, precision="f32", path=path)
    g.init(_dev(snaps[0]))
    assert g.ranks() == orc.ranks
    for k in range(1, sp.steps + 1):
        rec = orc.ingest(snaps[k].astype(np.float64))
        g.ingest(_dev(snaps[k]))
        st = g.stats()
        assert st["event"] == rec.event, k
        assert abs(st["eps"] - rec.eps) <= 1e-6 * rec.nu, k
    r, C, U = g.get_core_and_bases()
    rel = _rel(O.reconstruct(C, U), orc.reconstruct())
    rels = _sigma_rel(g.stats()["sigma"], O.core_singular_values(orc.C))
    _say(f"  ensemble member: ranks {r}, reconstruction rel diff {rel:.3e}, core singular values rel {rels:.3e}")
    assert rel < 1e-6 and rels < 1e-6
    g.close()


@pytest.mark.parametrize("dims,caps", [((300, 40, 6), (40, 24, 6)), ((512, 32, 4), (64, 32, 4))])
def test_hosvd_init_large_mode_matches_oracle(dims, caps):
    """Device HOSVD with a long first mode (the multi-workgroup tridiagonal reduction,
    bisection and inverse iteration on a 300 x 300 and a 512 x 512 Gram) against the
    oracle's LAPACK eigendecomposition: projectors of the chosen ranks, core singular
    values and eps0."""
    _say(f"case hosvd-init large mode {dims}")
    rng = np.random.default_rng(11)
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    # a decaying spectrum in every mode
    base = np.zeros(dims)
    for q in range(30):
        a = [rng.normal(size=n) for n in dims]
        base += 0.7 ** q * np.einsum("i,j,k->ijk", *a)
    V0 = base + 1e-6 * rng.normal(size=dims)
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.01, rank_max=caps, rank_init=None, adaptive=True, eps_th=1e-3)
    orc = O.OracleTDB(cfg).init(V0)
    from paper_2201_06958_amd import Compressor
    g = Compressor(dims, 0.01, rank_max=caps, weights=w, data_dtype="f64", precision="f64", adaptive=True,
                   eps_th=1e-3)
    g.init(_dev(V0))
    r, C, U = g.get_core_and_bases()
    _say(f"  ranks gpu {r} oracle {orc.ranks}")
    assert r == orc.ranks
    for n in range(3):
        Pg = U[n] @ U[n].T * w[n][None, :]
        Po = orc.U[n] @ orc.U[n].T * w[n][None, :]
        assert np.abs(Pg - Po).max() < 1e-9, n
    assert _rel(O.reconstruct(C, U), O.reconstruct(orc.C, orc.U)) < 1e-9
    assert g.stats()["eps"] == pytest.approx(orc.records[0].eps, rel=1e-6)
    g.close()
