"""GPU parity of the time-scheme options (Sec. 3.1): the explicit Euler integrator
against the FP64 oracle's Euler step, and steps with a given data derivative
(tdb_ingest_with_derivative) against the oracle fed the same derivative, raw state per
step at 1e-10 relative (FP64) on both paths, 1e-6 on the reconstruction for FP32; and
the scheme study on an exactly low-rank stream, where the error is pure
time-integration error: the observed order of the device's Heun step is two, of its
Euler step one, with the difference quotient and with the exact derivative."""
import math
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import lowrank_manifold_spec

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


@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("dims,ranks", [((20, 17, 9), (3, 4, 2)), ((9, 7, 6, 5), (2, 3, 2, 2)),
                                        ((70, 130, 5), (6, 5, 4))])
def test_euler_fp64_matches_oracle(dims, ranks, path):
    """Random weights, random snapshots around a low-rank base, fixed ranks, started
    from the oracle's factors: core, bases and eps after every Euler step."""
    _say(f"case euler fp64 dims {dims} ranks {ranks} {path}")
    rng = np.random.default_rng(sum(dims) + 11)
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = rng.normal(size=dims)
    snaps = [base + 0.005 * k * rng.normal(size=dims) for k in range(7)]
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks,
                         adaptive=False, eps_th=1.0, integrator="euler")
    orc = O.OracleTDB(cfg).init(snaps[0])
    from paper_2201_06958_amd import Compressor
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f64",
                   precision="f64", adaptive=False, path=path, eps_th=1.0, integrator="euler")
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    heun = O.OracleTDB(O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks,
                                      adaptive=False, eps_th=1.0)).init(snaps[0])
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k])
        heun.ingest(snaps[k])
        g.ingest(_dev(snaps[k]))
        r, C, U = g.get_core_and_bases()
        assert _rel(C, orc.C) < 1e-10, k
        for n in range(len(dims)):
            assert _rel(U[n], orc.U[n]) < 1e-10, (k, n)
        assert g.stats()["eps"] == pytest.approx(rec.eps, rel=1e-9)
    # the two schemes really differ on this stream (the flag is not ignored)
    assert _rel(O.reconstruct(orc.C, orc.U), O.reconstruct(heun.C, heun.U)) > 1e-8
    g.close()


def _device_error(sp, T, dt, integrator, path, fd_order=1):
    from paper_2201_06958_amd import Compressor
    sp.dt = dt
    steps = int(round(T / dt))
    g = Compressor(sp.dims, dt, rank_max=sp.rank_max, rank_init=sp.rank_init, weights=sp.weights,
                   data_dtype="f64", precision="f64", adaptive=False, path=path, eps_th=1.0,
                   integrator=integrator, fd_order=fd_order)
    g.init(_dev(sp.snapshot_np(0)))
    for k in range(1, steps + 1):
        g.ingest(_dev(sp.snapshot_np(k)))
    st = g.stats()
    g.close()
    return st["eps"] / st["nu"]


@pytest.mark.parametrize("path", ["plain", "fused"])
@pytest.mark.parametrize("integrator,order,fd", [("heun", 2.0, 1), ("euler", 1.0, 1), ("heun", 2.0, 2)])
def test_scheme_order_on_exactly_low_rank_stream(integrator, order, fd, path):
    """Halving the step twice: the observed order of the final error is that of the
    scheme (the stream stays exactly on the rank-(3,3,2) manifold, so only the time
    integration contributes), with the first- and second-order differences."""
    _say(f"case scheme order {integrator} fd{fd} {path}")
    sp = lowrank_manifold_spec(dims=(12, 10, 8), ranks=(3, 3, 2), seed=0, rot=0.8)
    T = 0.4
    e = [_device_error(sp, T, dt, integrator, path, fd) for dt in (0.02, 0.01, 0.005)]
    o2 = math.log2(e[1] / e[2])
    _say(f"  errors {e}, observed order {o2:.3f}")
    assert abs(o2 - order) < 0.2, (e, o2)


@pytest.mark.parametrize("integrator", ["heun", "euler"])
@pytest.mark.parametrize("path,precision", [("plain", "f64"), ("fused", "f64"), ("fused", "f32")])
def test_derivative_ingest_matches_oracle(path, precision, integrator):
    """Steps with a given data derivative (here an arbitrary random field, so that the
    projections see nothing of the snapshots' difference): raw state per step at 1e-10
    (FP64), reconstruction at 1e-6 (FP32 data and passes), eps as the oracle's."""
    _say(f"case derivative ingest {path} {precision} {integrator}")
    dims, ranks = (20, 17, 9), (3, 4, 2)
    rng = np.random.default_rng(29)
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = rng.normal(size=dims)
    st = np.float64 if precision == "f64" else np.float32
    snaps = [(base + 0.005 * k * rng.normal(size=dims)).astype(st) for k in range(6)]
    ders = [(0.1 * rng.normal(size=dims)).astype(st) for k in range(6)]
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks,
                         adaptive=False, eps_th=1.0, integrator=integrator)
    orc = O.OracleTDB(cfg).init(snaps[0].astype(np.float64))
    from paper_2201_06958_amd import Compressor
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype=precision,
                   precision=precision, adaptive=False, path=path, eps_th=1.0, integrator=integrator)
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k].astype(np.float64), D=ders[k].astype(np.float64))
        g.ingest_with_derivative(_dev(snaps[k]), _dev(ders[k]))
        r, C, U = g.get_core_and_bases()
        if precision == "f64":
            assert _rel(C, orc.C) < 1e-10, k
            for n in range(len(dims)):
                assert _rel(U[n], orc.U[n]) < 1e-10, (k, n)
            assert g.stats()["eps"] == pytest.approx(rec.eps, rel=1e-9)
        else:
            assert _rel(O.reconstruct(C, U), orc.reconstruct()) < 1e-6, k
            assert abs(g.stats()["eps"] - rec.eps) <= 1e-6 * rec.nu, k
    g.close()


def _device_error_exact(sp, T, dt, integrator):
    from paper_2201_06958_amd import Compressor
    sp.dt = dt
    steps = int(round(T / dt))
    g = Compressor(sp.dims, dt, rank_max=sp.rank_max, rank_init=sp.rank_init, weights=sp.weights,
                   data_dtype="f64", precision="f64", adaptive=False, path="fused", eps_th=1.0,
                   integrator=integrator)
    g.init(_dev(sp.snapshot_np(0)))
    for k in range(1, steps + 1):
        # the exact derivative at the step's midpoint, held over the step's stages
        D = sp.deriv_fn(sp.time(k - 1) + 0.5 * dt, "cpu", torch.float64).numpy()
        g.ingest_with_derivative(_dev(sp.snapshot_np(k)), _dev(D))
    st = g.stats()
    g.close()
    return st["eps"] / st["nu"]


@pytest.mark.parametrize("integrator,order", [("heun", 2.0), ("euler", 1.0)])
def test_scheme_order_with_exact_derivative(integrator, order):
    """The time-scheme comparison with the exact data derivative on an exactly
    low-rank stream: Heun second order, Euler first, Heun's error the smaller."""
    _say(f"case exact-derivative order {integrator}")
    sp = lowrank_manifold_spec(dims=(12, 10, 8), ranks=(3, 3, 2), seed=0, rot=0.8)
    T = 0.4
    e = [_device_error_exact(sp, T, dt, integrator) for dt in (0.02, 0.01, 0.005)]
    o2 = math.log2(e[1] / e[2])
    _say(f"  errors {e}, observed order {o2:.3f}")
    assert abs(o2 - order) < 0.2, (e, o2)


@pytest.mark.parametrize("path,precision,mode,integrator", [
    ("plain", "f64", "copy", "heun"), ("fused", "f64", "copy", "heun"), ("fused", "f64", "borrow", "heun"),
    ("plain", "f64", "borrow", "euler"), ("fused", "f32", "copy", "heun")])
def test_fd2_matches_oracle(path, precision, mode, integrator):
    """Second-order stage derivatives (fd_order 2: central difference at t_k, one-sided
    second-order difference at t_{k+1}; first-order quotient on the first step) on a
    random walk around a low-rank base, fixed ranks from the oracle's factors: raw
    state per step at 1e-10 relative (FP64), reconstruction at 1e-6 (FP32), eps as the
    oracle's; the first-order run differs (the option is not ignored)."""
    _say(f"case fd2 {path} {precision} {mode} {integrator}")
    dims, ranks = (20, 17, 9), (3, 4, 2)
    rng = np.random.default_rng(41)
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = rng.normal(size=dims)
    st = np.float64 if precision == "f64" else np.float32
    snaps = [base]
    for k in range(1, 8):
        snaps.append(snaps[-1] + 0.01 * rng.normal(size=dims))
    snaps = [s.astype(st) for s in snaps]
    mk = lambda fd: O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks, adaptive=False,
                                   eps_th=1.0, integrator=integrator, fd_order=fd)
    orc = O.OracleTDB(mk(2)).init(snaps[0].astype(np.float64))
    first = O.OracleTDB(mk(1)).init(snaps[0].astype(np.float64))
    from paper_2201_06958_amd import Compressor
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype=precision,
                   precision=precision, adaptive=False, path=path, eps_th=1.0, integrator=integrator,
                   snapshot_mode=mode, fd_order=2)
    held = [_dev(snaps[0])]   # borrowed snapshots stay alive
    g.init_from_factors(held[0], orc.C, orc.U)
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k].astype(np.float64))
        first.ingest(snaps[k].astype(np.float64))
        held.append(_dev(snaps[k]))
        g.ingest(held[-1])
        r, C, U = g.get_core_and_bases()
        if precision == "f64":
            assert _rel(C, orc.C) < 1e-10, k
            for n in range(len(dims)):
                assert _rel(U[n], orc.U[n]) < 1e-10, (k, n)
            assert g.stats()["eps"] == pytest.approx(rec.eps, rel=1e-9)
        else:
            assert _rel(O.reconstruct(C, U), orc.reconstruct()) < 1e-6, k
            assert abs(g.stats()["eps"] - rec.eps) <= 1e-6 * rec.nu, k
        assert g.stats()["path_used"] == path
    assert _rel(orc.reconstruct(), first.reconstruct()) > 1e-7
    g.close()


def test_fd2_batches_refuse():
    """Batches take the first-order difference quotient only."""
    _say("case fd2 batch refused")
    from paper_2201_06958_amd import tdb
    dims = (16, 12, 4)
    V = _dev(np.random.default_rng(0).normal(size=dims))
    with pytest.raises(tdb.TDBError) as ei:
        tdb.Batch([dict(dims=dims, dt=0.1, rank_max=(2, 2, 2), fd_order=2)]).init([V])
    assert "first-order" in str(ei.value)


@pytest.mark.parametrize("fd", [1, 2])
def test_runge_adaptive_matches_oracle(fd):
    """The calibrated Runge study (Sec. 3.1) on a 32^3 grid, 400 steps from the rank-3
    truncated HOSVD, adaptive with eps_th 2.5e-3 and the 99.99 % budget, FP64 on the
    fused path: the device takes the oracle's events at the oracle's steps, its eps
    follows the oracle's at 1e-8 relative, and the rank rises while a(t) dips and
    returns to (3, 3, 3). The field is symmetric in its three axes, so the modes'
    singular values tie and which mode an addition grows is decided by rounding: the
    sorted ranks are compared, not the mode."""
    _say(f"case runge adaptive fd{fd}")
    from streams import runge_spec
    from paper_2201_06958_amd import Compressor
    sp = runge_spec(n=32, steps=400)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(8, 8, 8), rank_init=(3, 3, 3),
                         adaptive=True, eps_th=2.5e-3, gamma_th=99.99, fd_order=fd)
    V0 = sp.snapshot_np(0).astype(np.float64)
    C0, U0 = O.hosvd(V0, sp.weights, cfg.caps()).truncate((3, 3, 3))
    orc = O.OracleTDB(cfg).init_from_factors(V0, C0, U0)
    g = Compressor(sp.dims, sp.dt, rank_max=(8, 8, 8), rank_init=(3, 3, 3), weights=sp.weights, data_dtype="f64",
                   precision="f64", path="fused", adaptive=True, eps_th=2.5e-3, gamma_th=99.99, fd_order=fd)
    g.init_from_factors(_dev(V0), C0, U0)
    ev_o, ev_d, rmax = [], [], 0
    for k in range(1, sp.steps + 1):
        V = sp.snapshot_np(k).astype(np.float64)
        rec = orc.ingest(V)
        g.ingest(_dev(V))
        st = g.stats()
        if rec.event:
            ev_o.append((k, rec.event, tuple(sorted(rec.ranks))))
        if st["event"]:
            ev_d.append((k, st["event"], tuple(sorted(st["ranks"][:3]))))
        assert ev_d == ev_o, (k, ev_d, ev_o)
        assert st["eps"] == pytest.approx(rec.eps, rel=1e-8), k
        rmax = max(rmax, max(rec.ranks))
    _say(f"  events {ev_o}, final ranks {tuple(orc.records[-1].ranks)}, crbar {g.stats()['crbar']:.1f}")
    assert rmax >= 4 and tuple(orc.records[-1].ranks) == (3, 3, 3)
    g.close()
