"""GPU checks of the numerical contract and of the controller's inputs through the C
ABI, against the FP64 oracle:

* non-finite data (NaN or Inf in a snapshot) returns TDB_ENUMERIC and leaves the core,
  bases, ranks and statistics unchanged, on the fused path (synchronous and pipelined),
  the plain path, a batch and the given-derivative step; the stream then resumes as
  the oracle does from the same previous snapshot;
* a rank-deficient core given to init_from_factors makes the first step's
  pseudo-inverse singular (Sec. 2.2): the numerical event restarts from a HOSVD at
  the oracle's ranks;
* the paper-style budget gamma_th (eq. (percentage)) and set_threshold (Sec. 2.5)
  give the oracle's events and ranks;
* the orthonormality invariant U_n^T W_n U_n = I (Sec. 2.2) holds below 1e-12 after
  many steps, in FP64 and in the FP32 forms.
"""
import math
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import analytic_cp5_spec, plume_spec, switched_term_spec

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


def _small_stream(seed=5, dims=(24, 20, 6), steps=8):
    rng = np.random.default_rng(seed)
    w = []
    for n in dims:
        x = rng.uniform(0.5, 1.5, size=n)
        w.append(x / x.sum())
    base = rng.normal(size=dims)
    snaps = [base + 0.01 * k * rng.normal(size=dims) for k in range(steps)]
    return dims, w, snaps


def _state(g):
    r, C, U = g.get_core_and_bases()
    return r, C.copy(), [u.copy() for u in U]


@pytest.mark.parametrize("mode", ["fused-copy", "fused-borrow", "plain-copy"])
@pytest.mark.parametrize("bad", ["nan", "inf"])
def test_nonfinite_snapshot_is_not_applied(mode, bad):
    """A NaN (or Inf) in one snapshot: TDB_ENUMERIC, state and statistics unchanged;
    the next step's difference quotient is non-finite too and is not applied; the
    stream then resumes from the snapshot after, exactly as the oracle does when its
    previous snapshot is that one (FP64 parity 1e-10)."""
    from paper_2201_06958_amd import Compressor
    from paper_2201_06958_amd.tdb import ENUMERIC, TDBError
    path, smode = mode.split("-")
    _say(f"case nonfinite {mode} {bad}")
    dims, w, snaps = _small_stream()
    ranks = (4, 4, 3)
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks, adaptive=False, eps_th=1.0)
    orc = O.OracleTDB(cfg).init(snaps[0])
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f64", precision="f64",
                   adaptive=False, path=path, eps_th=1.0, snapshot_mode="borrow" if smode == "borrow" else "copy")
    dev = [_dev(s) for s in snaps]
    g.init_from_factors(dev[0], orc.C, orc.U)
    for k in (1, 2, 3):
        orc.ingest(snaps[k])
        g.ingest(dev[k])
    r0, C0, U0 = _state(g)
    st0 = g.stats()
    badv = snaps[4].copy()
    badv[3, 5, 1] = np.nan if bad == "nan" else np.inf
    bad_dev = _dev(badv)

    def expect_enumeric(fn):
        with pytest.raises(TDBError) as ei:
            fn()
        assert ei.value.status == ENUMERIC

    if smode == "borrow":
        g.ingest(bad_dev)                       # pipelined: reported by the next call
        expect_enumeric(g.flush)
    else:
        expect_enumeric(lambda: g.ingest(bad_dev))
    r1, C1, U1 = _state(g)
    st1 = g.stats()
    assert r1 == r0 and np.array_equal(C1, C0) and all(np.array_equal(a, b) for a, b in zip(U1, U0))
    assert st1["step"] == st0["step"] and st1["eps"] == st0["eps"]
    assert st1["n_nonfinite"] == 1
    # the following step differences against the non-finite snapshot: also not applied
    if smode == "borrow":
        g.ingest(dev[5])
        expect_enumeric(g.flush)
    else:
        expect_enumeric(lambda: g.ingest(dev[5]))
    r2, C2, _ = _state(g)
    assert np.array_equal(C2, C0) and g.stats()["n_nonfinite"] == 2
    # then the stream goes on from snapshot 5
    orc.V_prev = snaps[5].copy()
    rec = orc.ingest(snaps[6])
    g.ingest(dev[6])
    if smode == "borrow":
        g.flush()
    st = g.stats()
    assert st["step"] == st0["step"] + 1
    assert abs(st["eps"] - rec.eps) <= 1e-10 * rec.nu
    r, C, U = g.get_core_and_bases()
    assert _rel(O.reconstruct(C, U), orc.reconstruct()) < 1e-10
    g.close()


def test_nonfinite_in_batch_member():
    """One batch member gets a NaN snapshot: the batch step returns TDB_ENUMERIC, that
    member keeps its state, the other members advance as the oracle does."""
    from paper_2201_06958_amd import Batch
    from paper_2201_06958_amd.tdb import ENUMERIC, TDBError
    _say("case nonfinite batch")
    streams = [_small_stream(seed=s, dims=d) for s, d in ((1, (24, 20, 6)), (2, (32, 18, 4)))]
    ranks = (4, 4, 3)
    cfgs, orcs = [], []
    for dims, w, snaps in streams:
        cfgs.append(dict(dims=dims, dt=0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f64",
                         precision="f64", adaptive=False, eps_th=1.0))
        orcs.append(O.OracleTDB(O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks,
                                               adaptive=False, eps_th=1.0)).init(snaps[0]))
    b = Batch(cfgs).init([_dev(s[2][0]) for s in streams])
    for k in (1, 2):
        b.ingest([_dev(s[2][k]) for s in streams])
        for o, s in zip(orcs, streams):
            o.ingest(s[2][k])
    _, C0, _ = _state(b.streams[1])
    bad = streams[1][2][3].copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(TDBError) as ei:
        b.ingest([_dev(streams[0][2][3]), _dev(bad)])
    assert ei.value.status == ENUMERIC
    rec = orcs[0].ingest(streams[0][2][3])
    st = b.streams[0].stats()
    assert abs(st["eps"] - rec.eps) <= 1e-10 * rec.nu
    r, C, U = b.streams[0].get_core_and_bases()
    assert _rel(O.reconstruct(C, U), orcs[0].reconstruct()) < 1e-10
    _, C1, _ = _state(b.streams[1])
    assert np.array_equal(C1, C0)
    assert b.streams[1].stats()["n_nonfinite"] == 1
    b.close()


def test_nonfinite_first_snapshot_and_derivative():
    from paper_2201_06958_amd import Compressor
    from paper_2201_06958_amd.tdb import ENUMERIC, TDBError
    _say("case nonfinite init and derivative")
    dims, w, snaps = _small_stream()
    bad = snaps[0].copy()
    bad[1, 1, 1] = np.nan
    g = Compressor(dims, 0.05, rank_max=(4, 4, 3), rank_init=(4, 4, 3), weights=w, data_dtype="f64",
                   precision="f64", adaptive=False, eps_th=1.0)
    with pytest.raises(TDBError) as ei:
        g.init(_dev(bad))
    assert ei.value.status == ENUMERIC
    g = Compressor(dims, 0.05, rank_max=(4, 4, 3), rank_init=(4, 4, 3), weights=w, data_dtype="f64",
                   precision="f64", adaptive=False, eps_th=1.0)
    g.init(_dev(snaps[0]))
    g.ingest(_dev(snaps[1]))
    _, C0, _ = _state(g)
    D = (snaps[2] - snaps[1]) / 0.05
    for v, d in ((bad, D), (snaps[2], np.where(np.arange(D.size).reshape(D.shape) == 7, np.inf, D))):
        with pytest.raises(TDBError) as ei:
            g.ingest_with_derivative(_dev(v), _dev(d))
        assert ei.value.status == ENUMERIC
        _, C1, _ = _state(g)
        assert np.array_equal(C1, C0)
    g.close()


@pytest.mark.parametrize("path", ["fused", "plain"])
def test_rank_deficient_core_restarts_numerically(path):
    """Factors whose core has a zero mode-1 slice: the first step's core Gram is
    singular, the numerical event restarts from a HOSVD of that step's snapshot; the
    oracle (given the same factors) takes the same event and ranks."""
    from paper_2201_06958_amd import Compressor
    _say(f"case rank-deficient core {path}")
    sp = analytic_cp5_spec(n=24, steps=4)
    ranks = (5, 5, 5)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=ranks, rank_init=ranks,
                         adaptive=True, eps_th=1e-3)
    V0 = sp.snapshot_np(0)
    h = O.hosvd(V0, sp.weights, ranks)
    C, U = h.truncate(ranks)
    C = C.copy()
    C[4, :, :] = 0.0                      # mode-1 unfolding loses rank
    orc = O.OracleTDB(cfg).init_from_factors(V0, C, U)
    g = Compressor(sp.dims, sp.dt, rank_max=ranks, rank_init=ranks, weights=sp.weights, data_dtype="f64",
                   precision="f64", adaptive=True, eps_th=1e-3, path=path)
    g.init_from_factors(_dev(V0), C, U)
    V1 = sp.snapshot_np(1)
    rec = orc.ingest(V1)
    g.ingest(_dev(V1))
    st = g.stats()
    assert rec.event == "numeric" and st["event"] == "numeric"
    assert st["ranks"] == rec.ranks
    assert st["n_numeric"] == 1
    # eps_after^2 = nu^2 - ||C||^2: compared squared (its square root magnifies the
    # cancellation of about 1e-16 nu^2 when the restart is nearly exact)
    assert abs(st["eps_after"] ** 2 - rec.eps_after ** 2) <= 1e-13 * rec.nu ** 2
    for k in (2, 3):
        rec = orc.ingest(sp.snapshot_np(k))
        g.ingest(_dev(sp.snapshot_np(k)))
        assert abs(g.stats()["eps"] - rec.eps) <= 1e-9 * rec.nu
    g.close()


@pytest.mark.parametrize("path", ["fused", "plain"])
@pytest.mark.parametrize("side", ["below", "above"])
def test_gamma_budget_on_device(path, side):
    """Paper-style budget (1 - gamma_th/100) ||V||^2 on the switched stream: the ranks
    grow at the add only when the extra term's closed-form energy exceeds it."""
    from paper_2201_06958_amd import Compressor
    _say(f"case gamma_th {path} {side}")
    sp = switched_term_spec()
    m = sp.meta
    k_fire = next(k for k in range(1, sp.steps + 1) if m["h"](sp.time(k)) * m["qnorm"] > sp.eps_th)
    hq = m["h"](sp.time(k_fire)) * m["qnorm"]
    V = sp.snapshot_np(k_fire)
    nu2 = float(np.sum(O.weight_tensor(sp.weights) * V * V))
    B = 2.0 * hq * hq if side == "below" else 0.5 * hq * hq
    gamma = 100.0 * (1.0 - B / nu2)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th, gamma_th=gamma)
    V0 = sp.snapshot_np(0)
    orc = O.OracleTDB(cfg).init(V0)
    g = Compressor(sp.dims, sp.dt, rank_max=sp.rank_max, rank_init=sp.rank_init, weights=sp.weights,
                   data_dtype="f64", precision="f64", adaptive=True, eps_th=sp.eps_th, gamma_th=gamma, path=path)
    g.init(_dev(V0))
    # up to the step after the add: two steps later the error (linear in t) equals
    # twice the reinit error exactly, the raised trigger of the "below" case, a tie
    for k in range(1, k_fire + 2):
        rec = orc.ingest(sp.snapshot_np(k))
        g.ingest(_dev(sp.snapshot_np(k)))
        st = g.stats()
        assert st["event"] == rec.event, k
        assert st["ranks"] == rec.ranks, k
        if rec.event:
            assert abs(st["eps_after"] ** 2 - rec.eps_after ** 2) <= 1e-13 * rec.nu ** 2
    want = (3, 3, 3) if side == "below" else (4, 4, 4)
    assert g.stats()["ranks"] == want
    g.close()


@pytest.mark.parametrize("snapshot_mode", ["copy", "borrow"])
def test_set_threshold_moves_the_add_on_device(snapshot_mode):
    from paper_2201_06958_amd import Compressor
    _say(f"case set_threshold {snapshot_mode}")
    sp = switched_term_spec(steps=80)
    m = sp.meta
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th)
    V0 = sp.snapshot_np(0)
    orc = O.OracleTDB(cfg).init(V0)
    g = Compressor(sp.dims, sp.dt, rank_max=sp.rank_max, rank_init=sp.rank_init, weights=sp.weights,
                   data_dtype="f64", precision="f64", adaptive=True, eps_th=sp.eps_th, snapshot_mode=snapshot_mode)
    g.init(_dev(V0))
    dev = [_dev(sp.snapshot_np(k)) for k in range(sp.steps + 1)]
    new_th = 5.0 * sp.eps_th
    fired_o = fired_g = None
    for k in range(1, sp.steps + 1):
        if k == 11:
            orc.set_threshold(new_th)
            g.set_threshold(new_th)
        rec = orc.ingest(sp.snapshot_np(k))
        g.ingest(dev[k])
        st = g.stats()
        if rec.event and fired_o is None:
            fired_o = k
        if st["event"] and fired_g is None:
            fired_g = k
        assert st["event"] == rec.event, k
    expected = next(k for k in range(11, sp.steps + 1) if m["h"](sp.time(k)) * m["qnorm"] > new_th)
    assert fired_o == expected and fired_g == expected
    g.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16s"])
def test_orthonormality_invariant_over_steps(precision):
    """||U_n^T W_n U_n - I||_max < 1e-12 after every one of 40 steps (the bases stay
    FP64 in every precision form, re-orthonormalised after each step)."""
    from paper_2201_06958_amd import Compressor
    _say(f"case orthonormality {precision}")
    if precision == "f64":
        sp = analytic_cp5_spec(n=32, steps=40)
        store = "f64"
        rmax, rinit, adaptive = (5, 5, 5), (5, 5, 5), False
    else:
        sp = plume_spec(nx=128, ny=64, nv=8, steps=40)
        store = "f32"
        rmax, rinit, adaptive = (32, 32, 8), None, True
    g = Compressor(sp.dims, sp.dt, rank_max=rmax, rank_init=rinit, weights=sp.weights, data_dtype=store,
                   precision=precision, adaptive=adaptive, eps_th=sp.eps_th if sp.eps_th > 0 else 1.0)
    g.init(_dev(sp.snapshot_np(0)))
    worst = 0.0
    for k in range(1, 41):
        g.ingest(_dev(sp.snapshot_np(k)))
        if k % 5 == 0:
            r, C, U = g.get_core_and_bases()
            for n in range(3):
                G = (U[n].T * sp.weights[n][None, :]) @ U[n]
                worst = max(worst, float(np.abs(G - np.eye(r[n])).max()))
    _say(f"  max |U^T W U - I| = {worst:.2e}")
    assert worst < 1e-12
    g.close()
