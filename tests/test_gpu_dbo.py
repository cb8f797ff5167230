"""GPU parity of order-2 streams on the row passes: the dynamically bi-orthonormal
form that the method reduces to for p = 2 (Sec. 2.2), used as TDB-2 in Sec. 3.2 with
the two spatial axes grouped into one tall mode. Against the FP64 oracle, through the
C ABI:

* fixed ranks from the oracle's factors, Heun and Euler, for short modes in each row
  bucket (8, 16, 32 entries) and tall modes on both sides of the eigensolver's size:
  core and bases per step at 1e-10 relative, eps at 1e-9 (FP64);
* second-order stage derivatives and given derivatives;
* FP32 data and passes: reconstruction at 1e-6, eps within 1e-6 of nu;
* the HOSVD initialisation, whose tall-mode basis comes from the short mode's
  eigenvectors (U1 = V W2 U2 Sigma^-1, sign-fixed): ranks, core and bases at 1e-10;
* an adaptive run whose fourth term rises and decays: the oracle's add and removal at
  the oracle's steps, eps per step at 1e-8."""
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O

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


def _weights(M, K, seed):
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(0.5, 1.5, M)
    w2 = rng.uniform(0.5, 1.5, K)
    return [w1 / w1.sum(), w2 / w2.sum()]


def _walk(M, K, seed, n=7, amp=0.01, rank=4):
    """A base of the run's rank (amplitudes 1 down to 0.3, so that the core is well
    conditioned) plus a small random walk: every step moves the subspaces."""
    rng = np.random.default_rng(seed)
    base = (rng.normal(size=(M, rank)) * np.linspace(1.0, 0.3, rank)) @ rng.normal(size=(rank, K))
    snaps = [base]
    for _ in range(1, n):
        snaps.append(snaps[-1] + amp * rng.normal(size=(M, K)))
    return snaps


def _bump_stream(M, K, seed=3):
    """Three rotating terms and a fourth whose amplitude is a bump around t = 0.3."""
    rng = np.random.default_rng(seed)
    A, B = rng.normal(size=(M, 4)), rng.normal(size=(K, 4))
    Ra, Rb = 0.3 * rng.normal(size=(M, 4)), 0.3 * rng.normal(size=(K, 4))
    amps = np.array([1.0, 0.6, 0.35])

    def V(t):
        a = np.concatenate([amps * (1 + 0.2 * np.sin(3 * t + np.arange(3))), [0.25 * np.exp(-((t - 0.3) / 0.08) ** 2)]])
        return ((A + t * Ra) * a) @ (B + t * Rb).T
    return V


def _compressor(dims, ranks, w, prec="f64", **kw):
    from paper_2201_06958_amd import Compressor
    return Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype=prec, precision=prec,
                      adaptive=False, eps_th=1.0, **kw)


@pytest.mark.parametrize("integrator", ["heun", "euler"])
@pytest.mark.parametrize("M,K,r", [(300, 8, 3), (960, 8, 5), (700, 12, 4), (1500, 24, 6), (520, 32, 32)])
def test_dbo_fixed_rank_fp64_matches_oracle(M, K, r, integrator):
    _say(f"case dbo fp64 M {M} K {K} r {r} {integrator}")
    w = _weights(M, K, M + K)
    snaps = _walk(M, K, M + 7 * K, rank=r)
    cfg = O.OracleConfig(dims=(M, K), weights=w, dt=0.05, rank_max=(r, r), rank_init=(r, r), adaptive=False,
                         eps_th=1.0, integrator=integrator)
    orc = O.OracleTDB(cfg).init(snaps[0])
    g = _compressor((M, K), (r, r), w, integrator=integrator)
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k])
        g.ingest(_dev(snaps[k]))
        _, C, U = g.get_core_and_bases()
        assert _rel(C, orc.C) < 1e-10, k
        assert _rel(U[0], orc.U[0]) < 1e-10, k
        assert _rel(U[1], orc.U[1]) < 1e-10, k
        st = g.stats()
        assert st["eps"] == pytest.approx(rec.eps, rel=1e-9), k
        assert st["path_used"] == "fused"
    g.close()


@pytest.mark.parametrize("mode", ["fd2", "derivative"])
def test_dbo_stage_derivatives_match_oracle(mode):
    """Second-order stage derivatives (three snapshots resident) and a given
    derivative held over both stages."""
    _say(f"case dbo {mode}")
    M, K, r = 900, 10, 4
    w = _weights(M, K, 5)
    snaps = _walk(M, K, 6)
    ders = [0.1 * np.random.default_rng(k).normal(size=(M, K)) for k in range(len(snaps))]
    cfg = O.OracleConfig(dims=(M, K), weights=w, dt=0.05, rank_max=(r, r), rank_init=(r, r), adaptive=False,
                         eps_th=1.0, fd_order=2 if mode == "fd2" else 1)
    orc = O.OracleTDB(cfg).init(snaps[0])
    g = _compressor((M, K), (r, r), w, fd_order=2 if mode == "fd2" else 1)
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, len(snaps)):
        if mode == "fd2":
            rec = orc.ingest(snaps[k])
            g.ingest(_dev(snaps[k]))
        else:
            rec = orc.ingest(snaps[k], D=ders[k])
            g.ingest_with_derivative(_dev(snaps[k]), _dev(ders[k]))
        _, C, U = g.get_core_and_bases()
        assert _rel(C, orc.C) < 1e-10, k
        assert _rel(U[0], orc.U[0]) < 1e-10 and _rel(U[1], orc.U[1]) < 1e-10, k
        assert g.stats()["eps"] == pytest.approx(rec.eps, rel=1e-9), k
    g.close()


def test_dbo_fp32_matches_oracle():
    _say("case dbo fp32")
    M, K, r = 4096, 8, 5
    w = _weights(M, K, 9)
    snaps = [s.astype(np.float32) for s in _walk(M, K, 10, n=9, rank=r)]
    cfg = O.OracleConfig(dims=(M, K), weights=w, dt=0.05, rank_max=(r, r), rank_init=(r, r), adaptive=False,
                         eps_th=1.0)
    orc = O.OracleTDB(cfg).init(snaps[0].astype(np.float64))
    g = _compressor((M, K), (r, r), w, prec="f32")
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k].astype(np.float64))
        g.ingest(_dev(snaps[k]))
        _, C, U = g.get_core_and_bases()
        assert _rel(O.reconstruct(C, U), orc.reconstruct()) < 1e-6, k
        assert _rel(C, orc.C) < 1e-6, k
        assert abs(g.stats()["eps"] - rec.eps) <= 1e-6 * rec.nu, k
    g.close()


@pytest.mark.parametrize("M,K", [(400, 8), (1200, 8), (2000, 20)])
def test_dbo_hosvd_init_matches_oracle(M, K):
    """Rank chosen by the rule at init (eps_th), then core, bases and eps0; for M above
    the eigensolver's size the tall basis comes from the short mode's eigenvectors."""
    _say(f"case dbo hosvd M {M} K {K}")
    from paper_2201_06958_amd import Compressor
    w = _weights(M, K, 21)
    V0 = _walk(M, K, 22, n=1)[0] + 0.003 * np.random.default_rng(23).normal(size=(M, K))
    cfg = O.OracleConfig(dims=(M, K), weights=w, dt=0.05, rank_max=(8, 8), adaptive=True, eps_th=5e-2)
    orc = O.OracleTDB(cfg).init(V0)
    g = Compressor((M, K), 0.05, rank_max=(8, 8), weights=w, data_dtype="f64", precision="f64", eps_th=5e-2)
    g.init(_dev(V0))
    r, C, U = g.get_core_and_bases()
    assert tuple(r[:2]) == tuple(orc.C.shape)
    assert _rel(C, orc.C) < 1e-10
    assert _rel(U[0], orc.U[0]) < 1e-10 and _rel(U[1], orc.U[1]) < 1e-10
    assert g.stats()["eps"] == pytest.approx(O.error_and_norm(V0, orc.C, orc.U, w)[0], rel=1e-8)
    g.close()


@pytest.mark.parametrize("M,K", [(600, 8), (1200, 12)])
def test_dbo_adaptive_events_match_oracle(M, K):
    """Adaptive from the HOSVD: the fourth term's bump makes the oracle add a rank and
    remove it again; the device takes the same events at the same steps."""
    _say(f"case dbo adaptive M {M} K {K}")
    from paper_2201_06958_amd import Compressor
    V = _bump_stream(M, K)
    w = _weights(M, K, 1)
    cfg = O.OracleConfig(dims=(M, K), weights=w, dt=0.01, rank_max=(8, 8), adaptive=True, eps_th=5e-3)
    orc = O.OracleTDB(cfg).init(V(0.0))
    g = Compressor((M, K), 0.01, rank_max=(8, 8), weights=w, data_dtype="f64", precision="f64", eps_th=5e-3)
    g.init(_dev(V(0.0)))
    ev_o, ev_d = [], []
    for k in range(1, 81):
        x = V(k * 0.01)
        rec = orc.ingest(x)
        g.ingest(_dev(x))
        st = g.stats()
        if rec.event:
            ev_o.append((k, rec.event, tuple(rec.ranks)))
        if st["event"]:
            ev_d.append((k, st["event"], tuple(st["ranks"][:2])))
        assert ev_d == ev_o, (k, ev_d, ev_o)
        assert st["eps"] == pytest.approx(rec.eps, rel=1e-8), k
    _say(f"  events {ev_o}")
    assert [e[1] for e in ev_o] == ["add", "remove"]
    g.close()
