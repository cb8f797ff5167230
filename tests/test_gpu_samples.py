"""GPU parity of samples as a tensor mode (the stochastic case of Sec. 3.3, eq. (UQ)):
an ensemble of samples stacked along a leading mode whose weights are the
probabilistic-collocation (product Gauss) weights, compressed as one order-4 tensor.
Against the FP64 oracle, through the C ABI:

* a random walk around a well-conditioned Tucker tensor of that shape (six samples of
  a 2 x 3 collocation grid, so the sample weights are not uniform): core and bases per
  step at 1e-10 relative, eps at 1e-9 (FP64);
* the stochastic reactive-flow samples themselves (FP32 data and passes): the
  reconstruction at 1e-6 relative and eps within 1e-6 of nu per step (their cores are
  ill-conditioned by nature, so the factors themselves are not compared)."""
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


def _pcm_weights(s1, s2):
    _, q1 = np.polynomial.legendre.leggauss(s1)
    _, q2 = np.polynomial.legendre.leggauss(s2)
    w = np.kron(q1, q2)
    return w / w.sum()


def _tucker_walk(dims, ranks, seed, n=7, amp=0.01):
    """A Tucker tensor with a diagonally dominant core (every unfolding well
    conditioned) plus a small random walk."""
    rng = np.random.default_rng(seed)
    C = 0.2 * rng.normal(size=ranks)
    for i in range(min(ranks)):
        C[(i,) * len(ranks)] += 1.0 - 0.1 * i
    X = C
    for k, (N, r) in enumerate(zip(dims, ranks)):
        X = np.moveaxis(np.tensordot(rng.normal(size=(N, r)), X, axes=([1], [k])), 0, k)
    snaps = [X]
    for _ in range(1, n):
        snaps.append(snaps[-1] + amp * rng.normal(size=dims))
    return snaps


def test_sample_mode_fp64_matches_oracle():
    _say("case sample mode fp64")
    from paper_2201_06958_amd import Compressor
    dims, ranks = (6, 16, 12, 3), (3, 4, 4, 3)
    w = [_pcm_weights(2, 3), np.full(16, 1 / 16), np.full(12, 1 / 12), np.full(3, 1 / 3)]
    snaps = _tucker_walk(dims, ranks, 31)
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.05, rank_max=ranks, rank_init=ranks, adaptive=False, eps_th=1.0)
    orc = O.OracleTDB(cfg).init(snaps[0])
    g = Compressor(dims, 0.05, rank_max=ranks, rank_init=ranks, weights=w, data_dtype="f64", precision="f64",
                   adaptive=False, eps_th=1.0)
    g.init_from_factors(_dev(snaps[0]), orc.C, orc.U)
    for k in range(1, len(snaps)):
        rec = orc.ingest(snaps[k])
        g.ingest(_dev(snaps[k]))
        _, C, U = g.get_core_and_bases()
        assert _rel(C, orc.C) < 1e-10, k
        for n in range(4):
            assert _rel(U[n], orc.U[n]) < 1e-10, (k, n)
        assert g.stats()["eps"] == pytest.approx(rec.eps, rel=1e-9), k
    g.close()


def test_stochastic_plume_samples_fp32_match_oracle():
    _say("case stochastic plume samples fp32")
    from streams import stochastic_plume_spec
    from paper_2201_06958_amd import Compressor
    sp = stochastic_plume_spec(nx=24, ny=16, nv=4, s=(2, 3), steps=10, dt=5e-3)
    ranks = (2, 3, 3, 2)   # every core unfolding's sigma ratio above 1e-2 on these samples
    V0 = sp.snapshot_np(0)
    h = O.hosvd(V0.astype(np.float64), sp.weights, ranks)
    C0, U0 = h.truncate(ranks)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=ranks, rank_init=ranks,
                         adaptive=False, eps_th=1.0)
    orc = O.OracleTDB(cfg).init_from_factors(V0.astype(np.float64), C0, U0)
    g = Compressor(sp.dims, sp.dt, rank_max=ranks, rank_init=ranks, weights=sp.weights, data_dtype="f32",
                   precision="f32", adaptive=False, eps_th=1.0)
    g.init_from_factors(_dev(V0), C0, U0)
    for k in range(1, 11):
        x = sp.snapshot_np(k)
        rec = orc.ingest(x.astype(np.float64))
        g.ingest(_dev(x))
        _, C, U = g.get_core_and_bases()
        assert _rel(O.reconstruct(C, U), orc.reconstruct()) < 1e-6, k
        assert abs(g.stats()["eps"] - rec.eps) <= 1e-6 * rec.nu, k
    g.close()
