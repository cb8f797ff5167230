"""GPU parity of the fused third-order step at the shapes of the TDB-against-HOSVD sweep
(N x N x N cubes of the five-term analytic stream in FP32 storage, ranks fixed at
(5, 5, 5); Sec. 2.6 and the scalability comparison of the paper). With N_3 > 8 the stage
pass runs on the vector-ALU tiles, and at N = 192 the tile plan is shrunk to fit LDS.
Against the FP64 oracle fed the same rounded snapshots: the reconstruction at 1e-6
relative and eps within 1e-6 of nu per step, and the HOSVD at init (ranks and
reconstruction) at 1e-6."""
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_06958_amd import load_library
    load_library()


@pytest.mark.parametrize("n,steps", [(40, 5), (96, 4), (192, 2)])
def test_sweep_shape_fp32_matches_oracle(n, steps):
    _say(f"case sweep cube N {n}")
    from streams import analytic_cp5_spec
    from paper_2201_06958_amd import Compressor
    sp = analytic_cp5_spec(n=n, steps=steps + 1)
    snaps = [sp.snapshot_np(k).astype(np.float32) for k in range(steps + 1)]
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(5, 5, 5), rank_init=(5, 5, 5),
                         adaptive=False, eps_th=1.0)
    orc = O.OracleTDB(cfg).init(snaps[0].astype(np.float64))
    g = Compressor(sp.dims, sp.dt, rank_max=(5, 5, 5), rank_init=(5, 5, 5), weights=sp.weights, data_dtype="f32",
                   precision="f32", adaptive=False, eps_th=1.0)
    g.init(torch.from_numpy(snaps[0]).cuda())
    r, C, U = g.get_core_and_bases()
    assert tuple(r[:3]) == (5, 5, 5)
    assert _rel(O.reconstruct(C, U), orc.reconstruct()) < 1e-6
    for k in range(1, steps + 1):
        rec = orc.ingest(snaps[k].astype(np.float64))
        g.ingest(torch.from_numpy(snaps[k]).cuda())
        st = g.stats()
        _, C, U = g.get_core_and_bases()
        assert _rel(O.reconstruct(C, U), orc.reconstruct()) < 1e-6, k
        assert abs(st["eps"] - rec.eps) <= 1e-6 * rec.nu, k
        assert st["path_used"] == "fused"
    g.close()
