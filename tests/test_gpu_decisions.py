"""Full-size decision parity on the reactive-flow-shaped stream (512 x 256 x 8, FP32
snapshots, FP32 and BF16-split passes, caps (64, 64, 8) as in the benchmark): from the
oracle's state after 310 steps (tests/golden/plume512_state310.npz, written by
tests/golden/make_plume_state.py from the oracle alone) both sides step through a
window that holds the stream's first reinitialisation (step 322).

Every decision must match the oracle's unless the oracle's error sits inside the
ambiguity band around the threshold it was compared with (|x - thr| <= delta thr,
delta 1e-3 for FP32 and 1e-2 for BF16-split products): then either decision is
correct and the oracle replays the device's decision (its replay mode) and goes on
from there. Per-step errors stay within the precision bar of ||V||_W."""
import copy
import os
import sys

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import plume_spec

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "plume512_state310.npz")
BAR = {"f32": 1e-6, "bf16s": 1e-4}
DELTA = {"f32": 1e-3, "bf16s": 1e-2}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_06958_amd import load_library
    load_library()


def _ambiguous(orc_before, rec, delta):
    """Whether the oracle's decision at this step rested on a comparison inside the
    band: the add trigger (eps vs the trigger), or the removal test's error headroom
    (eps vs eps_th/2) and budget (eps^2 + sigma^2 vs B)."""
    eps = rec.eps
    if abs(eps - orc_before.eps_trig) <= delta * orc_before.eps_trig:
        return True
    if abs(eps - 0.5 * orc_before.eps_th) <= delta * 0.5 * orc_before.eps_th:
        return True
    B = orc_before.budget2(rec.nu ** 2)
    sig = O.core_singular_values(orc_before.C)
    return any(abs(eps * eps + sig[n][orc_before.ranks[n] - 1] ** 2 - B) <= delta * B for n in range(3))


@pytest.mark.parametrize("precision", ["f32", "bf16s"])
def test_full_size_window_with_reinit(precision):
    from paper_2201_06958_amd import Compressor
    g0 = np.load(GOLDEN, allow_pickle=False)
    k0 = int(g0["k0"])
    C, U = g0["C"], [g0["U0"], g0["U1"], g0["U2"]]
    sp = plume_spec()
    caps = (64, 64, 8)
    k1 = k0 + 30
    _say(f"case full-size plume window {k0}..{k1} {precision} ranks {C.shape}")
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=caps, rank_init=None,
                         adaptive=True, eps_th=sp.eps_th)
    V0 = sp.snapshot_np(k0)
    orc = O.OracleTDB(cfg).init_from_factors(V0.astype(np.float64), C, U)
    g = Compressor(sp.dims, sp.dt, rank_max=caps, weights=sp.weights, data_dtype="f32", precision=precision,
                   adaptive=True, eps_th=sp.eps_th)
    g.init_from_factors(_dev(V0), C, U)
    bar, delta = BAR[precision], DELTA[precision]
    events, replays = [], []
    for k in range(k0 + 1, k1 + 1):
        V = sp.snapshot_np(k)
        g.ingest(_dev(V))
        st = g.stats()
        before = copy.deepcopy(orc)
        rec = orc.ingest(V.astype(np.float64))
        assert abs(st["eps"] - rec.eps) <= bar * rec.nu, (k, st["eps"], rec.eps)
        if st["event"] != rec.event:
            assert _ambiguous(before, rec, delta), (k, st["event"], rec.event, rec.eps)
            orc = before
            rec = orc.ingest(V.astype(np.float64), force=st["event"])
            replays.append((k, st["event"]))
        assert st["ranks"] == rec.ranks, k
        if rec.event:
            events.append((k, rec.event, rec.ranks))
            assert abs(st["eps_after"] - rec.eps_after) <= bar * rec.nu, k
    r, Cg, Ug = g.get_core_and_bases()
    rel = float(np.abs(O.reconstruct(Cg, Ug) - orc.reconstruct()).max() / np.abs(orc.reconstruct()).max())
    _say(f"  events {events}, replayed {replays}, final reconstruction rel {rel:.2e}")
    assert events, "the window must hold a controller event"
    assert rel < bar
    g.close()
