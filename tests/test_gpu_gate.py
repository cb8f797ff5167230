"""GPU tests of the learned error gate: its forward pass, gradient and Adam step
against the FP64 oracle (bar 1e-4 relative, FP32 arithmetic), and what the trained
network gains over the method without it on streams it has not seen."""
import sys

import numpy as np
import pytest

from oracle import gate_oracle as GO
from streams import fourier_ensemble_specs, gate_init_params, plume_spec

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


def _batch_data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, GO.N_IN)).astype(np.float32)
    t = rng.normal(loc=-6.0, size=n).astype(np.float32)
    return X, t


def test_forward_gradient_and_adam_against_oracle():
    from paper_2201_06958_amd import Gate
    theta = gate_init_params(11)
    X, t = _batch_data(96, 3)
    g = Gate(max_batch=128)
    g.set_params(theta)
    Xd = torch.from_numpy(X).cuda()
    td = torch.from_numpy(t).cuda()
    y = g.forward(Xd).cpu().numpy()
    yo, cache = GO.forward(theta.astype(np.float64), X.astype(np.float64))
    rel_y = np.abs(y - yo).max() / np.abs(yo).max()
    grad, loss = g.grad(Xd, td)
    grad = grad.cpu().numpy()
    go = GO.backward(theta.astype(np.float64), cache, yo, t.astype(np.float64))
    rel_g = np.abs(grad - go).max() / np.abs(go).max()
    rel_l = abs(loss - GO.loss(yo, t)) / GO.loss(yo, t)
    _say(f"  gate forward rel {rel_y:.2e}, gradient rel {rel_g:.2e}, loss rel {rel_l:.2e}")
    assert rel_y < 1e-5 and rel_g < 1e-4 and rel_l < 1e-5
    # one Adam step from fresh moments
    g.train_step(Xd, td, 1e-3)
    new = g.get_params().astype(np.float64)
    expect, _, _ = GO.adam(theta.astype(np.float64), go, np.zeros_like(go), np.zeros_like(go), 1, 1e-3)
    step_g = new - theta
    step_o = expect - theta
    # Adam's first step is lr * g / (|g| + eps): compare where the gradient is not tiny
    big = np.abs(go) > 1e-4 * np.abs(go).max()
    rel_s = np.abs(step_g[big] - step_o[big]).max() / np.abs(step_o[big]).max()
    _say(f"  adam step rel {rel_s:.2e}")
    assert rel_s < 1e-3
    g.close()


def _cfg(sp, rank_max=None):
    return dict(dims=sp.dims, dt=sp.dt, rank_max=rank_max or sp.rank_max, weights=sp.weights, data_dtype="f32",
                precision="f32", adaptive=True, eps_th=sp.eps_th, snapshot_mode="copy")


def _streams(seed0, n_ens, n_plume, steps):
    specs = fourier_ensemble_specs(n_streams=n_ens, seed0=seed0, steps=steps + 1)
    cfgs = [_cfg(sp) for sp in specs]
    rng = np.random.default_rng(seed0)
    for j in range(n_plume):
        sp = plume_spec(nx=128, ny=64, nv=8, steps=steps + 1, noise_seed=100 * seed0 + 17 * j,
                        centre_shift=(float(rng.uniform(0, 2)), float(rng.uniform(0, 1))))
        specs.append(sp)
        cfgs.append(_cfg(sp, rank_max=(32, 32, 8)))
    cache = {}

    def snapshot(k):
        if k not in cache:
            cache.clear()
            cache[k] = [sp.snapshot(k, device="cuda") for sp in specs]
        return cache[k]
    return specs, cfgs, snapshot


def test_trained_gate_skips_error_passes_without_misdecisions():
    """Train on histories of held-out streams (ensemble members and reactive-flow
    streams with shifted plumes and other noise seeds), then run fresh streams: the
    gate must skip most error passes far below the threshold, never skip a step whose
    exact error exceeds the threshold or that takes an event, and leave the compressed
    state unchanged."""
    from paper_2201_06958_amd import Batch, Gate
    from paper_2201_06958_amd import gate as GP
    steps = 60
    specs, cfgs, snap = _streams(5000, 12, 4, steps)
    _say(f"case gate training histories: {len(cfgs)} streams x {steps} steps")
    h = GP.record_histories(cfgs, snap, steps)
    X, t = GP.make_samples(h)
    ms = GP.standardisation(X)
    g = Gate(max_batch=1024)
    g.set_params(gate_init_params(11))
    hist = GP.train(g, X, t, ms, epochs=30, batch=256, lr=1e-3)
    _say(f"  {X.shape[0]} samples, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.25 * hist[0]
    # fresh streams
    specs2, cfgs2, snap2 = _streams(9000, 8, 2, 40)
    ev = GP.evaluate(cfgs2, snap2, 40, g, ms, [sp.eps_th for sp in specs2])
    _say(f"  evaluation: {ev}")
    assert ev["skipped_fraction"] > 0.4
    assert ev["misdecisions"] == 0 and ev["decision_mismatches"] == 0
    # gated and exact runs end in the same state
    outs = []
    for mode in ("off", "active"):
        b = Batch(cfgs2).init(snap2(0))
        if mode == "active":
            b.gate_attach(g, ms, "active")
        gated = 0
        for k in range(1, 41):
            b.ingest(snap2(k))
            gated += sum(int(b.streams[i].stats()["gated"]) for i in range(len(cfgs2)))
        outs.append([b.streams[i].get_core_and_bases() for i in range(len(cfgs2))])
        if mode == "active":
            _say(f"  gated passes: {gated}")
            assert gated > 0
        b.close()
    for (r0, C0, U0), (r1, C1, U1) in zip(*outs):
        assert r0 == r1
        assert np.array_equal(C0, C1)
        for a, c in zip(U0, U1):
            assert np.array_equal(a, c)
    g.close()


def _single_stream(seed=3):
    sp = plume_spec(nx=128, ny=64, nv=8, steps=30, noise_seed=seed)
    cfg = dict(dims=sp.dims, dt=sp.dt, rank_max=(32, 32, 8), weights=sp.weights, data_dtype="f32",
               precision="f32", adaptive=True, eps_th=sp.eps_th, snapshot_mode="borrow")
    return sp, cfg


def test_single_stream_gate_features_match_training_features():
    """Train/serve skew: in shadow mode the device predicts from FP32 log10 features
    it forms itself; the same network evaluated in FP64 on features built by the
    training pipeline (numpy log10 of the reported singular values) must agree."""
    from paper_2201_06958_amd import Compressor
    from paper_2201_06958_amd import gate as GP
    sp, cfg = _single_stream()
    _say("case single-stream gate features")
    rng = np.random.default_rng(5)
    theta = gate_init_params(11)
    ms = np.concatenate([rng.normal(size=GO.N_IN) - 3.0, rng.uniform(0.5, 2.0, size=GO.N_IN)]).astype(np.float32)
    g = Compressor(**cfg)
    g.init(sp.snapshot(0, device="cuda"))
    g.gate_load(theta, ms, "shadow")
    snaps = [sp.snapshot(k, device="cuda") for k in range(sp.steps + 1)]
    sig_hist = []
    worst = 0.0
    checked = 0
    for k in range(1, sp.steps + 1):
        g.ingest(snaps[k])
        g.flush()
        st = g.stats()
        if st["event"]:
            sig_hist = []
            continue
        sig_hist.append(np.asarray(st["sigma16"])[:3, :16])
        if len(sig_hist) >= 8:
            x = GP.window_features(np.asarray(sig_hist[-8:]))
            xs = (x - ms[:GO.N_IN].astype(np.float64)) / ms[GO.N_IN:].astype(np.float64)
            y, _ = GO.forward(theta.astype(np.float64), xs[None, :])
            yd = np.log10(st["eps_pred"])
            worst = max(worst, abs(float(y[0]) - yd))
            checked += 1
    _say(f"  {checked} predictions, worst |log10 difference| {worst:.2e}")
    assert checked >= 10
    assert worst < 1e-4 * max(1.0, abs(float(y[0])))
    g.close()


@pytest.mark.parametrize("bias,expect_skip", [(-40.0, True), (10.0, False)])
def test_single_stream_gate_active_skips_and_keeps_state(bias, expect_skip):
    """tdb_gate_load on one stream: a network whose output is the constant b3 skips
    every pass it may (b3 far below the threshold) or none (b3 above it); the
    compressed state equals the always-exact run's bit for bit, and a skipped step
    reports NaN as its error. The analytic stream at fixed ranks with a tiny
    threshold has no removal candidate, so only the prediction decides."""
    from paper_2201_06958_amd import Compressor
    from streams import analytic_cp5_spec
    sp = analytic_cp5_spec(n=32, steps=30)
    cfg = dict(dims=sp.dims, dt=sp.dt, rank_max=(5, 5, 5), rank_init=(5, 5, 5), weights=sp.weights,
               data_dtype="f64", precision="f64", adaptive=False, eps_th=1e-8, snapshot_mode="borrow")
    _say(f"case single-stream gate active b3={bias}")
    theta = np.zeros(GO.N_PARAMS, dtype=np.float32)
    theta[-1] = bias
    ms = np.concatenate([np.zeros(384), np.ones(384)]).astype(np.float32)
    snaps = [torch.from_numpy(sp.snapshot_np(k)).cuda() for k in range(sp.steps + 1)]
    states, gated = [], 0
    for mode in ("off", "active"):
        g = Compressor(**cfg)
        g.init(snaps[0])
        if mode == "active":
            g.gate_load(theta, ms, "active")
        for k in range(1, sp.steps + 1):
            g.ingest(snaps[k])
            if mode == "active":
                g.flush()
                st = g.stats()
                if st["gated"]:
                    gated += 1
                    assert np.isnan(st["eps"])
                else:
                    assert np.isfinite(st["eps"])
        states.append(g.get_core_and_bases())
        g.close()
    (r0, C0, U0), (r1, C1, U1) = states
    assert r0 == r1 and np.array_equal(C0, C1)
    for a, c in zip(U0, U1):
        assert np.array_equal(a, c)
    _say(f"  gated steps {gated}")
    assert (gated == sp.steps - 7) if expect_skip else (gated == 0)
