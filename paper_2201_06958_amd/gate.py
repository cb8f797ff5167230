"""Training and evaluation pipeline of the learned error gate (kernels in
csrc/gate_ops.hip, entry points in include/tdb.h).

The gate predicts log10 of a step's reconstruction error (eq. (error)) from the 16
leading singular values of the three core unfoldings over the last 8 steps (the
singular values of eq. (rot)). Training data are histories of the method itself:
batches of streams advanced with the exact error pass at every step, recording
each step's singular values and exact error. A window of 8 consecutive steps is a
sample when no reinitialisation happened inside it (the device history restarts at
every reinitialisation); its target is the error of its newest step.
"""
from __future__ import annotations

import math
import time
from typing import Callable, Dict, List, Sequence

import numpy as np

from .tdb import Batch, Gate

WINDOW, TOPK, MODES = 8, 16, 3
N_IN = WINDOW * MODES * TOPK


def record_histories(cfgs: Sequence[dict], snapshot: Callable[[int], list], steps: int) -> Dict[str, np.ndarray]:
    """Advance a batch of streams `steps` snapshots with the exact error pass and record,
    per step k (1..steps) and stream i: sigma[k-1, i, n, :16], eps and whether an event
    (reinitialisation) happened."""
    b = Batch(cfgs).init(snapshot(0))
    n = len(cfgs)
    sig = np.zeros((steps, n, MODES, TOPK))
    eps = np.zeros((steps, n))
    ev = np.zeros((steps, n), dtype=bool)
    for k in range(1, steps + 1):
        b.ingest(snapshot(k))
        for i in range(n):
            st = b.streams[i].stats()
            sig[k - 1, i] = np.asarray(st["sigma16"])[:MODES, :TOPK]
            eps[k - 1, i] = st["eps"]
            ev[k - 1, i] = st["event"] != ""
    b.close()
    return {"sigma": sig, "eps": eps, "event": ev}


def window_features(sig_window: np.ndarray) -> np.ndarray:
    """One sample's 384 raw features: log10(max(sigma, 1e-30)), oldest step first, then
    mode, then singular-value index."""
    return np.log10(np.maximum(sig_window, 1e-30)).reshape(-1)


def make_samples(h: Dict[str, np.ndarray]):
    """All windows of 8 steps with no reinitialisation before their newest step; returns
    (X, t) with t = log10 of the newest step's exact error."""
    sig, eps, ev = h["sigma"], h["eps"], h["event"]
    steps, n = eps.shape
    X, t = [], []
    for i in range(n):
        for j in range(WINDOW - 1, steps):
            if ev[j - WINDOW + 1:j, i].any():
                continue
            if not (eps[j, i] > 0.0):
                continue
            X.append(window_features(sig[j - WINDOW + 1:j + 1, i]))
            t.append(math.log10(eps[j, i]))
    return np.asarray(X, dtype=np.float64), np.asarray(t, dtype=np.float64)


def standardisation(X: np.ndarray) -> np.ndarray:
    """Per-feature mean and standard deviation (768 floats); features that never vary
    (e.g. padding beyond the ranks) keep a unit deviation."""
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 1e-6, std, 1.0)
    return np.concatenate([mean, std]).astype(np.float32)


def train(gate: Gate, X: np.ndarray, t: np.ndarray, mean_std: np.ndarray, epochs: int = 30, batch: int = 256,
          lr: float = 1e-3, seed: int = 7, device: str = "cuda") -> List[float]:
    """Adam on mini-batches of standardised samples, one shuffle per epoch (PCG64(seed));
    returns the mean squared error over the whole set after each epoch."""
    import torch
    Xs = (X - mean_std[:N_IN]) / mean_std[N_IN:]
    Xd = torch.tensor(Xs, dtype=torch.float32, device=device)
    td = torch.tensor(t, dtype=torch.float32, device=device)
    rng = np.random.Generator(np.random.PCG64(seed))
    hist = []
    n = Xd.shape[0]
    for _ in range(epochs):
        perm = torch.tensor(rng.permutation(n), device=device)
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            gate.train_step(Xd[idx].contiguous(), td[idx].contiguous(), lr)
        with torch.no_grad():
            ys = [gate.forward(Xd[s:s + gate.max_batch]) for s in range(0, n, gate.max_batch)]
            y = torch.cat(ys)
            hist.append(float(((y - td) ** 2).mean()))
    return hist


def evaluate(cfgs: Sequence[dict], snapshot: Callable[[int], list], steps: int, gate: Gate, mean_std: np.ndarray,
             eps_th: Sequence[float]) -> dict:
    """Shadow run (exact pass at every step, the gate's verdict recorded): skipped-pass
    fraction and mis-decisions, i.e. steps the gate would skip while the exact error
    exceeded the threshold or an add/remove event fired; then the same streams timed
    gated and always exact."""
    import torch
    n = len(cfgs)
    b = Batch(cfgs).init(snapshot(0))
    b.gate_attach(gate, mean_std, "shadow")
    would = 0
    mis = 0
    total = 0
    for k in range(1, steps + 1):
        b.ingest(snapshot(k))
        for i in range(n):
            st = b.streams[i].stats()
            total += 1
            if st["would_skip"]:
                would += 1
                if st["eps"] > eps_th[i] or st["event"] != "":
                    mis += 1
    b.close()
    out = {"steps": total, "skipped_fraction": would / total, "misdecision_rate": mis / total, "misdecisions": mis}
    # the decisions themselves, exact and gated: any difference (e.g. a removal delayed
    # because skipped steps emptied the slope window) counts as a mis-decision too
    events = {}
    for mode in ("off", "active"):
        b = Batch(cfgs).init(snapshot(0))
        if mode == "active":
            b.gate_attach(gate, mean_std, "active")
        seq = []
        for k in range(1, steps + 1):
            b.ingest(snapshot(k))
            seq.append([b.streams[i].stats()["event"] for i in range(n)])
        events[mode] = seq
        b.close()
    out["decision_mismatches"] = sum(1 for k in range(steps) for i in range(n)
                                     if events["off"][k][i] != events["active"][k][i])
    out["events_exact"] = sum(1 for k in range(steps) for i in range(n) if events["off"][k][i])
    rates = {}
    for mode in ("off", "active"):
        b = Batch(cfgs).init(snapshot(0))
        if mode == "active":
            b.gate_attach(gate, mean_std, "active")
        for k in range(1, 4):
            b.ingest(snapshot(k))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(4, steps + 1):
            b.ingest(snapshot(k))
        torch.cuda.synchronize()
        rates[mode] = n * (steps - 3) / (time.perf_counter() - t0)
        b.close()
    out["snapshots_per_s_exact"] = rates["off"]
    out["snapshots_per_s_gated"] = rates["active"]
    return out
