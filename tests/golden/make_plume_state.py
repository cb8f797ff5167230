"""Writes plume512_state310.npz: the FP64 oracle's state after 310 steps of the
reactive-flow-shaped stream (512 x 256 x 8, FP32 snapshots, caps (64, 64, 8),
threshold 1e-4, ranks from the rank rule), the starting point of the full-size
decision-parity window in tests/test_gpu_decisions.py. Calls only the oracle and the
seeded stream generator.

    python tests/golden/make_plume_state.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tdb_oracle as O  # noqa: E402
from streams import plume_spec  # noqa: E402

K0 = 310
CAPS = (64, 64, 8)


def main():
    sp = plume_spec()
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=CAPS, rank_init=None,
                         adaptive=True, eps_th=sp.eps_th)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0).astype(np.float64))
    events = []
    for k in range(1, K0 + 1):
        rec = o.ingest(sp.snapshot_np(k).astype(np.float64))
        if rec.event:
            events.append((k, rec.event))
    out = os.path.join(HERE, f"plume512_state{K0}.npz")
    np.savez_compressed(out, k0=K0, C=o.C, U0=o.U[0], U1=o.U[1], U2=o.U[2],
                        events=np.array([e[0] for e in events], dtype=np.int64))
    print(out, o.ranks, events)


if __name__ == "__main__":
    main()
