"""Pins of the oracle's time schemes (Sec. 2.3 and 2.4, the Runge study of Sec. 3.1):
the second-order stage derivatives against closed forms, a whole run with them against
the run given the exact stage derivatives, the convergence orders of the Heun and
explicit Euler steps by step halving, and the calibrated Runge behaviour (the rank
rises and falls, fixed low ranks exceed the threshold, RK2 beats explicit Euler)."""
import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import runge_spec


def test_fd2_stage_derivatives_exact_for_quadratics():
    """For V(t) = A + tB + t^2 G the two stage derivatives are the exact dV/dt at t_k
    and t_{k+1} (a wrong coefficient, sign or step breaks this)."""
    rng = np.random.default_rng(5)
    A, B, G = (rng.normal(size=(4, 3, 2)) for _ in range(3))
    dt, tk = 0.03, 0.7
    V = lambda t: A + t * B + t * t * G
    dV = lambda t: B + 2.0 * t * G
    D1, D2 = O.fd2_stage_derivatives(V(tk - dt), V(tk), V(tk + dt), dt)
    assert np.abs(D1 - dV(tk)).max() < 1e-12 * np.abs(dV(tk)).max()
    assert np.abs(D2 - dV(tk + dt)).max() < 1e-12 * np.abs(dV(tk + dt)).max()
    # and second order on a cubic: the errors shrink by 4 when dt halves
    H = rng.normal(size=(4, 3, 2))
    Vc = lambda t: V(t) + t ** 3 * H
    dVc = lambda t: dV(t) + 3.0 * t * t * H
    errs = []
    for h in (0.02, 0.01):
        d1, d2 = O.fd2_stage_derivatives(Vc(tk - h), Vc(tk), Vc(tk + h), h)
        errs.append((np.abs(d1 - dVc(tk)).max(), np.abs(d2 - dVc(tk + h)).max()))
    assert 3.5 < errs[0][0] / errs[1][0] < 4.5 and 3.5 < errs[0][1] / errs[1][1] < 4.5


def _quadratic_stream(dims=(9, 8, 6), seed=7):
    """V(t) = A + t B + t^2 G with A, B, G of rank 3 plus a small full-rank part, so
    that a rank-3 run has to turn its bases (on data exactly of the run's rank every
    scheme is exact: the bases stand still and C follows the data's coefficients)."""
    rng = np.random.default_rng(seed)

    def part(scale):
        X = rng.normal(size=(3, 3, 3)) * np.array([1.0, 0.5, 0.25])[:, None, None]
        for n, N in enumerate(dims):
            X = np.moveaxis(np.tensordot(rng.normal(size=(N, 3)), X, axes=([1], [n])), 0, n)
        return scale * X + 0.02 * rng.normal(size=dims)

    A, B, G = part(1.0), part(0.5), part(0.3)
    return [np.full(n, 1.0 / n) for n in dims], (lambda t: A + t * B + t * t * G), (lambda t: B + 2.0 * t * G)


def _run_quadratic(dt, integrator="heun", fd_order=1, given=None, T=0.5, dims=(9, 8, 6)):
    """Fixed rank 3 from the truncated HOSVD of V(0) to t = T; given(k, t0, t1) -> D."""
    w, V, dV = _quadratic_stream(dims)
    cfg = O.OracleConfig(dims=dims, weights=w, dt=dt, rank_max=(3, 3, 3), rank_init=(3, 3, 3), adaptive=False,
                         eps_th=1.0, integrator=integrator, fd_order=fd_order)
    o = O.OracleTDB(cfg).init(V(0.0))
    out = []
    for k in range(1, int(round(T / dt)) + 1):
        t0, t1 = (k - 1) * dt, k * dt
        rec = o.ingest(V(t1), D=None if given is None else given(k, t0, t1, dV))
        out.append((rec.eps, o.reconstruct()))
    return out


def test_fd2_run_equals_exact_stage_derivatives_on_quadratic_data():
    """With data quadratic in t the second-order stage derivatives are exact, so the
    run equals, step by step, the run given dV/dt at both stage times (both take the
    first-order quotient on the first step, where no earlier snapshot exists); the
    first-order quotient held over both stages does not."""
    dt = 0.02
    a = _run_quadratic(dt, fd_order=2)
    b = _run_quadratic(dt, given=lambda k, t0, t1, dV: None if k == 1 else (dV(t0), dV(t1)))
    c = _run_quadratic(dt)
    for (ea, Xa), (eb, Xb) in zip(a, b):
        assert abs(ea - eb) <= 1e-11 * max(ea, 1e-300)
        assert np.abs(Xa - Xb).max() <= 1e-11 * np.abs(Xb).max()
    assert np.abs(c[-1][1] - b[-1][1]).max() > 1e-5 * np.abs(b[-1][1]).max()


@pytest.mark.parametrize("integrator,order", [("heun", 2), ("euler", 1)])
def test_scheme_convergence_order(integrator, order):
    """Step halving with the exact derivative (dV/dt at t_k, and at t_{k+1} for Heun's
    second stage): successive differences of the state at t = 0.5 shrink by 2^order."""
    given = (lambda k, t0, t1, dV: dV(t0)) if integrator == "euler" else (lambda k, t0, t1, dV: (dV(t0), dV(t1)))
    X = [_run_quadratic(0.05 / 2 ** j, integrator, given=given)[-1][1] for j in range(4)]
    d = [np.abs(X[j] - X[j + 1]).max() for j in range(3)]
    for j in range(2):
        assert 0.8 * 2 ** order < d[j] / d[j + 1] < 1.2 * 2 ** order, d


RUNGE_N = 32
RUNGE_EPS_TH = 2.5e-3   # calibrated between the rank-3 and rank-4 truncation errors over t in [0, 2]
RUNGE_GAMMA = 99.99     # total-energy budget that separates rank 3 (t = 0, 2) from rank 4 (t = 1)


def _runge_run(adaptive, r0, steps=400, integrator="heun", n=RUNGE_N, exact=False):
    sp = runge_spec(n=n, steps=steps)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(8, 8, 8) if adaptive else r0,
                         rank_init=r0, adaptive=adaptive, eps_th=RUNGE_EPS_TH, gamma_th=RUNGE_GAMMA,
                         integrator=integrator)
    V0 = sp.snapshot_np(0).astype(np.float64)
    C0, U0 = O.hosvd(V0, sp.weights, cfg.caps()).truncate(r0)
    o = O.OracleTDB(cfg).init_from_factors(V0, C0, U0)
    recs = []
    for k in range(1, steps + 1):
        D = None
        if exact:
            D = sp.derivative_np(k - 1) if integrator == "euler" else (sp.derivative_np(k - 1), sp.derivative_np(k))
        recs.append(o.ingest(sp.snapshot_np(k).astype(np.float64), D=D))
    return recs


def test_runge_calibrated_rank_history():
    """The Runge stream from rank 3 (Sec. 3.1): the adaptive run grows a rank while a(t)
    dips towards t = 1 and returns to rank 3 before t = 2, keeping the error at the
    threshold except on the steps that trigger an event; fixed ranks 2 and 3 exceed it."""
    recs = _runge_run(True, (3, 3, 3))
    t = np.array([r.k * 5e-3 for r in recs])
    rmax = np.array([max(r.ranks) for r in recs])
    assert rmax[t < 0.3].max() == 3
    assert rmax[(t > 0.3) & (t < 1.0)].max() >= 4
    assert tuple(recs[-1].ranks) == (3, 3, 3)
    events = [r for r in recs if r.event]
    over = sum(r.eps > RUNGE_EPS_TH * (1 + 1e-9) for r in recs)
    assert over <= len(events) + 2, (over, [(r.k, r.event) for r in events])
    assert any(r.event == "add" for r in events) and any(r.event == "remove" for r in events)
    for rr, frac in (((2, 2, 2), 0.99), ((3, 3, 3), 0.3)):
        fixed = _runge_run(False, rr)
        assert sum(r.eps > RUNGE_EPS_TH for r in fixed) >= frac * len(fixed), rr


def test_runge_rk2_beats_euler_with_exact_derivative():
    """Fixed rank 4 on a 24^3 Runge grid over t in [0, 1] with the exact derivative: the
    second-order Heun step ends closer to the data than explicit Euler."""
    heun = _runge_run(False, (4, 4, 4), steps=200, n=24, exact=True)
    euler = _runge_run(False, (4, 4, 4), steps=200, n=24, exact=True, integrator="euler")
    assert heun[-1].eps < euler[-1].eps
    assert max(r.eps for r in heun) < max(r.eps for r in euler)
