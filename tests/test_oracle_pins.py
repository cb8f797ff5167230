"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types an oracle formula: each one checks the oracle against
an independent construction (a brute-force least-squares solve over the tangent
space of the Tucker manifold, a brute-force SVD, a closed-form error, a
convergence order, an invariant, or arithmetic printed in the paper).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import (analytic_cp5_spec, lowrank_manifold_spec, switched_term_spec)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_weights(rng, dims):
    out = []
    for n in dims:
        w = rng.uniform(0.5, 1.5, size=n)
        out.append(w / w.sum())
    return out


def _w_orthonormal(rng, n, r, w):
    s = np.sqrt(w)[:, None]
    q, _ = np.linalg.qr(s * rng.normal(size=(n, r)))
    return q / s


def _complement(U, w):
    """W-orthonormal basis of the W-orthogonal complement of span(U)."""
    n, r = U.shape
    s = np.sqrt(w)[:, None]
    q, _ = np.linalg.qr(np.hstack([s * U, np.eye(n)]))
    return q[:, r:n] / s


# ----------------------------------------------------------------------------- RHS
def _tangent_vector(C, U, dC, dU):
    """dC x_n U_n + sum_n C x_n dU_n x_{k!=n} U_k, written as explicit einsums."""
    p = C.ndim
    assert p == 3
    out = np.einsum("abc,ia,jb,kc->ijk", dC, U[0], U[1], U[2])
    out += np.einsum("abc,ia,jb,kc->ijk", C, dU[0], U[1], U[2])
    out += np.einsum("abc,ia,jb,kc->ijk", C, U[0], dU[1], U[2])
    out += np.einsum("abc,ia,jb,kc->ijk", C, U[0], U[1], dU[2])
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rhs_equals_bruteforce_tangent_least_squares(seed):
    """Sec. 2.2: the closed-form evolution is the weighted least-squares projection
    of the data derivative onto the tangent space of the Tucker manifold (gauge
    U_n^T W_n dU_n = 0). Build that tangent space as a dense matrix and solve."""
    rng = np.random.default_rng(seed)
    dims, ranks = (6, 5, 4), (2, 2, 2)
    w = _rand_weights(rng, dims)
    U = [_w_orthonormal(rng, n, r, wn) for n, r, wn in zip(dims, ranks, w)]
    C = rng.normal(size=ranks)
    D = rng.normal(size=dims)
    Z = [_complement(Un, wn) for Un, wn in zip(U, w)]
    # columns of J: core directions, then K_n entries with dU_n = Z_n K_n
    cols, slots = [], []
    for idx in np.ndindex(*ranks):
        dC = np.zeros(ranks)
        dC[idx] = 1.0
        cols.append(_tangent_vector(C, U, dC, [np.zeros_like(u) for u in U]).ravel())
        slots.append(("C", idx))
    for n in range(3):
        for a in range(Z[n].shape[1]):
            for b in range(ranks[n]):
                dU = [np.zeros_like(u) for u in U]
                dU[n][:, b] = Z[n][:, a]
                cols.append(_tangent_vector(C, U, np.zeros(ranks), dU).ravel())
                slots.append((n, a, b))
    J = np.stack(cols, axis=1)
    sw = np.sqrt(O.weight_tensor(w)).ravel()
    theta, *_ = np.linalg.lstsq(sw[:, None] * J, sw * D.ravel(), rcond=None)
    dC_ls = np.zeros(ranks)
    K = [np.zeros((z.shape[1], r)) for z, r in zip(Z, ranks)]
    for th, sl in zip(theta, slots):
        if sl[0] == "C":
            dC_ls[sl[1]] = th
        else:
            K[sl[0]][sl[1], sl[2]] = th
    Cdot, Udot = O.rhs(C, U, w, D)
    assert np.allclose(Cdot, dC_ls, rtol=0, atol=1e-12 * np.abs(dC_ls).max())
    for n in range(3):
        ref = Z[n] @ K[n]
        assert np.abs(Udot[n] - ref).max() <= 1e-11 * np.abs(ref).max()
    # the tangent vectors agree as well
    tv = _tangent_vector(C, U, Cdot, Udot)
    tv_ls = (J @ theta).reshape(dims)
    assert np.abs(tv - tv_ls).max() <= 1e-12 * np.abs(tv_ls).max()


def test_dynamically_orthogonal_condition():
    """phi = 0 gauge: U_n^T W_n U_dot_n = 0 (Sec. 2.2, after eq. (basecont))."""
    rng = np.random.default_rng(5)
    dims, ranks = (9, 7, 6), (3, 2, 3)
    w = _rand_weights(rng, dims)
    U = [_w_orthonormal(rng, n, r, wn) for n, r, wn in zip(dims, ranks, w)]
    C = rng.normal(size=ranks)
    D = rng.normal(size=dims)
    _, Udot = O.rhs(C, U, w, D)
    for n in range(3):
        g = (U[n].T * w[n][None, :]) @ Udot[n]
        assert np.abs(g).max() <= 1e-13 * max(1.0, np.abs(Udot[n]).max())


def test_rhs_reproduces_derivative_on_manifold():
    """If V(t) stays exactly of multilinear rank r and the state equals V(t), the
    tangent space contains V_dot, so the projection returns it unchanged."""
    sp = lowrank_manifold_spec(dims=(10, 9, 7), ranks=(3, 2, 3), seed=4)
    t = 0.3
    V = sp.field_fn(t, "cpu", None).numpy()
    Vd = sp.deriv_fn(t, "cpu", None).numpy()
    h = O.hosvd(V, sp.weights, (3, 2, 3))
    C, U = h.truncate((3, 2, 3))
    Cdot, Udot = O.rhs(C, U, sp.weights, Vd)
    tv = _tangent_vector(C, U, Cdot, Udot)
    assert np.abs(tv - Vd).max() <= 1e-10 * np.abs(Vd).max()


def test_matrix_case_matches_dynamical_low_rank_projector():
    """p = 2 (the DBO special case, Sec. 2.2): the tangent projection of a rank-r
    matrix is P(D) = P_U D + D P_V - P_U D P_V with W-orthogonal projectors
    P_U = U U^T W_1 and P_V = W_2 V V^T (Koch-Lubich form)."""
    rng = np.random.default_rng(8)
    dims, ranks = (11, 8), (3, 3)
    w = _rand_weights(rng, dims)
    U = [_w_orthonormal(rng, n, r, wn) for n, r, wn in zip(dims, ranks, w)]
    C = rng.normal(size=ranks)
    D = rng.normal(size=dims)
    Cdot, Udot = O.rhs(C, U, w, D)
    tv = U[0] @ Cdot @ U[1].T + Udot[0] @ C @ U[1].T + U[0] @ C @ Udot[1].T
    PU = U[0] @ U[0].T @ np.diag(w[0])
    PVt = np.diag(w[1]) @ U[1] @ U[1].T
    ref = PU @ D + D @ PVt - PU @ D @ PVt
    assert np.abs(tv - ref).max() <= 1e-12 * np.abs(ref).max()


def test_full_rank_mode_has_zero_basis_derivative():
    """r_n = N_n: the complement projection vanishes, so U_dot_n = 0."""
    rng = np.random.default_rng(2)
    dims, ranks = (7, 6, 3), (3, 3, 3)
    w = _rand_weights(rng, dims)
    U = [_w_orthonormal(rng, n, r, wn) for n, r, wn in zip(dims, ranks, w)]
    C = rng.normal(size=ranks)
    _, Udot = O.rhs(C, U, w, rng.normal(size=dims))
    assert np.abs(Udot[2]).max() <= 1e-13
    assert np.abs(Udot[0]).max() > 1e-3


# ----------------------------------------------------------------------------- HOSVD
def test_hosvd_matches_bruteforce_svd():
    """Sec. 2.3/2.4: the bases are the leading left singular vectors of the
    weighted unfoldings; the core is the projection; eps0^2 = nu^2 - ||C||^2."""
    rng = np.random.default_rng(11)
    dims, caps = (8, 7, 5), (4, 3, 5)
    w = _rand_weights(rng, dims)
    V = rng.normal(size=dims) + 3 * np.einsum("i,j,k->ijk", *[rng.normal(size=n) for n in dims])
    h = O.hosvd(V, w, caps)
    Vs = V * O.weight_tensor([np.sqrt(x) for x in w])
    for n in range(3):
        Mn = np.moveaxis(Vs, n, 0).reshape(dims[n], -1)        # any column order
        Us, S, _ = np.linalg.svd(Mn, full_matrices=False)
        assert np.allclose(h.sigma[n][: len(S)], S, rtol=1e-12, atol=1e-12 * S[0])
        r = caps[n]
        P_ref = Us[:, :r] @ Us[:, :r].T
        Ut = np.sqrt(w[n])[:, None] * h.U[n]
        assert np.abs(Ut @ Ut.T - P_ref).max() <= 1e-11
    for ranks in [(1, 1, 1), (2, 3, 2), (4, 3, 5)]:
        C, U = h.truncate(ranks)
        direct = O.weighted_norm2(V - O.reconstruct(C, U), w)
        assert abs(h.truncation_error2(ranks) - direct) <= 1e-11 * O.weighted_norm2(V, w)
        proj = V
        for n in range(3):
            proj = O.mode_product(proj, (U[n].T * w[n][None, :]), n)
        assert np.abs(proj - C).max() <= 1e-12 * np.abs(C).max()


def test_rank_rule_meets_budget_and_validity():
    """The rank rule's result meets the budget (checked by a direct reconstruction)
    and satisfies r_n <= prod_{k != n} r_k. Its growth order is pinned against an
    exhaustive search in test_oracle_pins_control.py."""
    rng = np.random.default_rng(3)
    dims = (9, 8, 6)
    w = [np.full(n, 1.0 / n) for n in dims]
    base = sum(np.einsum("i,j,k->ijk", *[rng.normal(size=n) for n in dims]) * 0.5 ** k for k in range(6))
    V = base + 1e-3 * rng.normal(size=dims)
    caps = (6, 6, 6)
    h = O.hosvd(V, w, caps)
    for budget in [1e-2, 1e-4, 1e-6]:
        B = budget * h.nu2
        r = O.rank_rule(h, caps, B, (1, 1, 1))
        err = O.weighted_norm2(V - O.reconstruct(*h.truncate(r)), w)
        assert err <= B * (1 + 1e-9) or r == caps
        for n in range(3):
            assert r[n] <= np.prod([r[k] for k in range(3) if k != n])


def test_init_is_truncated_hosvd():
    sp = analytic_cp5_spec(n=24, steps=3)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(5, 5, 5),
                         rank_init=(5, 5, 5), adaptive=False)
    V0 = sp.snapshot_np(0)
    o = O.OracleTDB(cfg).init(V0)
    eps_direct, nu = O.error_and_norm(V0, o.C, o.U, sp.weights)
    assert o.records[0].eps == pytest.approx(eps_direct, abs=1e-7 * nu)
    assert eps_direct <= 1e-12 * nu          # exactly rank (5,5,5)


# ----------------------------------------------------------------------------- stepping
def test_orthonormality_and_qr_fold_invariant():
    rng = np.random.default_rng(21)
    dims, ranks = (10, 9, 8), (3, 3, 2)
    w = _rand_weights(rng, dims)
    U = [_w_orthonormal(rng, n, r, wn) + 1e-3 * rng.normal(size=(n, r))
         for n, r, wn in zip(dims, ranks, w)]
    C = rng.normal(size=ranks)
    rec0 = O.reconstruct(C, U)
    C2, U2 = O.reorthonormalize(C, U, w)
    assert np.abs(O.reconstruct(C2, U2) - rec0).max() <= 1e-14 * np.abs(rec0).max() * 10
    for n in range(3):
        g = (U2[n].T * w[n][None, :]) @ U2[n]
        assert np.abs(g - np.eye(ranks[n])).max() < 1e-13


def test_orthonormality_holds_over_steps():
    sp = analytic_cp5_spec(n=32, steps=30)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(5, 5, 5),
                         rank_init=(5, 5, 5), adaptive=False)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    for k in range(1, 31):
        o.ingest(sp.snapshot_np(k))
        for n in range(3):
            g = (o.U[n].T * sp.weights[n][None, :]) @ o.U[n]
            assert np.abs(g - np.eye(5)).max() < 1e-12


def _run_to(sp, T, dt, integrator="heun", use_exact=False):
    sp.dt = dt
    steps = int(round(T / dt))
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=False, integrator=integrator)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    for k in range(1, steps + 1):
        o.ingest(sp.snapshot_np(k))
    return o.records[-1].eps / o.records[-1].nu


@pytest.mark.parametrize("integrator,order", [("heun", 2.0), ("euler", 1.0)])
def test_time_integration_order_on_exactly_low_rank_stream(integrator, order):
    """On an exactly low-rank stream the error is pure time-integration error:
    Heun with the step-average difference quotient is second order; Euler first."""
    sp = lowrank_manifold_spec(dims=(12, 10, 8), ranks=(3, 3, 2), seed=0, rot=0.8)
    T = 0.4
    e1 = _run_to(sp, T, 0.02, integrator)
    e2 = _run_to(sp, T, 0.01, integrator)
    e3 = _run_to(sp, T, 0.005, integrator)
    o1 = math.log2(e1 / e2)
    o2 = math.log2(e2 / e3)
    assert abs(o2 - order) < 0.2, (e1, e2, e3, o1, o2)


def test_core_sigma_follows_hosvd_sigma():
    """Sec. 2.4: the core unfolding singular values follow the leading HOSVD
    singular values of the data (exact here up to integration error)."""
    sp = analytic_cp5_spec(n=32, steps=40)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=(5, 5, 5),
                         rank_init=(5, 5, 5), adaptive=False)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    for k in range(1, 41):
        o.ingest(sp.snapshot_np(k))
    h = O.hosvd(sp.snapshot_np(40), sp.weights, (5, 5, 5))
    sig = O.core_singular_values(o.C)
    for n in range(3):
        assert np.allclose(sig[n], h.sigma[n][:5], rtol=1e-6)


def test_scaling_equivariance():
    """V -> cV gives C -> cC, unchanged bases and eps -> c eps (linearity of the
    evolution equations in the data)."""
    sp = lowrank_manifold_spec(dims=(9, 8, 7), ranks=(2, 3, 2), seed=6)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=0.02, rank_max=(2, 3, 2),
                         rank_init=(2, 3, 2), adaptive=False)
    c = 3.5
    snaps = [sp.field_fn(0.02 * k, "cpu", None).numpy() + 1e-3 * np.sin(k + np.arange(9 * 8 * 7)).reshape(9, 8, 7)
             for k in range(8)]
    a = O.OracleTDB(cfg).init(snaps[0])
    b = O.OracleTDB(cfg).init(c * snaps[0])
    for V in snaps[1:]:
        ra = a.ingest(V)
        rb = b.ingest(c * V)
        assert rb.eps == pytest.approx(c * ra.eps, rel=1e-9)
    assert np.allclose(b.C, c * a.C, rtol=1e-9, atol=1e-12)
    for n in range(3):
        assert np.allclose(b.U[n], a.U[n], rtol=1e-9, atol=1e-12)


def test_full_rank_decomposition_is_exact():
    rng = np.random.default_rng(9)
    dims = (5, 4, 3)
    w = _rand_weights(rng, dims)
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.01, rank_max=dims, rank_init=dims,
                         adaptive=False)
    Vs = [rng.normal(size=dims) for _ in range(5)]
    o = O.OracleTDB(cfg).init(Vs[0])
    for V in Vs[1:]:
        r = o.ingest(V)
        assert r.eps <= 1e-12 * r.nu


# ----------------------------------------------------------------------------- controller
def test_add_fires_when_closed_form_error_crosses_threshold():
    """A base of exact rank (3,3,3) with a static span plus an orthogonal separable
    term ramped on at t_on: the tracked error is h(t) ||q1|| ||q2|| ||q3|| exactly,
    so the add event must fire at the first step where that crosses eps_th."""
    sp = switched_term_spec()
    m = sp.meta
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    expected = next(k for k in range(1, sp.steps + 1) if m["h"](sp.time(k)) * m["qnorm"] > sp.eps_th)
    fired = None
    for k in range(1, sp.steps + 1):
        rec = o.ingest(sp.snapshot_np(k))
        if fired is None:
            # before the first event the tracked error is the closed form
            assert rec.eps == pytest.approx(m["h"](sp.time(k)) * m["qnorm"], abs=1e-10)
        else:
            assert rec.eps <= 1e-10             # rank 4 captures the extra term exactly
        if rec.event in ("add", "reinit") and fired is None:
            fired = k
            assert rec.ranks == (4, 4, 4)
            assert rec.eps_after <= 1e-10
    assert fired == expected


def test_remove_after_term_switches_off():
    """The extra term ramps up (add fires, ranks grow to 4), then decays to a small
    floor: once the weakest core direction fits inside the budget (second form of
    eq. (percentage)) and the error slope over the window is negative, the
    controller removes the extra mode and the error returns to the closed form."""
    t_on, t_peak, t_low, h_min = 0.05, 0.15, 0.35, 0.002

    def h(t):
        if t <= t_on:
            return 0.0
        if t <= t_peak:
            return 2.0 * (t - t_on)
        if t <= t_low:
            return 0.2 + (h_min - 0.2) * (t - t_peak) / (t_low - t_peak)
        return h_min

    def g(t):
        # an unresolved orthogonal term below the budget, decaying: the tracked
        # error is g(t) and its slope is negative
        return 0.004 * math.exp(-t)

    sp = switched_term_spec(steps=140, profile=h, profile2=g)
    q = sp.meta["qnorm"]
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    B = (0.5 * sp.eps_th) ** 2
    events = []
    for k in range(1, sp.steps + 1):
        rec = o.ingest(sp.snapshot_np(k))
        events.append((k, rec.event, rec.ranks))
        t = sp.time(k)
        if rec.event == "":
            assert rec.eps == pytest.approx(math.hypot(h(t), g(t)) if rec.ranks == (3, 3, 3) else g(t),
                                            rel=1e-6)
        if rec.event == "remove":
            # the weakest direction (the extra term, energy h) fits the budget
            assert h(t) ** 2 + g(t) ** 2 <= B
            assert rec.ranks == (3, 3, 3)
            assert rec.eps_after == pytest.approx(math.hypot(h(t), g(t)), rel=1e-8)
    assert any(e[1] == "add" for e in events)
    assert [e for e in events if e[1] == "remove"]
    assert events[-1][2] == (3, 3, 3)
    assert not [e for e in events if e[1] == "numeric"]


def test_numerical_event_restarts_at_numerical_rank():
    """The extra term vanishes exactly: the rank-4 core becomes singular; the
    oracle must restart at the data's numerical rank instead of looping."""
    def h(t):
        return 0.0 if t <= 0.05 or t >= 0.12 else 0.3

    sp = switched_term_spec(steps=40, profile=h)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    evs = [o.ingest(sp.snapshot_np(k)) for k in range(1, sp.steps + 1)]
    numeric = [r for r in evs if r.event == "numeric"]
    assert len(numeric) <= 1
    assert evs[-1].ranks == (3, 3, 3)
    assert evs[-1].eps <= 1e-10


# ----------------------------------------------------------------------------- CR
def test_compression_ratio_arithmetic_from_paper_ranks():
    """Sec. 2.6 CR formula at the channel case's initial ranks (Sec. 3.4), checked
    against exact rational arithmetic."""
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))
    ch = g["channel_initial_ranks"]
    dims = ch["dims"]
    for case, expect in (("case_I", 11.06), ("case_II", 25.40)):
        r = ch[case]["ranks"]
        exact = Fraction(int(np.prod(dims)), sum(a * b for a, b in zip(r, dims)) + int(np.prod(r)))
        assert O.compression_ratio(dims, r) == pytest.approx(float(exact), rel=1e-15)
        assert round(float(exact), 2) == expect


def test_weighted_compression_ratio():
    """Time-weighted harmonic mean (Sec. 2.6): constant CR gives CR; two equal
    intervals at CR a and b give 2ab/(a+b)."""
    assert O.weighted_compression_ratio([0, 1, 2, 3], [7.0, 7.0, 7.0]) == pytest.approx(7.0)
    assert O.weighted_compression_ratio([0.0, 0.5, 1.0], [4.0, 12.0]) == pytest.approx(6.0)
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["reactive_flow"]
    # the printed storage sizes agree with the printed weighted ratio to GB rounding
    assert abs(g["gb_full"] / g["gb_tdb1"] - g["crbar_tdb1"]) / g["crbar_tdb1"] < 0.03
