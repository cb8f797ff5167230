"""Pins of the oracle's controller-side functions and of the energetic rotation.

Each test checks the oracle against something it does not compute itself: an
exhaustive enumeration, a closed-form error or budget on a stream built from
W-orthonormal separable terms, a singular value decomposition from the library, or
an invariant the paper states. Next to each test is the plausible mistake in the
oracle that it catches.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import tdb_oracle as O
from streams import switched_term_spec


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


# ------------------------------------------------------------------ eq. (rot)
@pytest.mark.parametrize("seed", [0, 1])
def test_core_rotation_is_the_energetic_rotation(seed):
    """Sec. 2.4, eq. (rot): rotating each basis by the descending eigenvectors of its
    core unfolding's Gram (and the core by their transposes) leaves the
    reconstruction unchanged and makes every mode-n Gram of the rotated core diagonal
    with the squared singular values of C_(n) on it, largest first.

    Caught mistakes: ascending eigenvectors (diagonal not descending); C x_n Psi in
    place of Psi^T (reconstruction changes, Grams not diagonal); rotating U by
    Psi^T (reconstruction changes); a missing sign fix (sign test)."""
    rng = np.random.default_rng(seed)
    dims, ranks = (9, 8, 7), (4, 3, 5)
    w = _rand_weights(rng, dims)
    U = [_w_orthonormal(rng, n, r, wn) for n, r, wn in zip(dims, ranks, w)]
    C = rng.normal(size=ranks)
    Co, Uo = O.core_rotation(C, U)
    rec, reco = O.reconstruct(C, U), O.reconstruct(Co, Uo)
    assert np.abs(reco - rec).max() <= 1e-13 * np.abs(rec).max()
    for n in range(3):
        # Kolda-Bader unfolding written out independently of the oracle's helper
        perm = [n] + [k for k in range(3) if k != n]
        Mn = np.transpose(Co, perm).reshape(ranks[n], -1)
        G = Mn @ Mn.T
        off = G - np.diag(np.diag(G))
        assert np.abs(off).max() <= 1e-12 * np.abs(G).max()
        d = np.diag(G)
        assert np.all(d[:-1] >= d[1:])
        s_ref = np.linalg.svd(np.transpose(C, perm).reshape(ranks[n], -1), compute_uv=False)
        assert np.allclose(np.sqrt(d), s_ref, rtol=1e-12, atol=1e-13 * s_ref[0])
        # the rotated bases stay W-orthonormal
        g = (Uo[n].T * w[n][None, :]) @ Uo[n]
        assert np.abs(g - np.eye(ranks[n])).max() <= 1e-13
        # Psi = U^T W U_rot: each column's entry of largest magnitude is positive
        Psi = (U[n].T * w[n][None, :]) @ Uo[n]
        for j in range(ranks[n]):
            i = int(np.argmax(np.abs(Psi[:, j])))
            assert Psi[i, j] > 0


# ------------------------------------------------------------------ rank rule
def _merged_order(h, caps):
    """Every growth step (mode n, its j-th direction, j >= 2) sorted by the next
    full-data singular value, largest first; a tie goes to the lower mode."""
    items = []
    for n in range(len(caps)):
        for j in range(1, caps[n]):
            items.append((-h.sigma[n][j], n, j))
    items.sort()
    return [(n, j) for _, n, j in items]


def _search_rank(h, caps, B):
    """Exhaustive search over every rank tuple up to the caps: among the tuples whose
    added directions are exactly a prefix of the merged order (the directions kept
    are the strongest ones overall), the one with the fewest directions that meets
    the budget; the caps when none does."""
    order = _merged_order(h, caps)
    best = None
    for r in itertools.product(*[range(1, c + 1) for c in caps]):
        added = {(n, j) for n in range(len(caps)) for j in range(1, r[n])}
        m = len(added)
        if set(order[:m]) != added:
            continue
        if h.truncation_error2(r) <= B and (best is None or m < best[0]):
            best = (m, r)
    return best[1] if best else tuple(caps)


def _valid(r):
    return all(r[n] <= np.prod([r[k] for k in range(len(r)) if k != n]) for n in range(len(r)))


def test_rank_rule_against_exhaustive_search():
    """Sec. 2.5, eq. (percentage): the greedy growth equals an exhaustive search over
    every rank tuple up to the caps (the fewest strongest directions meeting the
    budget), and validity repair only grows.

    Caught mistakes: growing the mode with the smallest next singular value, or by
    mode index; stopping one step late or early; a budget test on e instead of e^2."""
    rng = np.random.default_rng(3)
    dims = (9, 8, 6)
    w = [np.full(n, 1.0 / n) for n in dims]
    base = sum(np.einsum("i,j,k->ijk", *[rng.normal(size=n) for n in dims]) * 0.5 ** k for k in range(6))
    V = base + 1e-3 * rng.normal(size=dims)
    caps = (6, 6, 6)
    h = O.hosvd(V, w, caps)
    seen = set()
    for frac in [3e-1, 1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8]:
        B = frac * h.nu2
        want = _search_rank(h, caps, B)
        # the greedy before its validity repair is the searched tuple
        r = [1, 1, 1]
        while h.truncation_error2(r) > B:
            cand = [n for n in range(3) if O._can_grow(h, caps, r, n)]
            if not cand:
                break
            r[max(cand, key=lambda n: (O._next_sigma(h, r, n), -n))] += 1
        assert tuple(r) == want, (frac, r, want)
        got = O.rank_rule(h, caps, B, (1, 1, 1))
        assert _valid(got)
        assert all(g >= a for g, a in zip(got, want))
        if _valid(want):
            assert got == want
        # the budget holds for the final tuple, by a direct reconstruction
        err = O.weighted_norm2(V - O.reconstruct(*h.truncate(got)), w)
        assert err <= B * (1 + 1e-9) or got == caps
        seen.add(got)
    assert len(seen) >= 5        # the budgets exercise many different tuples


def test_rank_rule_tie_goes_to_lowest_mode():
    """A supersymmetric tensor has the same singular values in every mode, so every
    growth step is a three-way tie. With a symmetric core whose entry (2, 1, 1) is
    not zero, growing any one mode to rank 2 lowers the error; for a budget between
    e(1,1,1)^2 and e(2,1,1)^2 the greedy stops after one growth, which must go to
    the lowest mode, and validity repair then grows the lowest other mode: (2, 2, 1).

    Caught mistakes: the highest mode on a tie (gives (1, 2, 2)); ties broken by an
    unstable sort."""
    rng = np.random.default_rng(4)
    n, r = 7, 4
    G = rng.normal(size=(r, r, r)) * np.array([1.0, 0.5, 0.25, 0.125])[:, None, None]
    G = sum(np.transpose(G, pm) for pm in itertools.permutations(range(3))) / 6.0
    q, _ = np.linalg.qr(rng.normal(size=(n, r)))
    V = np.einsum("abc,ia,jb,kc->ijk", G, q, q, q)
    Vs = np.empty_like(V)           # exact symmetry: every entry from its sorted index
    for idx in np.ndindex(*V.shape):
        Vs[idx] = V[tuple(sorted(idx))]
    w = [np.full(n, 1.0 / n)] * 3
    caps = (4, 4, 4)
    h = O.hosvd(Vs, w, caps)
    for k in range(3):
        assert np.array_equal(h.sigma[0], h.sigma[k])
    e111, e211 = h.truncation_error2((1, 1, 1)), h.truncation_error2((2, 1, 1))
    assert e211 < 0.9 * e111
    assert h.truncation_error2((1, 1, 2)) == pytest.approx(e211, rel=1e-10)
    B = 0.5 * (e111 + e211)
    assert _search_rank(h, caps, B) == (2, 1, 1)
    assert O.rank_rule(h, caps, B, (1, 1, 1)) == (2, 2, 1)
    assert _merged_order(h, caps)[:3] == [(0, 1), (1, 1), (2, 1)]


# ------------------------------------------------------------------ gamma_th budget
def _diag_tensor(rng, dims, a, w):
    """sum_k a_k q1_k o q2_k o q3_k with W-orthonormal factors: its weighted HOSVD
    has core energies a_k^2 on the diagonal, so the truncation error at (r, r, r)
    is sum_{k > r} a_k^2 in closed form."""
    Q = [_w_orthonormal(rng, n, len(a), wn) for n, wn in zip(dims, w)]
    return sum(ak * np.einsum("i,j,k->ijk", Q[0][:, k], Q[1][:, k], Q[2][:, k]) for k, ak in enumerate(a))


@pytest.mark.parametrize("r_want", [1, 2, 3, 4])
def test_gamma_budget_at_init_closed_form(r_want):
    """Sec. 2.5, eq. (percentage), paper-style: with gamma_th the rank rule keeps the
    captured energy above gamma_th percent of ||V||_W^2, i.e. budget
    (1 - gamma_th/100) nu^2. On a diagonal-core stream the smallest such rank is
    known in closed form; gamma_th is put halfway between two captured fractions.

    Caught mistakes: gamma/100 in place of 1 - gamma/100; nu in place of nu^2;
    a captured fraction measured against ||C||^2 instead of ||V||^2."""
    rng = np.random.default_rng(7)
    dims = (10, 9, 8)
    w = _rand_weights(rng, dims)
    a = np.array([4.0, 2.0, 1.0, 0.5, 0.25, 0.125])
    V = _diag_tensor(rng, dims, a, w)
    nu2 = float(np.sum(a ** 2))
    tail = [float(np.sum(a[r:] ** 2)) for r in range(len(a) + 1)]
    # captured fraction at rank r is 1 - tail[r]/nu2; choose gamma between r-1 and r
    frac = 0.5 * ((1 - tail[r_want - 1] / nu2) + (1 - tail[r_want] / nu2))
    gamma = 100.0 * frac
    cfg = O.OracleConfig(dims=dims, weights=w, dt=0.01, rank_max=(6, 6, 6), adaptive=True,
                         eps_th=1e-12, gamma_th=gamma)
    o = O.OracleTDB(cfg).init(V)
    assert o.budget2(nu2) == pytest.approx((1 - frac) * nu2, rel=1e-12)
    assert o.ranks == (r_want,) * 3
    assert o.records[0].eps == pytest.approx(math.sqrt(tail[r_want]), rel=1e-8)


@pytest.mark.parametrize("side", ["below", "above"])
def test_gamma_budget_decides_the_add(side):
    """Switched stream: at the first step whose closed-form error h(t) exceeds eps_th
    the controller reinitialises; the HOSVD at the current ranks leaves exactly h(t)
    (the extra term is W-orthogonal to the base span), and the rank rule grows the
    ranks to (4, 4, 4) only when h^2 exceeds the paper-style budget
    (1 - gamma_th/100) nu^2, with nu^2 = ||base||^2 + h^2 in closed form."""
    sp0 = switched_term_spec()
    m = sp0.meta
    k_fire = next(k for k in range(1, sp0.steps + 1) if m["h"](sp0.time(k)) * m["qnorm"] > sp0.eps_th)
    t = sp0.time(k_fire)
    hq = m["h"](t) * m["qnorm"]
    V = sp0.snapshot_np(k_fire)
    nu2 = float(np.sum(O.weight_tensor(sp0.weights) * V * V))
    # budget at twice (below: the ranks stay) or half (above: they grow) of h^2
    B = 2.0 * hq * hq if side == "below" else 0.5 * hq * hq
    gamma = 100.0 * (1.0 - B / nu2)
    cfg = O.OracleConfig(dims=sp0.dims, weights=sp0.weights, dt=sp0.dt, rank_max=sp0.rank_max,
                         rank_init=sp0.rank_init, adaptive=True, eps_th=sp0.eps_th, gamma_th=gamma)
    o = O.OracleTDB(cfg).init(sp0.snapshot_np(0))
    for k in range(1, k_fire):
        rec = o.ingest(sp0.snapshot_np(k))
        assert rec.event == ""
    rec = o.ingest(V)
    assert rec.eps == pytest.approx(hq, rel=1e-8)
    if side == "below":
        assert rec.event == "reinit" and rec.ranks == (3, 3, 3)
        assert rec.eps_after == pytest.approx(hq, rel=1e-8)
        # the target is out of reach at these ranks: the trigger rises to 2 eps_re
        assert o.unmet and o.eps_trig == pytest.approx(2.0 * hq, rel=1e-8)
    else:
        assert rec.event == "add" and rec.ranks == (4, 4, 4)
        assert rec.eps_after <= 1e-10


# ------------------------------------------------------------------ set_threshold
def test_set_threshold_mid_run_moves_the_add():
    """Raising eps_th before the crossing (Sec. 2.5: the threshold is the user's
    knob) moves the add to the first step whose closed-form error h(t) exceeds the
    new threshold; lowering it makes the very next step fire.

    Caught mistake: set_threshold not moving the trigger (the add fires at the old
    threshold)."""
    sp = switched_term_spec(steps=80)
    m = sp.meta
    hq = lambda k: m["h"](sp.time(k)) * m["qnorm"]   # noqa: E731
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th)
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    k_set = 10
    new_th = 5.0 * sp.eps_th
    expected = next(k for k in range(k_set + 1, sp.steps + 1) if hq(k) > new_th)
    assert hq(expected - 1) > sp.eps_th      # the old threshold would have fired earlier
    fired = None
    for k in range(1, sp.steps + 1):
        if k == k_set + 1:
            o.set_threshold(new_th)
        rec = o.ingest(sp.snapshot_np(k))
        if rec.event and fired is None:
            fired = k
            break
    assert fired == expected
    # lowering it below the current error fires at the next step
    o2 = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    for k in range(1, 20):
        o2.ingest(sp.snapshot_np(k))
    k_low = next(k for k in range(20, sp.steps + 1) if hq(k) > 0)
    o2.set_threshold(0.5 * hq(k_low))
    rec = o2.ingest(sp.snapshot_np(k_low))
    assert rec.event in ("add", "reinit")


# ------------------------------------------------------------------ replay mode
def _run(sp, cfg, forces=None, upto=None):
    o = O.OracleTDB(cfg).init(sp.snapshot_np(0))
    recs = []
    for k in range(1, (upto or sp.steps) + 1):
        f = None if forces is None else forces.get(k)
        recs.append(o.ingest(sp.snapshot_np(k), force=f))
    return o, recs


def test_replay_of_natural_decisions_reproduces_the_run():
    """Replay mode adopting at every step the decision the controller itself took
    must give the same run bit for bit (it only skips the comparisons)."""
    sp = switched_term_spec(steps=70)
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th)
    o1, r1 = _run(sp, cfg)
    assert any(r.event for r in r1)
    forces = {k + 1: r.event for k, r in enumerate(r1)}
    o2, r2 = _run(sp, cfg, forces)
    assert [r.event for r in r1] == [r.event for r in r2]
    assert [r.ranks for r in r1] == [r.ranks for r in r2]
    assert np.array_equal(o1.C, o2.C)
    for a, b in zip(o1.U, o2.U):
        assert np.array_equal(a, b)


def test_replay_forced_decisions_closed_form():
    """Forced decisions on the switched stream, checked against the closed-form error:
    no event at the natural add step keeps the evolved state (the tracked error stays
    h(t)); a forced reinit before the crossing keeps the ranks and leaves exactly
    h(t); a forced removal after the term has decayed returns to rank 3 with error
    h(t).

    Caught mistakes: replay ignoring '' (the add still fires); a forced reinit that
    also grows ranks; a forced removal that keeps the ranks."""
    sp = switched_term_spec(steps=60)
    m = sp.meta
    hq = lambda k: m["h"](sp.time(k)) * m["qnorm"]   # noqa: E731
    cfg = O.OracleConfig(dims=sp.dims, weights=sp.weights, dt=sp.dt, rank_max=sp.rank_max,
                         rank_init=sp.rank_init, adaptive=True, eps_th=sp.eps_th)
    k_fire = next(k for k in range(1, sp.steps + 1) if hq(k) > sp.eps_th)
    # '' at the natural add step and the two after it: no event, error still h(t)
    _, recs = _run(sp, cfg, {k_fire: "", k_fire + 1: "", k_fire + 2: ""}, upto=k_fire + 2)
    for k in (k_fire, k_fire + 1, k_fire + 2):
        assert recs[k - 1].event == ""
        assert recs[k - 1].ranks == (3, 3, 3)
        assert recs[k - 1].eps == pytest.approx(hq(k), abs=1e-10)
    # a forced reinit before the crossing (h > 0 but below eps_th)
    k_re = next(k for k in range(1, k_fire) if hq(k) > 0)
    _, recs = _run(sp, cfg, {k_re: "reinit"}, upto=k_re)
    assert recs[-1].event == "reinit" and recs[-1].ranks == (3, 3, 3)
    assert recs[-1].eps_after == pytest.approx(hq(k_re), rel=1e-8)
    # forced removal once the extra term is gone again
    prof = lambda t: 0.3 if 0.05 < t < 0.1 else 1e-4   # noqa: E731
    sp2 = switched_term_spec(steps=40, profile=prof)
    cfg2 = O.OracleConfig(dims=sp2.dims, weights=sp2.weights, dt=sp2.dt, rank_max=sp2.rank_max,
                          rank_init=sp2.rank_init, adaptive=True, eps_th=sp2.eps_th)
    o, recs = _run(sp2, cfg2, upto=25)
    assert o.ranks == (4, 4, 4)
    rec = o.ingest(sp2.snapshot_np(26), force="remove")
    assert rec.event == "remove" and rec.ranks == (3, 3, 3)
    # eps_after^2 = nu^2 - ||C||^2 cancels about 1e-15 nu^2, i.e. 1e-7 of eps^2 here
    assert rec.eps_after == pytest.approx(1e-4 * sp2.meta["qnorm"], rel=1e-5)
