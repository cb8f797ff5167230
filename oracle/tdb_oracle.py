"""Plain FP64 CPU oracle of the time-dependent-basis (TDB) in situ compressor.

TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module. The product path (the HIP
library and its Python binding) never calls it, and shares no code with it.

Everything here follows the paper's methodology section, in its order and
notation, written out in float64 numpy with no blocking or fusion:

* weighted inner products with diagonal quadrature weights (eq. (inner) and the
  discrete form in Sec. 2.3), a mode-n unfolding and n-mode products (Sec. 2.1,
  Kolda-Bader convention);
* the Tucker-form TDB ansatz (eq. (reconstructed));
* the evolution equations with the skew gauge phi = 0: the core derivative
  eq. (Corecont) and the basis derivative eq. (basecont), i.e. the complement
  projection of the partial projection of the data derivative, times the
  least-squares pseudo-inverse of the core unfolding (Sec. 2.2);
* a finite-difference data derivative and an explicit Runge-Kutta integrator
  (Sec. 2.3), with HOSVD initialisation and reinitialisation (Sec. 2.3, 2.5);
* the reconstruction error eq. (error) and captured energy eq. (percentage)
  driving mode addition and removal (Sec. 2.5);
* the compression ratio CR and the time-weighted ratio (Sec. 2.6).

Readings taken where the paper is silent or ambiguous (each one is listed in the
design notes): Heun's method as the second-order Runge-Kutta scheme, one
first-order difference quotient used by both stages, a W-orthonormal QR after
every full step with R folded into the core, density-normalised weights, a sign
convention for HOSVD vectors, and a deterministic add/remove controller written
from the prose of Sec. 2.5.

Parity status: every function here is pinned by a `-m "not gpu"` test against a
closed form, a brute-force construction or a printed value; the controller's
rank choice on noisy data beyond those pins is "parity unpinned" (the paper's
curves are not available).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


class NumericalEvent(Exception):
    """The core-unfolding Gram matrix is singular or too ill-conditioned to invert."""


# ----------------------------------------------------------------- tensor algebra
def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding X_(n) (Sec. 2.1): rows indexed by mode n, columns by the
    remaining indices with the first remaining index varying fastest."""
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def fold(M: np.ndarray, n: int, shape: Sequence[int]) -> np.ndarray:
    """Inverse of `unfold` for a tensor of the given shape."""
    rest = [shape[k] for k in range(len(shape)) if k != n]
    return np.moveaxis(np.reshape(M, [shape[n]] + rest, order="F"), 0, n)


def mode_product(X: np.ndarray, M: np.ndarray, n: int) -> np.ndarray:
    """n-mode product X x_n M (Sec. 2.1), with M of shape (J, N_n)."""
    return np.moveaxis(np.tensordot(M, X, axes=([1], [n])), 0, n)


def weight_tensor(w: Sequence[np.ndarray]) -> np.ndarray:
    """Outer product of the per-mode quadrature weights (diagonal W, Sec. 2.3)."""
    out = np.asarray(w[0], dtype=np.float64)
    for wn in w[1:]:
        out = np.multiply.outer(out, wn)
    return out


def weighted_norm2(X: np.ndarray, w: Sequence[np.ndarray]) -> float:
    """||X||^2 in the weighted inner product of eq. (inner), discretised."""
    return float(np.sum(weight_tensor(w) * X * X))


def reconstruct(C: np.ndarray, U: Sequence[np.ndarray]) -> np.ndarray:
    """TDB reconstruction of eq. (reconstructed): C x_1 U_1 x_2 ... x_p U_p."""
    out = C
    for n, Un in enumerate(U):
        out = mode_product(out, Un, n)
    return out


def projector_T(Un: np.ndarray, wn: np.ndarray) -> np.ndarray:
    """U_n^T W_n: the discrete form of the inner product with each basis vector."""
    return Un.T * wn[None, :]


# ----------------------------------------------------------------- evolution
def core_pinv(C: np.ndarray, n: int, cond_limit: float = 1e-12):
    """Pseudo-inverse of the mode-n core unfolding, C_(n)^T (C_(n) C_(n)^T)^-1
    (least-squares solution, Sec. 2.2). Solved with a Cholesky factorisation of
    the Gram matrix; raises NumericalEvent if it is singular or its eigenvalue
    ratio falls below `cond_limit`."""
    Cn = unfold(C, n)
    G = Cn @ Cn.T
    lam = np.linalg.eigvalsh(G)
    if not np.all(np.isfinite(lam)) or lam[-1] <= 0.0 or lam[0] / lam[-1] < cond_limit:
        raise NumericalEvent(f"mode {n}: core Gram eigenvalue ratio {lam[0] / max(lam[-1], 1e-300):.3e}")
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError as exc:  # pragma: no cover - guarded by the ratio test
        raise NumericalEvent(str(exc))
    Y = np.linalg.solve(L.T, np.linalg.solve(L, Cn))      # G^-1 C_(n)
    return Y.T


def partial_projection(D: np.ndarray, U: Sequence[np.ndarray], w: Sequence[np.ndarray], n: int):
    """F_n = D x_{k != n} (U_k^T W_k): the inner product of the data derivative
    with every basis except mode n (eq. (basecont), the <v_dot, prod u>_{x \\ x_n} term)."""
    F = D
    for k in range(D.ndim):
        if k != n:
            F = mode_product(F, projector_T(U[k], w[k]), k)
    return F


def rhs(C: np.ndarray, U: Sequence[np.ndarray], w: Sequence[np.ndarray], D: np.ndarray):
    """Right-hand side of the TDB evolution for a data derivative D.

    Core: eq. (Corecont), C_dot = D x_1 (U_1^T W_1) ... x_p (U_p^T W_p).
    Bases: eq. (basecont), U_dot_n = (I - U_n U_n^T W_n) F_n(n) C_(n)^dagger.
    """
    p = D.ndim
    Cdot = D
    for k in range(p):
        Cdot = mode_product(Cdot, projector_T(U[k], w[k]), k)
    Udot = []
    for n in range(p):
        if U[n].shape[1] == U[n].shape[0]:
            # a full-rank mode: the complement of span(U_n) is empty, U_dot_n = 0
            Udot.append(np.zeros_like(U[n]))
            continue
        Fn = unfold(partial_projection(D, U, w, n), n)
        comp = Fn - U[n] @ (projector_T(U[n], w[n]) @ Fn)   # orthogonal-complement projection
        Udot.append(comp @ core_pinv(C, n))
    return Cdot, Udot


def heun_step(C, U, w, D, dt, D2=None):
    """Explicit second-order Runge-Kutta step (Heun / trapezoid): stage 1 at t_k with
    the data derivative D, stage 2 at t_{k+1} with D2 (D held over both stages when
    D2 is None)."""
    k1C, k1U = rhs(C, U, w, D)
    Cs = C + dt * k1C
    Us = [Un + dt * kU for Un, kU in zip(U, k1U)]
    k2C, k2U = rhs(Cs, Us, w, D if D2 is None else D2)
    C1 = C + 0.5 * dt * (k1C + k2C)
    U1 = [Un + 0.5 * dt * (a + b) for Un, a, b in zip(U, k1U, k2U)]
    return C1, U1


def fd2_stage_derivatives(V_m1, V_0, V_1, dt):
    """Second-order finite differences of the data at the two Heun stage times from
    the snapshots at t_{k-1}, t_k, t_{k+1} (Sec. 2.3 names first-order and central
    differences; this reading takes the central difference at t_k for stage 1 and the
    one-sided second-order difference at t_{k+1} for stage 2):
        D(t_k)     ~ (V_1 - V_m1) / (2 dt)
        D(t_{k+1}) ~ (3 V_1 - 4 V_0 + V_m1) / (2 dt)
    Both are exact for data quadratic in t."""
    return (V_1 - V_m1) / (2.0 * dt), (3.0 * V_1 - 4.0 * V_0 + V_m1) / (2.0 * dt)


def euler_step(C, U, w, D, dt):
    """Explicit first-order Euler step."""
    kC, kU = rhs(C, U, w, D)
    return C + dt * kC, [Un + dt * k for Un, k in zip(U, kU)]


def reorthonormalize(C, U, w):
    """Restore U_n^T W_n U_n = I (eq. (orhonormality)) without changing the
    reconstruction: W^(1/2) U_n = Q_n R_n with diag(R_n) > 0 (Householder QR),
    U_n <- W^(-1/2) Q_n and C <- C x_n R_n."""
    U_out = []
    for n, (Un, wn) in enumerate(zip(U, w)):
        s = np.sqrt(wn)[:, None]
        Q, R = np.linalg.qr(s * Un)
        sg = np.sign(np.diag(R))
        sg[sg == 0] = 1.0
        Q = Q * sg[None, :]
        R = R * sg[:, None]
        U_out.append(Q / s)
        C = mode_product(C, R, n)
    return C, U_out


# ----------------------------------------------------------------- diagnostics
def error_and_norm(V, C, U, w):
    """eps = ||V - V_TDB||_W (eq. (error), weighted Frobenius) and nu = ||V||_W."""
    Wt = weight_tensor(w)
    E = V - reconstruct(C, U)
    return math.sqrt(float(np.sum(Wt * E * E))), math.sqrt(float(np.sum(Wt * V * V)))


def core_singular_values(C: np.ndarray) -> List[np.ndarray]:
    """Singular values of every core unfolding C_(n) (Sec. 2.4), descending."""
    out = []
    for n in range(C.ndim):
        Cn = unfold(C, n)
        lam = np.linalg.eigvalsh(Cn @ Cn.T)[::-1]
        out.append(np.sqrt(np.maximum(lam, 0.0)))
    return out


def core_rotation(C: np.ndarray, U: Sequence[np.ndarray]):
    """Energetic rotation of eq. (rot): U_n <- U_n Psi_n, C <- C x_n Psi_n^T, with
    Psi_n the descending left singular vectors of C_(n); each column of Psi_n is
    sign-fixed so that its largest-magnitude entry is positive."""
    Uo, Co = [], C
    for n in range(C.ndim):
        Cn = unfold(C, n)
        lam, Psi = np.linalg.eigh(Cn @ Cn.T)
        Psi = sign_fix(Psi[:, ::-1])
        Uo.append(U[n] @ Psi)
        Co = mode_product(Co, Psi.T, n)
    return Co, Uo


def sign_fix(Q: np.ndarray) -> np.ndarray:
    """Make each column's largest-|entry| positive (lowest index on a tie)."""
    Q = Q.copy()
    for j in range(Q.shape[1]):
        i = int(np.argmax(np.abs(Q[:, j])))
        if Q[i, j] < 0:
            Q[:, j] = -Q[:, j]
    return Q


def compression_ratio(dims: Sequence[int], ranks: Sequence[int]) -> float:
    """CR = prod N_n / (sum r_n N_n + prod r_n) (Sec. 2.6)."""
    return float(np.prod(dims)) / (sum(r * n for r, n in zip(ranks, dims)) + float(np.prod(ranks)))


def weighted_compression_ratio(times: Sequence[float], crs: Sequence[float]) -> float:
    """Time-weighted harmonic mean of the CRs over intervals (Sec. 2.6):
    (t_m - t_0) / sum_i (t_i - t_{i-1}) / CR_i, with `crs[i]` charged to
    the interval (times[i], times[i+1])."""
    span = times[-1] - times[0]
    den = sum((times[i + 1] - times[i]) / crs[i] for i in range(len(times) - 1))
    return span / den


# ----------------------------------------------------------------- HOSVD
@dataclass
class Hosvd:
    """Truncated HOSVD of a snapshot at the rank caps (Sec. 2.3, 2.4)."""

    sigma: List[np.ndarray]      # full singular values of each weighted unfolding, descending
    U: List[np.ndarray]          # N_n x cap_n bases (W-orthonormal), sign-fixed
    C: np.ndarray                # cap_1 x ... x cap_p core, the projection onto the bases
    nu2: float                   # ||V||_W^2

    def truncation_error2(self, ranks) -> float:
        """Exact squared error of the rank-`ranks` truncation: nu^2 - ||C[:r]||^2."""
        sub = self.C[tuple(slice(0, r) for r in ranks)]
        return max(self.nu2 - float(np.sum(sub * sub)), 0.0)

    def truncate(self, ranks):
        C = self.C[tuple(slice(0, r) for r in ranks)].copy()
        U = [Un[:, :r].copy() for Un, r in zip(self.U, ranks)]
        return C, U


def hosvd(V: np.ndarray, w: Sequence[np.ndarray], caps: Sequence[int]) -> Hosvd:
    """HOSVD in the weighted inner product: eigen-decompose the Gram matrix of each
    scaled unfolding (V scaled by the square roots of the weights), keep the
    leading `caps` eigenvectors, then project V onto them."""
    p = V.ndim
    s = [np.sqrt(wn) for wn in w]
    Vt = V * weight_tensor(s)
    sig, Ut = [], []
    for n in range(p):
        Vn = unfold(Vt, n)
        lam, Q = np.linalg.eigh(Vn @ Vn.T)
        lam, Q = lam[::-1], Q[:, ::-1]
        sig.append(np.sqrt(np.maximum(lam, 0.0)))
        Ut.append(sign_fix(Q[:, : caps[n]]))
    Cmax = Vt
    for n in range(p):
        Cmax = mode_product(Cmax, Ut[n].T, n)
    U = [Q / sn[:, None] for Q, sn in zip(Ut, s)]
    return Hosvd(sig, U, Cmax, float(np.sum(Vt * Vt)))


# ----------------------------------------------------------------- controller
@dataclass
class OracleConfig:
    dims: tuple
    weights: List[np.ndarray]
    dt: float
    rank_max: tuple
    rank_init: Optional[tuple] = None
    adaptive: bool = True
    eps_th: float = 1e-4
    gamma_th: float = 0.0           # > 0: paper-style percentage budget
    slope_window: int = 10
    integrator: str = "heun"        # 'heun' or 'euler'
    fd_order: int = 1               # 1: (V_{k+1} - V_k)/dt over both stages; 2: fd2_stage_derivatives

    def caps(self):
        """Rank caps clamped to the mode sizes and to the product of the other caps."""
        c = [min(int(r), int(n)) for r, n in zip(self.rank_max, self.dims)]
        for n in range(len(c)):
            others = int(np.prod([c[k] for k in range(len(c)) if k != n]))
            c[n] = min(c[n], others)
        return tuple(c)


def _valid(r):
    return all(r[n] <= int(np.prod([r[k] for k in range(len(r)) if k != n])) for n in range(len(r)))


# A direction whose full-data singular value is below this fraction of the mode's
# largest one is numerically absent: adding it would make the core Gram matrix
# singular (eigenvalue ratio below the 1e-12 limit of `core_pinv`).
SIGMA_FLOOR = 1e-6


def _next_sigma(h: Hosvd, r, n) -> float:
    return h.sigma[n][r[n]] if r[n] < len(h.sigma[n]) else -1.0


def _can_grow(h: Hosvd, caps, r, n) -> bool:
    return r[n] < caps[n] and _next_sigma(h, r, n) > SIGMA_FLOOR * h.sigma[n][0]


def numerical_ranks(h: Hosvd, caps) -> tuple:
    """Per mode, the number of singular values above SIGMA_FLOOR * sigma_1, capped."""
    return tuple(max(1, min(int(c), int(np.sum(sg > SIGMA_FLOOR * sg[0])))) for sg, c in zip(h.sigma, caps))


def repair_ranks(h: Hosvd, caps, r) -> tuple:
    """Grow modes until every r_n <= prod_{k != n} r_k (otherwise the core Gram of
    mode n is singular: the least-squares system of Sec. 2.2 is underdetermined).
    The mode grown is the one, other than the offending mode, with the largest next
    full-data singular value (lowest mode on a tie)."""
    r = list(r)
    p = len(r)
    while not _valid(r):
        bad = next(n for n in range(p) if r[n] > int(np.prod([r[k] for k in range(p) if k != n])))
        cand = [m for m in range(p) if m != bad and _can_grow(h, caps, r, m)]
        if not cand:
            r[bad] = int(np.prod([r[k] for k in range(p) if k != bad]))
            continue
        best = max(cand, key=lambda m: (_next_sigma(h, r, m), -m))
        r[best] += 1
    return tuple(r)


def rank_rule(h: Hosvd, caps, budget2: float, start) -> tuple:
    """Greedy rank choice from the captured-energy relation eq. (percentage).

    Starting from `start`, while the exact truncation error exceeds the budget,
    grow the mode whose next full-data singular value is largest (lowest mode on a
    tie); then repair validity with `repair_ranks`."""
    r = [min(int(a), int(c)) for a, c in zip(start, caps)]
    p = len(r)
    while h.truncation_error2(r) > budget2:
        cand = [n for n in range(p) if _can_grow(h, caps, r, n)]
        if not cand:
            break
        best = max(cand, key=lambda n: (_next_sigma(h, r, n), -n))
        r[best] += 1
    return repair_ranks(h, caps, r)


@dataclass
class StepRecord:
    k: int
    t: float
    eps: float                    # exact error of the evolved state at t_k
    nu: float
    ranks: tuple                  # ranks held after the step (after any event)
    event: str = ""               # '', 'add', 'reinit', 'remove', 'numeric'
    eps_after: float = float("nan")
    sigma: List[np.ndarray] = field(default_factory=list)
    cr: float = 0.0


class OracleTDB:
    """Step-by-step FP64 reference of the streaming compressor."""

    def __init__(self, cfg: OracleConfig):
        self.cfg = cfg
        self.w = [np.asarray(wn, dtype=np.float64) for wn in cfg.weights]
        self.caps = cfg.caps()
        self.C = None
        self.U = None
        self.V_prev = None
        self.k = 0
        self.t = 0.0
        self.records: List[StepRecord] = []
        self.window: List[float] = []
        self.unmet = False
        self.eps_trig = cfg.eps_th
        self.eps_th = cfg.eps_th
        self.gamma_th = cfg.gamma_th

    # -- budget of the rank rule: (eps_th/2)^2, or the paper's percentage form
    def budget2(self, nu2: float) -> float:
        if self.gamma_th > 0.0:
            return (1.0 - self.gamma_th / 100.0) * nu2
        return (0.5 * self.eps_th) ** 2

    def set_threshold(self, eps_th: float, gamma_th: float = 0.0):
        self.eps_th = eps_th
        self.gamma_th = gamma_th
        if not self.unmet:
            self.eps_trig = eps_th

    def _clamp_ranks(self, r):
        r = [max(1, min(int(a), int(c))) for a, c in zip(r, self.caps)]
        guard = 0
        while not _valid(r) and guard < 10000:
            guard += 1
            n = next(n for n in range(len(r)) if r[n] > int(np.prod([r[k] for k in range(len(r)) if k != n])))
            r[n] -= 1
        return tuple(r)

    # -- initialisation (Sec. 2.3: HOSVD of the first snapshot)
    def init(self, V0: np.ndarray, t0: float = 0.0):
        V0 = np.asarray(V0, dtype=np.float64)
        h = hosvd(V0, self.w, self.caps)
        if self.cfg.rank_init is not None:
            r = self._clamp_ranks(self.cfg.rank_init)
        else:
            r = rank_rule(h, self.caps, self.budget2(h.nu2), [1] * V0.ndim)
        self.C, self.U = h.truncate(r)
        self.V_prev = V0.copy()
        self.V_prev2 = None
        self.t = t0
        self.k = 0
        eps0 = math.sqrt(h.truncation_error2(r))
        self.records = [StepRecord(0, t0, eps0, math.sqrt(h.nu2), tuple(r),
                                   sigma=core_singular_values(self.C),
                                   cr=compression_ratio(self.cfg.dims, r))]
        self.window = []
        return self

    def init_from_factors(self, V0, C, U, t0: float = 0.0):
        self.C = np.array(C, dtype=np.float64)
        self.U = [np.array(u, dtype=np.float64) for u in U]
        self.V_prev = np.asarray(V0, dtype=np.float64).copy()
        self.V_prev2 = None
        self.t = t0
        self.k = 0
        eps0, nu0 = error_and_norm(self.V_prev, self.C, self.U, self.w)
        self.records = [StepRecord(0, t0, eps0, nu0, tuple(self.C.shape),
                                   sigma=core_singular_values(self.C),
                                   cr=compression_ratio(self.cfg.dims, self.C.shape))]
        self.window = []
        return self

    @property
    def ranks(self):
        return tuple(self.C.shape)

    def _reinit(self, h: Hosvd, r):
        self.C, self.U = h.truncate(r)
        return math.sqrt(h.truncation_error2(r))

    # -- one snapshot
    def ingest(self, V_new: np.ndarray, D: Optional[np.ndarray] = None, force: Optional[str] = None):
        """Advance the state from t_k to t_{k+1} with snapshot V_{k+1}.

        D defaults to the first-order difference (V_{k+1} - V_k)/dt (Sec. 2.3), or with
        fd_order 2 (from the second step on) to the stage derivatives of
        fd2_stage_derivatives; a given D is held over both stages, a given pair
        (D1, D2) gives the two stages' derivatives.
        `force` (replay mode) overrides the controller's decision with the one a
        device run took: '', 'add', 'reinit', 'remove'."""
        cfg = self.cfg
        V_new = np.asarray(V_new, dtype=np.float64)
        dt = cfg.dt
        D2 = None
        if isinstance(D, tuple):
            D, D2 = D
        elif D is None:
            if cfg.fd_order == 2 and getattr(self, "V_prev2", None) is not None:
                D, D2 = fd2_stage_derivatives(self.V_prev2, self.V_prev, V_new, dt)
            else:
                D = (V_new - self.V_prev) / dt
        numeric = False
        try:
            if cfg.integrator == "euler":
                C1, U1 = euler_step(self.C, self.U, self.w, D, dt)
            else:
                C1, U1 = heun_step(self.C, self.U, self.w, D, dt, D2)
            self.C, self.U = reorthonormalize(C1, U1, self.w)
        except NumericalEvent:
            numeric = True
        self.k += 1
        self.t += dt
        eps, nu = error_and_norm(V_new, self.C, self.U, self.w)
        rec = StepRecord(self.k, self.t, eps, nu, self.ranks)
        if cfg.adaptive or numeric or force is not None:
            self._control(V_new, rec, numeric, force)
        rec.ranks = self.ranks
        rec.sigma = core_singular_values(self.C)
        rec.cr = compression_ratio(cfg.dims, rec.ranks)
        self.records.append(rec)
        self.V_prev2 = self.V_prev
        self.V_prev = V_new.copy()
        return rec

    def _control(self, V, rec: StepRecord, numeric: bool, force: Optional[str]):
        """Mode addition / removal and HOSVD reinitialisation (Sec. 2.5)."""
        eps = rec.eps
        nu2 = rec.nu ** 2
        B = self.budget2(nu2)
        if numeric and force is None:
            # the core lost rank: restart from the snapshot at ranks no larger than
            # the current ones nor than the data's numerical rank
            h = hosvd(V, self.w, self.caps)
            nr = numerical_ranks(h, self.caps)
            cap_r = [min(a, b) for a, b in zip(self.ranks, nr)]
            if self.cfg.adaptive:
                r_rule = rank_rule(h, self.caps, B, [1] * len(self.caps))
                cap_r = [min(a, b) for a, b in zip(cap_r, r_rule)]
            r_new = repair_ranks(h, self.caps, cap_r)
            rec.eps_after = self._reinit(h, r_new)
            rec.event = "numeric"
            self._after_reinit(rec.eps_after)
            return
        want_add = eps > self.eps_trig
        if force is not None:
            want_add = force in ("add", "reinit")
        if want_add:
            h = hosvd(V, self.w, self.caps)
            r = self.ranks
            eps_re = self._reinit(h, r)
            rec.event = "reinit"
            if eps_re > self.eps_th and force != "reinit":
                r2 = rank_rule(h, self.caps, B, r)
                if r2 != tuple(r):
                    eps_re = self._reinit(h, r2)
                    rec.event = "add"
            rec.eps_after = eps_re
            self._after_reinit(eps_re)
            return
        # removal test: negative average error slope over the window, headroom,
        # and a mode whose weakest direction fits inside the budget
        self.window.append(eps)
        if force is None and not self._removal_ready(eps, B):
            return
        if force is not None and force != "remove":
            return
        h = hosvd(V, self.w, self.caps)
        r_rule = rank_rule(h, self.caps, B, [1] * len(self.caps))
        r_new = repair_ranks(h, self.caps, [min(a, b) for a, b in zip(self.ranks, r_rule)])
        if r_new == self.ranks and force != "remove":
            self.window = []
            return
        rec.eps_after = self._reinit(h, r_new)
        rec.event = "remove"
        self._after_reinit(rec.eps_after)

    def _after_reinit(self, eps_re: float):
        """Reset the slope window; enter or leave the 'unmet' state in which the
        trigger is raised to twice the best error reachable at the caps."""
        self.window = []
        if eps_re > self.eps_th:
            self.unmet = True
            self.eps_trig = 2.0 * eps_re
        else:
            self.unmet = False
            self.eps_trig = self.eps_th

    def _removal_ready(self, eps, B) -> bool:
        nw = self.cfg.slope_window
        if len(self.window) < nw:
            return False
        slope = (self.window[-1] - self.window[-nw]) / ((nw - 1) * self.cfg.dt)
        if not slope < 0.0:
            return False
        if eps > 0.5 * self.eps_th:
            return False
        sig = core_singular_values(self.C)
        return any(eps * eps + sig[n][self.ranks[n] - 1] ** 2 <= B for n in range(self.C.ndim))

    def reconstruct(self):
        return reconstruct(self.C, self.U)

    def weighted_cr(self):
        times = [r.t for r in self.records]
        crs = [r.cr for r in self.records[1:]]
        if len(times) < 2:
            return self.records[0].cr
        return weighted_compression_ratio(times, crs)
