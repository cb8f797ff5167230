"""Closed-form synthetic streams with the shapes and structure of the paper's workloads.

The paper's own datasets (reactive-flow DNS, stochastic DNS ensemble, turbulent
channel) are not available, so each generator below is a seeded stand-in with the
same tensor shape, value range and spectral structure (see the workload recipes in
the design notes). A generator evaluates a field on its grid at time
``t = t0 + k*dt``; it never touches the compression method itself.

All evaluation goes through torch so that one definition runs on the host (float64,
for the oracle and for parity inputs) and on the device (for large benchmark
inputs). Parameters that are drawn at random are drawn on the host with numpy's
PCG64 from a stated seed; per-element noise uses a counter-based hash so host and
device produce identical integer streams.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

_M32 = 0xFFFFFFFF


# --------------------------------------------------------------------------- noise
def _mul32(x: torch.Tensor, c: int) -> torch.Tensor:
    """(x * c) mod 2**32 for int64 tensors holding values in [0, 2**32), without
    signed overflow: the multiplication is split into 16-bit halves."""
    lo = x & 0xFFFF
    hi = x >> 16
    return ((lo * c) + (((hi * c) & 0xFFFF) << 16)) & _M32


def _hash32(x: torch.Tensor) -> torch.Tensor:
    """A 32-bit integer finaliser (xorshift-multiply, 'lowbias32' constants)."""
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def counter_normal(n: int, seed: int, device="cpu") -> torch.Tensor:
    """n standard normal float64 draws, a pure function of (seed, index).

    Box-Muller on two hashed 32-bit counters; identical on every device because
    only integer ops feed the final float transform.
    """
    idx = torch.arange(n, dtype=torch.int64, device=device)
    key = _hash32(torch.tensor([seed & _M32], dtype=torch.int64, device=device) ^ 0x9E3779B9)
    h1 = _hash32(((2 * idx) & _M32) ^ key)
    h2 = _hash32(((2 * idx + 1) & _M32) ^ key)
    u1 = (h1.to(torch.float64) + 1.0) / 4294967296.0      # (0, 1]
    u2 = h2.to(torch.float64) / 4294967296.0              # [0, 1)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


# --------------------------------------------------------------------------- spec
@dataclass
class StreamSpec:
    """One streaming tensor: grid, quadrature weights, time grid and a field."""

    name: str
    dims: tuple
    weights: List[np.ndarray]
    dt: float
    steps: int
    field_fn: Callable[[float, str, torch.dtype], torch.Tensor]
    t0: float = 0.0
    storage: str = "f32"                       # 'f32' or 'f64' snapshot storage
    deriv_fn: Optional[Callable[[float, str, torch.dtype], torch.Tensor]] = None
    eps_th: float = 0.0
    gamma_th: float = 0.0
    rank_init: Optional[Sequence[int]] = None
    rank_max: Optional[Sequence[int]] = None
    adaptive: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def order(self) -> int:
        return len(self.dims)

    @property
    def size(self) -> int:
        return int(np.prod(self.dims))

    def time(self, k: int) -> float:
        return self.t0 + k * self.dt

    @property
    def np_storage(self):
        return np.float32 if self.storage == "f32" else np.float64

    @property
    def torch_storage(self):
        return torch.float32 if self.storage == "f32" else torch.float64

    def snapshot(self, k: int, device="cpu") -> torch.Tensor:
        """Snapshot k rounded once to the storage dtype (evaluated in float64)."""
        v = self.field_fn(self.time(k), device, torch.float64)
        return v.to(self.torch_storage).contiguous()

    def snapshot_np(self, k: int) -> np.ndarray:
        return self.snapshot(k, "cpu").numpy()

    def derivative_np(self, k: int) -> np.ndarray:
        if self.deriv_fn is None:
            raise ValueError(f"stream {self.name} has no closed-form derivative")
        return self.deriv_fn(self.time(k), "cpu", torch.float64).numpy()


def _uniform_weights(dims):
    return [np.full(n, 1.0 / n) for n in dims]


# --------------------------------------------------------------------------- C1
def analytic_cp5_spec(n: int = 64, steps: int = 200, dt: float = 1e-3) -> StreamSpec:
    """Plain single-stream case: a sum of five separable terms on [0,1]^3.

    V(x,y,z,t) = sum_k a_k(t) sin(k pi x + 0.3 t) cos(k pi y - 0.2 t) sin(k pi z + 0.1 k t),
    a_k(t) = exp(-k/2) (1 + 0.2 sin(2 pi k t)). Multilinear rank exactly (5,5,5).
    """
    x = torch.linspace(0.0, 1.0, n, dtype=torch.float64)

    def fld(t, device, dtype):
        xs = x.to(device)
        out = torch.zeros((n, n, n), dtype=torch.float64, device=device)
        for k in range(1, 6):
            a = math.exp(-0.5 * k) * (1.0 + 0.2 * math.sin(2.0 * math.pi * k * t))
            fx = torch.sin(k * math.pi * xs + 0.3 * t)
            fy = torch.cos(k * math.pi * xs - 0.2 * t)
            fz = torch.sin(k * math.pi * xs + 0.1 * k * t)
            out += a * fx[:, None, None] * fy[None, :, None] * fz[None, None, :]
        return out.to(dtype)

    def dfld(t, device, dtype):
        xs = x.to(device)
        out = torch.zeros((n, n, n), dtype=torch.float64, device=device)
        for k in range(1, 6):
            e = math.exp(-0.5 * k)
            a = e * (1.0 + 0.2 * math.sin(2.0 * math.pi * k * t))
            da = e * 0.2 * 2.0 * math.pi * k * math.cos(2.0 * math.pi * k * t)
            fx = torch.sin(k * math.pi * xs + 0.3 * t)
            fy = torch.cos(k * math.pi * xs - 0.2 * t)
            fz = torch.sin(k * math.pi * xs + 0.1 * k * t)
            dfx = 0.3 * torch.cos(k * math.pi * xs + 0.3 * t)
            dfy = 0.2 * torch.sin(k * math.pi * xs - 0.2 * t)
            dfz = 0.1 * k * torch.cos(k * math.pi * xs + 0.1 * k * t)
            out += da * fx[:, None, None] * fy[None, :, None] * fz[None, None, :]
            out += a * dfx[:, None, None] * fy[None, :, None] * fz[None, None, :]
            out += a * fx[:, None, None] * dfy[None, :, None] * fz[None, None, :]
            out += a * fx[:, None, None] * fy[None, :, None] * dfz[None, None, :]
        return out.to(dtype)

    return StreamSpec(
        name=f"analytic-cp5-{n}^3", dims=(n, n, n), weights=_uniform_weights((n, n, n)),
        dt=dt, steps=steps, field_fn=fld, deriv_fn=dfld, storage="f64",
        rank_init=(5, 5, 5), rank_max=(5, 5, 5), adaptive=False, eps_th=1.0)


# --------------------------------------------------------------------------- C2
_PLUME_C0 = ((0.5, 0.30), (0.9, 0.65), (1.3, 0.45))
_PLUME_S = (0.10, 0.08, 0.12)
_PLUME_R = (0.05, 0.04, 0.06)


def plume_spec(nx: int = 512, ny: int = 256, nv: int = 8, steps: int = 1000,
               dt: float = 5e-4, noise: float = 1e-6, noise_seed: int = 2,
               centre_shift=(0.0, 0.0), width_scale: float = 1.0, growth: float = 2.0) -> StreamSpec:
    """Reactive-flow-shaped stream: 3 advected Gaussian plumes with tanh reaction
    fronts and Arrhenius-like variable scaling, on the periodic box [0,2)x[0,1).

    Variable v: phi_v = sum_m g_m exp(-10 b_v / tau) / exp(-10 b_v / 4), with
    tau = 1 + 3 sum_m theta_m g_m, b_v = 1 + v/8, plus `noise` * N(0,1) i.i.d.
    (counter-based, seed noise_seed + k for snapshot k).
    """
    lx, ly = 2.0, 1.0
    xs = torch.arange(nx, dtype=torch.float64) * (lx / nx)
    ys = torch.arange(ny, dtype=torch.float64) * (ly / ny)
    beta = 1.0 + torch.arange(nv, dtype=torch.float64) / 8.0
    t_of = {}

    def fld_clean(t, device):
        X = xs.to(device)[:, None]
        Y = ys.to(device)[None, :]
        gs, th = [], []
        for m in range(3):
            cx = _PLUME_C0[m][0] + centre_shift[0] + 1.0 * t
            cy = _PLUME_C0[m][1] + centre_shift[1] + 0.2 * t
            dx = X - cx
            dx = dx - lx * torch.round(dx / lx)
            dy = Y - cy
            dy = dy - ly * torch.round(dy / ly)
            d = torch.sqrt(dx * dx + dy * dy)
            g = torch.exp(-(d * d) / (2.0 * (_PLUME_S[m] * width_scale) ** 2))
            R = _PLUME_R[m] * (1.0 + growth * t)
            theta = 0.5 * (1.0 + torch.tanh((R - d) / 0.02))
            gs.append(g)
            th.append(theta)
        tau = 1.0 + 3.0 * sum(t_ * g_ for t_, g_ in zip(th, gs))
        gsum = gs[0] + gs[1] + gs[2]
        b = beta.to(device)[None, None, :]
        return gsum[:, :, None] * torch.exp(-10.0 * b / tau[:, :, None]) / torch.exp(-10.0 * b / 4.0)

    def fld(t, device, dtype):
        v = fld_clean(t, device)
        if noise > 0.0:
            k = int(round((t - 0.0) / dt))
            z = counter_normal(nx * ny * nv, noise_seed + k, device).reshape(nx, ny, nv)
            v = v + noise * z
        return v.to(dtype)

    dims = (nx, ny, nv)
    return StreamSpec(
        name=f"plume-{nx}x{ny}x{nv}", dims=dims, weights=_uniform_weights(dims), dt=dt,
        steps=steps, field_fn=fld, storage="f32", eps_th=1e-4, rank_init=None,
        rank_max=(64, 64, nv), adaptive=True, meta={"start_ranks": (4, 4, 4)})


# --------------------------------------------------------------------------- samples as a mode
def stochastic_plume_spec(nx: int = 128, ny: int = 64, nv: int = 8, s=(4, 4), steps: int = 200,
                          dt: float = 5e-4, weights: str = "pcm", spread: float = 0.25,
                          noise: float = 1e-6) -> StreamSpec:
    """Samples as a tensor mode (the stochastic case of Sec. 3.3, eq. (UQ)): the
    reactive-flow-shaped field for s1 x s2 values (xi1, xi2) of two random
    coefficients, on the tensor-product Gauss-Legendre points of [-1, 1]^2. Coefficient
    xi1 scales the plume widths by 1 + spread xi1 (a diffusion-like parameter), xi2 the
    reaction fronts' growth rate by 1 + spread xi2. The samples are stacked along a
    leading mode (xi1 slow, xi2 fast), so a snapshot is (S, nx, ny, nv) and sample i is
    the i-th contiguous block. Sample-mode weights: the product Gauss weights
    (probabilistic collocation, "pcm") or 1/S (Monte Carlo, "mc"), normalised to sum 1.
    Sample i draws its noise from seed 2 + 1000 i + k at snapshot k."""
    g1, q1 = np.polynomial.legendre.leggauss(s[0])
    g2, q2 = np.polynomial.legendre.leggauss(s[1])
    pts = [(a, b) for a in g1 for b in g2]
    specs = [plume_spec(nx, ny, nv, steps, dt, noise=noise, noise_seed=2 + 1000 * i,
                        width_scale=1.0 + spread * a, growth=2.0 * (1.0 + spread * b))
             for i, (a, b) in enumerate(pts)]
    S = len(pts)
    if weights == "pcm":
        wq = np.kron(q1, q2)
        wq = wq / wq.sum()
    elif weights == "mc":
        wq = np.full(S, 1.0 / S)
    else:
        raise ValueError(f"unknown sample weights {weights!r}")

    def fld(t, device, dtype):
        return torch.stack([sp.field_fn(t, device, dtype) for sp in specs])

    dims = (S, nx, ny, nv)
    return StreamSpec(
        name=f"stochastic-plume-{S}x{nx}x{ny}x{nv}", dims=dims, weights=[wq] + list(specs[0].weights), dt=dt,
        steps=steps, field_fn=fld, storage="f32", eps_th=1e-4, rank_init=None,
        rank_max=(S, 32, 32, nv), adaptive=True,
        meta={"samples": pts, "sample_weights": weights, "sample_specs": specs})


# --------------------------------------------------------------------------- C3
def fourier_ensemble_specs(n_streams: int = 256, seed0: int = 1000, steps: int = 500,
                           dt: float = 1e-3, sizes=(128, 192, 256), nv: int = 4,
                           n_modes: int = 16, kmax: int = 8) -> List[StreamSpec]:
    """Batched stochastic ensemble: independent 2-D periodic fields of uneven size.

    Stream s (PCG64 seed seed0+s): N_x, N_y uniform on `sizes`; each of `nv`
    variables is sum_{m<16} a cos(kx x + ky y + phi0 + w t) with integer k on
    [-kmax,kmax]^2 minus the origin, a ~ N(0,1)|k|^(-5/6), phi0 ~ U[0,2pi),
    w ~ U(0.5,2). Multilinear rank is at most (2 kmax + 1, 2 kmax + 1, nv).
    """
    specs = []
    for s in range(n_streams):
        rng = np.random.Generator(np.random.PCG64(seed0 + s))
        nx = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        kx = np.zeros((nv, n_modes))
        ky = np.zeros((nv, n_modes))
        amp = np.zeros((nv, n_modes))
        ph = np.zeros((nv, n_modes))
        om = np.zeros((nv, n_modes))
        for v in range(nv):
            for m in range(n_modes):
                while True:
                    k = rng.integers(-kmax, kmax + 1, size=2)
                    if k[0] != 0 or k[1] != 0:
                        break
                kx[v, m], ky[v, m] = k
                amp[v, m] = rng.normal() * float(np.hypot(k[0], k[1])) ** (-5.0 / 6.0)
                ph[v, m] = rng.uniform(0.0, 2.0 * math.pi)
                om[v, m] = rng.uniform(0.5, 2.0)
        specs.append(_fourier_stream(s, nx, ny, nv, kx, ky, amp, ph, om, steps, dt))
    return specs


def _fourier_stream(s, nx, ny, nv, kx, ky, amp, ph, om, steps, dt) -> StreamSpec:
    xs = torch.arange(nx, dtype=torch.float64) * (2.0 * math.pi / nx)
    ys = torch.arange(ny, dtype=torch.float64) * (2.0 * math.pi / ny)
    KX = torch.tensor(kx)
    KY = torch.tensor(ky)
    A = torch.tensor(amp)
    PH = torch.tensor(ph)
    OM = torch.tensor(om)

    def fld(t, device, dtype):
        X = xs.to(device)
        Y = ys.to(device)
        out = torch.empty((nx, ny, nv), dtype=torch.float64, device=device)
        # elementwise over (x, y, mode), then a sum over the modes (no library matrix
        # product, so every device and run gives the same values)
        for v in range(nv):
            kx, ky = KX[v].to(device), KY[v].to(device)
            arg = (X[:, None, None] * kx[None, None, :] + Y[None, :, None] * ky[None, None, :]
                   + (PH[v] + OM[v] * t).to(device)[None, None, :])
            out[:, :, v] = (A[v].to(device)[None, None, :] * torch.cos(arg)).sum(dim=2)
        return out.to(dtype)

    dims = (nx, ny, nv)
    return StreamSpec(
        name=f"ensemble-{s}-{nx}x{ny}x{nv}", dims=dims, weights=_uniform_weights(dims), dt=dt,
        steps=steps, field_fn=fld, storage="f32", eps_th=1e-5, rank_init=None,
        rank_max=(24, 24, nv), adaptive=True, meta={"seed": s})


# --------------------------------------------------------------------------- C4
def _cheb_trapezoid_weights(ny: int) -> np.ndarray:
    y = np.cos(np.pi * np.arange(ny) / (ny - 1))
    w = np.zeros(ny)
    dy = np.abs(np.diff(y))
    w[:-1] += 0.5 * dy
    w[1:] += 0.5 * dy
    return w / w.sum()


def channel_spec(nx: int = 192, ny: int = 129, nz: int = 192, n_modes: int = 2048,
                 steps: int = 400, dt: float = 1e-3, seed: int = 4, kmax: int = 16,
                 kymax: float = 16.0, rms: float = 0.1) -> StreamSpec:
    """Channel-flow-shaped stream (x, wall-normal y on Chebyshev points, z, component).

    V_c = delta_{c0} (1 - y^2) + (1 - y^2) sum_m A_{m,c} cos(kx (x - U(y) t) + ky y
    + 2 kz z + phi_m), U = 1 - y^2, kx, kz uniform integers in [-kmax, kmax],
    ky ~ U[0, kymax), modes with |k| < 1 redrawn, A ~ N(0,1)|k|^(-5/6) rescaled so
    that sqrt(sum_m A_{m,c}^2 / 2) = rms for every component.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    kx = np.zeros(n_modes, dtype=np.int64)
    kz = np.zeros(n_modes, dtype=np.int64)
    ky = np.zeros(n_modes)
    for m in range(n_modes):
        while True:
            a = int(rng.integers(-kmax, kmax + 1))
            c = int(rng.integers(-kmax, kmax + 1))
            b = float(rng.uniform(0.0, kymax))
            if math.sqrt(a * a + b * b + (2 * c) ** 2) >= 1.0:
                break
        kx[m], kz[m], ky[m] = a, c, b
    kmag = np.sqrt(kx ** 2 + ky ** 2 + (2 * kz) ** 2)
    A = rng.normal(size=(n_modes, 3)) * kmag[:, None] ** (-5.0 / 6.0)
    A *= rms / np.sqrt((A ** 2).sum(axis=0) / 2.0)[None, :]
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)

    xs = torch.arange(nx, dtype=torch.float64) * (2.0 * math.pi / nx)
    zs = torch.arange(nz, dtype=torch.float64) * (math.pi / nz)
    ys = torch.cos(math.pi * torch.arange(ny, dtype=torch.float64) / (ny - 1))
    nkx = 2 * kmax + 1
    # Group modes by (kx, kz): each group contributes one separable x-z Fourier pair.
    gidx = torch.tensor((kx + kmax) * nkx + (kz + kmax))
    KX = torch.tensor(kx, dtype=torch.float64)
    KY = torch.tensor(ky)
    AM = torch.tensor(A)
    PHI = torch.tensor(phi)
    kxs = torch.arange(-kmax, kmax + 1, dtype=torch.float64)

    def fld(t, device, dtype):
        Y = ys.to(device)
        U = 1.0 - Y * Y
        # phase of each mode in y: ky y - kx U(y) t + phi     (n_modes x ny)
        ph = KY.to(device)[:, None] * Y[None, :] - KX.to(device)[:, None] * U[None, :] * t \
            + PHI.to(device)[:, None]
        ey = torch.polar(torch.ones_like(ph), ph)                      # complex
        coef = torch.zeros((nkx * nkx, ny, 3), dtype=torch.complex128, device=device)
        contrib = ey[:, :, None] * AM.to(device)[:, None, :].to(torch.complex128)
        coef.index_add_(0, gidx.to(device), contrib)
        coef = coef.reshape(nkx, nkx, ny, 3)                           # kx, kz, y, c
        ex = torch.polar(torch.ones((nx, nkx), dtype=torch.float64, device=device),
                         xs.to(device)[:, None] * kxs.to(device)[None, :])
        ez = torch.polar(torch.ones((nz, nkx), dtype=torch.float64, device=device),
                         2.0 * zs.to(device)[:, None] * kxs.to(device)[None, :])
        # sum over kz, then kx:  out[i, j, l, c] = Re sum ex[i,a] ez[l,b] coef[a,b,j,c]
        tmp = torch.einsum("lb,abjc->ajlc", ez, coef)
        out = torch.einsum("ia,ajlc->ijlc", ex, tmp).real
        out = out * U[None, :, None, None]
        out[:, :, :, 0] += U[None, :, None]
        return out.to(dtype)

    dims = (nx, ny, nz, 3)
    w = [np.full(nx, 1.0 / nx), _cheb_trapezoid_weights(ny), np.full(nz, 1.0 / nz),
         np.full(3, 1.0 / 3.0)]
    return StreamSpec(
        name=f"channel-{nx}x{ny}x{nz}x3", dims=dims, weights=w, dt=dt, steps=steps,
        field_fn=fld, storage="f32", eps_th=1e-3, rank_init=None, rank_max=(40, 40, 40, 3),
        adaptive=True, meta={"seed": seed})


# --------------------------------------------------------------------------- Runge
def runge_spec(n: int = 126, steps: int = 400, dt: float = 5e-3, alpha: float = 0.5,
               eps_th: float = 1e-6, gamma_th: float = 99.999) -> StreamSpec:
    """Time-dependent Runge function on [-pi,pi]^3:
    f = 1 / (a(t)^2 + x1^2 + x2^2 + x3^2), a(t) = 1 - 0.5 exp(-alpha (t-1)^2)."""
    x = torch.linspace(-math.pi, math.pi, n, dtype=torch.float64)

    def a_of(t):
        return 1.0 - 0.5 * math.exp(-alpha * (t - 1.0) ** 2)

    def fld(t, device, dtype):
        xs = x.to(device)
        r2 = xs[:, None, None] ** 2 + xs[None, :, None] ** 2 + xs[None, None, :] ** 2
        return (1.0 / (a_of(t) ** 2 + r2)).to(dtype)

    def dfld(t, device, dtype):
        xs = x.to(device)
        r2 = xs[:, None, None] ** 2 + xs[None, :, None] ** 2 + xs[None, None, :] ** 2
        a = a_of(t)
        # d/dt [1 - 0.5 exp(-alpha (t-1)^2)] = alpha (t-1) exp(-alpha (t-1)^2)
        da = alpha * (t - 1.0) * math.exp(-alpha * (t - 1.0) ** 2)
        return (-2.0 * a * da / (a * a + r2) ** 2).to(dtype)

    dims = (n, n, n)
    return StreamSpec(
        name=f"runge-{n}^3", dims=dims, weights=_uniform_weights(dims), dt=dt, steps=steps,
        field_fn=fld, deriv_fn=dfld, storage="f64", eps_th=eps_th, gamma_th=gamma_th,
        rank_init=(3, 3, 3), rank_max=(8, 8, 8), adaptive=True)


# --------------------------------------------------------------------------- pins
def _orthonormal(rng, n, r):
    q, _ = np.linalg.qr(rng.normal(size=(n, r)))
    return q


def lowrank_manifold_spec(dims=(12, 10, 8), ranks=(3, 3, 2), steps: int = 50,
                          dt: float = 1e-2, seed: int = 0, rot: float = 0.5) -> StreamSpec:
    """Exactly low-rank stream V(t) = K(t) x_n (expm(t A_n) B_n), A_n skew.

    Multilinear rank is exactly `ranks` for every t, with a smooth closed-form
    derivative (used for the time-integration order pin).
    """
    from scipy.linalg import expm

    rng = np.random.Generator(np.random.PCG64(seed))
    B = [_orthonormal(rng, n, r) for n, r in zip(dims, ranks)]
    A = []
    for n in dims:
        M = rng.normal(size=(n, n)) * (rot / math.sqrt(n))
        A.append(M - M.T)
    K0 = rng.normal(size=ranks)
    K1 = rng.normal(size=ranks) * 0.5
    K2 = rng.normal(size=ranks) * 0.3

    def core(t):
        return K0 + math.sin(t) * K1 + t * t * K2

    def dcore(t):
        return math.cos(t) * K1 + 2.0 * t * K2

    def factors(t):
        return [expm(t * a) @ b for a, b in zip(A, B)]

    def build(K, Fs):
        out = K
        for n, F in enumerate(Fs):
            out = np.moveaxis(np.tensordot(F, out, axes=([1], [n])), 0, n)
        return out

    def fld(t, device, dtype):
        return torch.tensor(build(core(t), factors(t))).to(device=device, dtype=dtype)

    def dfld(t, device, dtype):
        Fs = factors(t)
        dFs = [a @ f for a, f in zip(A, Fs)]
        out = build(dcore(t), Fs)
        for n in range(len(dims)):
            Gs = list(Fs)
            Gs[n] = dFs[n]
            out = out + build(core(t), Gs)
        return torch.tensor(out).to(device=device, dtype=dtype)

    return StreamSpec(
        name="lowrank-manifold", dims=tuple(dims), weights=_uniform_weights(dims), dt=dt,
        steps=steps, field_fn=fld, deriv_fn=dfld, storage="f64", rank_init=tuple(ranks),
        rank_max=tuple(ranks), adaptive=False, eps_th=1.0)


def switched_term_spec(dims=(16, 14, 12), ranks=(3, 3, 3), t_on: float = 0.1,
                       ramp: float = 2.0, amp6: float = 1.0, steps: int = 60,
                       dt: float = 5e-3, seed: int = 3, eps_th: float = 1e-2,
                       profile: Optional[Callable[[float], float]] = None,
                       profile2: Optional[Callable[[float], float]] = None) -> StreamSpec:
    """A static-span exactly low-rank stream plus extra separable terms whose
    factors are orthogonal (in the quadrature weights) to the base span and to
    each other: V = K(t) x_n Q_n + h(t) q1 o q2 o q3 + g(t) z1 o z2 o z3, with
    h(t) = amp6 * ramp * max(t - t_on, 0) unless `profile` gives h, and g given by
    `profile2` (default 0). All factors have unit W-norm, so while a rank-`ranks`
    decomposition tracks the base the exact weighted error is
    sqrt(h(t)^2 + g(t)^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _uniform_weights(dims)
    Q, q, z = [], [], []
    for n, r, wn in zip(dims, ranks, w):
        # W-orthonormal basis of r+2 columns; the last two are the extra factors.
        G = rng.normal(size=(n, r + 2))
        s = np.sqrt(wn)[:, None]
        qq, _ = np.linalg.qr(s * G)
        qq = qq / s
        Q.append(qq[:, :r])
        q.append(qq[:, r])
        z.append(qq[:, r + 1])
    K0 = rng.normal(size=ranks)
    K1 = rng.normal(size=ranks) * 0.3
    extra = np.einsum("i,j,k->ijk", q[0], q[1], q[2])
    extra2 = np.einsum("i,j,k->ijk", z[0], z[1], z[2])
    g = profile2 if profile2 is not None else (lambda t: 0.0)

    def h_default(t):
        return amp6 * ramp * max(t - t_on, 0.0)

    h = profile if profile is not None else h_default

    def base(t):
        out = K0 + math.sin(3.0 * t) * K1
        for n, F in enumerate(Q):
            out = np.moveaxis(np.tensordot(F, out, axes=([1], [n])), 0, n)
        return out

    def fld(t, device, dtype):
        return torch.tensor(base(t) + h(t) * extra + g(t) * extra2).to(device=device, dtype=dtype)

    qnorm = float(np.prod([math.sqrt(np.sum(wn * qn * qn)) for wn, qn in zip(w, q)]))
    return StreamSpec(
        name="switched-term", dims=tuple(dims), weights=w, dt=dt, steps=steps, field_fn=fld,
        storage="f64", eps_th=eps_th, rank_init=tuple(ranks),
        rank_max=tuple(r + 2 for r in ranks), adaptive=True,
        meta={"t_on": t_on, "qnorm": qnorm, "h": h, "g": g})


# --------------------------------------------------------------------------- gate init
def gate_init_params(seed: int = 11) -> np.ndarray:
    """Initial parameters of the 384-128-128-1 error-gate network (flat FP32 vector:
    W1 128x384, b1, W2 128x128, b2, w3, b3), each layer's weights and biases uniform on
    [-1/sqrt(fan_in), 1/sqrt(fan_in)] from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, shape in ((384, (128, 384)), (384, (128,)), (128, (128, 128)), (128, (128,)), (128, (128,)),
                          (128, (1,))):
        b = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, size=shape).ravel())
    return np.concatenate(parts).astype(np.float32)
