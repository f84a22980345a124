"""Seeded synthetic inputs for the space-time DG-SEM slab workloads.

This module holds no arithmetic of the method itself: it draws random numbers
and evaluates closed-form initial data at node coordinates that the caller
supplies (from whichever side -- product library or oracle -- is asking).
Both the GPU path and the oracle are fed from here, so every input is the
same array on both sides.

Workloads (the recipes are also listed in the design notes):
  * 1D advection: u0 = sin(2 pi x).
  * 2D advection-diffusion: u0 = sum_{m<8} A_m sin(2 pi (kx_m x + ky_m y) + phi_m),
    k uniform in {1..4}^2, A ~ U(-1, 1), phi ~ U(0, 2 pi), drawn in that order.
  * 2D Euler: the isentropic vortex of Sec. "Euler Equations" (strength S = 5,
    Mach 0.5, gamma = 1.4) centred at the origin, with multiplicative density
    noise rho <- rho (1 + 1e-3 xi), xi ~ U(-1, 1) per node, v and p held.
  * 1D Burgers: u0 = 0.5 + sum_{m<4} A_m sin(2 pi k_m x + phi_m), A ~ U(-0.05, 0.05).
  * 3D Navier-Stokes: Taylor-Green vortex on [0, 2 pi]^3, Mach 0.1, isothermal
    density rho = p / p0.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# closed-form initial data; X has shape (E, dim, ns) (physical node coordinates)
# ---------------------------------------------------------------------------
def sine_wave(X: np.ndarray) -> np.ndarray:
    """u0 = sin(2 pi x), shape (E, 1, ns)."""
    return np.sin(2.0 * np.pi * X[:, 0:1, :])


def fourier_params(seed: int, dim: int = 2, n_modes: int = 8, kmax: int = 4) -> dict:
    g = rng(seed)
    k = g.integers(1, kmax + 1, size=(n_modes, dim))
    A = g.uniform(-1.0, 1.0, size=n_modes)
    phi = g.uniform(0.0, 2.0 * np.pi, size=n_modes)
    return dict(k=k, A=A, phi=phi)


def fourier_modes(X: np.ndarray, params: dict) -> np.ndarray:
    """Sum of seeded Fourier modes, shape (E, 1, ns)."""
    dim = X.shape[1]
    out = np.zeros((X.shape[0], 1, X.shape[2]))
    for m in range(len(params["A"])):
        arg = params["phi"][m] + sum(2.0 * np.pi * params["k"][m, a] * X[:, a, :] for a in range(dim))
        out[:, 0, :] += params["A"][m] * np.sin(arg)
    return out


def burgers_params(seed: int, n_modes: int = 4, kmax: int = 4) -> dict:
    g = rng(seed)
    k = g.integers(1, kmax + 1, size=n_modes)
    A = g.uniform(-0.05, 0.05, size=n_modes)
    phi = g.uniform(0.0, 2.0 * np.pi, size=n_modes)
    return dict(k=k, A=A, phi=phi)


def burgers_smooth(X: np.ndarray, params: dict) -> np.ndarray:
    out = np.full((X.shape[0], 1, X.shape[2]), 0.5)
    for m in range(len(params["A"])):
        out[:, 0, :] += params["A"][m] * np.sin(2.0 * np.pi * params["k"][m] * X[:, 0, :] + params["phi"][m])
    return out


def euler_conservative(rho, vel, p, gamma):
    """Primitive -> conservative (rho, rho v, rho E) with E = p/(g-1) + rho |v|^2 / 2."""
    m = [rho * v for v in vel]
    E = p / (gamma - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho, *m, E], axis=1)


def isentropic_vortex(X: np.ndarray, strength=5.0, mach=0.5, gamma=1.4, noise=1e-3, seed=3,
                      t=0.0, center=(0.0, 0.0)) -> np.ndarray:
    """Vortex of Sec. "Euler Equations", translated by the unit background flow
    to time t; returns conservative variables, shape (E, 4, ns)."""
    x0 = X[:, 0, :] - center[0] - t
    x1 = X[:, 1, :] - center[1]
    f = 1.0 - x0 ** 2 - x1 ** 2
    S, M, g = strength, mach, gamma
    rho = (1.0 - S ** 2 * (g - 1.0) * M ** 2 * np.exp(f) / (8.0 * np.pi ** 2)) ** (1.0 / (g - 1.0))
    v1 = 1.0 - S * x1 * np.exp(f / 2.0) / (2.0 * np.pi)
    v2 = S * x0 * np.exp(f / 2.0) / (2.0 * np.pi)
    p = rho ** g / (g * M ** 2)
    if noise:
        xi = rng(seed).uniform(-1.0, 1.0, size=rho.shape)
        rho = rho * (1.0 + noise * xi)
    return euler_conservative(rho, [v1, v2], p, g)


def taylor_green(X: np.ndarray, mach=0.1, gamma=1.4) -> np.ndarray:
    """Taylor-Green vortex, V0 = L = rho0 = 1, isothermal density; shape (E, 5, ns)."""
    x, y, z = X[:, 0, :], X[:, 1, :], X[:, 2, :]
    p0 = 1.0 / (gamma * mach ** 2)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    rho = p / p0
    return euler_conservative(rho, [u, v, w], p, gamma)


def euler_bubble_3d(X: np.ndarray, t=0.0, gamma=1.4) -> np.ndarray:
    """Smooth density bubble advected by a uniform flow (the 3D Euler test of
    Sec. "Numerical Results", 4D space-time): constant pressure 0.3, velocity
    (cos(pi/5), sin(pi/5), sin(pi/5)), density 0.5 outside the ball of radius
    1/4 around the moving centre 0.25 + t v, 0.25 (cos(pi r) + 1)^2 + 0.5 inside
    with r = 16 |x - 0.25 - t v|^2.  The exact solution at any t; shape
    (E, 5, ns)."""
    vel = [math.cos(math.pi / 5), math.sin(math.pi / 5), math.sin(math.pi / 5)]
    r = sum((X[:, a, :] - 0.25 - t * vel[a]) ** 2 for a in range(3)) * 16.0
    rho = np.where(r > 1.0, 0.5, 0.25 * (np.cos(np.minimum(r, 1.0) * math.pi) + 1.0) ** 2 + 0.5)
    return euler_conservative(rho, [vel[a] + 0.0 * rho for a in range(3)], 0.3 + 0.0 * rho, gamma)


def rotating_pulse(X: np.ndarray, t=0.0, eps=1e-3) -> np.ndarray:
    """The rotating pulse of Sec. "Experiments / Advection-Diffusion"
    (analytic solution of eq. advdiffeq with b = (-4 y0, 4 x0), x0 = x - 0.5,
    y0 = y - 0.5, diffusivity eps) at time t; shape (E, ns)."""
    x0, y0 = X[:, 0, :] - 0.5, X[:, 1, :] - 0.5
    xq = x0 * np.cos(4 * t) + y0 * np.sin(4 * t) + 0.25
    yq = -x0 * np.sin(4 * t) + y0 * np.cos(4 * t)
    s = 0.004 + 4 * eps * t
    return 0.004 / s * np.exp(-(xq ** 2 + yq ** 2) / s)


def cfl_dt(cfl: float, h_min: float, N: int, lam_max: float) -> float:
    """dt = CFL h_min / ((2N + 1) lambda_max)."""
    return cfl * h_min / ((2 * N + 1) * lam_max)


def euler_max_speed(u: np.ndarray, gamma: float) -> float:
    """max over nodes of |v| + c for conservative states u of shape (E, d+2, ns)."""
    d = u.shape[1] - 2
    rho = u[:, 0, :]
    v2 = sum((u[:, 1 + a, :] / rho) ** 2 for a in range(d))
    p = (gamma - 1.0) * (u[:, d + 1, :] - 0.5 * rho * v2)
    return float(np.max(np.sqrt(v2) + np.sqrt(gamma * p / rho)))


# ---------------------------------------------------------------------------
# random slab states for parity tests
# ---------------------------------------------------------------------------
def random_slab(kind: int, dim: int, E: int, nv: int, Nt: int, ns: int, seed: int):
    """Random slab vector U, previous state u_prev and direction V in the ABI
    layout (flattened).  Scalar equations: standard normal.  Burgers: 0.5 plus
    noise.  Euler / Navier-Stokes: a fixed subsonic state times (1 + 0.05 xi)."""
    g = rng(seed)
    if kind in (4, 5):
        base = np.array([1.0] + [0.3, -0.2, 0.1][:dim] + [2.5])
        U = base[None, :, None, None] * (1.0 + 0.05 * g.standard_normal((E, nv, Nt, ns)))
        up = base[None, :, None] * (1.0 + 0.05 * g.standard_normal((E, nv, ns)))
        V = base[None, :, None, None] * g.standard_normal((E, nv, Nt, ns))
    elif kind == 3:
        U = 0.5 + 0.2 * g.standard_normal((E, nv, Nt, ns))
        up = 0.5 + 0.2 * g.standard_normal((E, nv, ns))
        V = g.standard_normal((E, nv, Nt, ns))
    else:
        U = g.standard_normal((E, nv, Nt, ns))
        up = g.standard_normal((E, nv, ns))
        V = g.standard_normal((E, nv, Nt, ns))
    return U.ravel(), up.ravel(), V.ravel()


# ---------------------------------------------------------------------------
# served request stream
# ---------------------------------------------------------------------------
def serving_stream(seed: int, n_requests: int, rate: float, kmin=8, kmax=256, n_choices=(2, 3, 4, 5),
                   nt_choices=(2, 3, 4)) -> list:
    """Mixed stream: half 1D Burgers, half 2D advection-diffusion, K uniform in
    [kmin, kmax] per axis, N and Nt uniform over the given sets, FP64 or
    FP32-inner 50/50, exponential inter-arrival times at `rate` per second."""
    g = rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += g.exponential(1.0 / rate) if rate > 0 else 0.0
        kind = "burgers" if g.random() < 0.5 else "advdiff"
        K = int(g.integers(kmin, kmax + 1))
        N = int(g.choice(n_choices))
        Nt = int(g.choice(nt_choices))
        fp32 = bool(g.random() < 0.5)
        out.append(dict(id=i, arrival=t, kind=kind, K=K, N=N, Nt=Nt, inner_fp32=fp32,
                        seed=int(g.integers(0, 2 ** 31 - 1))))
    return out


__all__ = [name for name in dir() if not name.startswith("_") and name not in ("np", "annotations")]
