"""Seeded synthetic inputs for the IRK stage-solve workloads.

This module holds only input construction (initial data, request streams);
none of the time-stepping arithmetic.  Both the HIP path and the CPU oracle
are fed from here, so it imports neither.

Workloads (periodic unit domains, nodes x_i = i h, h = 1/n; arrays indexed
[j (y), i (x)], x contiguous):

* Burgers-1D: u0 = sum_{k=1..4} a_k sin(2 pi k x + phi_k), a_k ~ U[0,1),
  phi_k ~ U[0, 2 pi) (NumPy PCG64 seeded).
* Nonlinear diffusion 2-D: u0 = sin(2 pi x) sin(2 pi y), the manufactured
  solution at t = 0.
* Vorticity-streamfunction 2-D: omega0 = sum_m sigma_m exp(-|x - x_m|^2 / r_m^2)
  over seeded Gaussian vortices (minimum-image periodic distance), centres
  U[0,1)^2, radii U[0.02, 0.05], strengths +-U[1, 5] with random sign; psi0 is
  the consistent streamfunction, -Lap_h psi0 = omega0 - mean(omega0) with
  mean(psi0) = 0, obtained spectrally from the 5-point symbol (the algebraic
  constraint of an index-1 DAE must hold for the initial value).
* Serving: a seeded stream of step-solve requests with Poisson arrivals.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def burgers_u0(n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.0, 1.0, size=4)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=4)
    x = np.arange(n) / n
    u = np.zeros(n)
    for k in range(1, 5):
        u += a[k - 1] * np.sin(2.0 * np.pi * k * x + phi[k - 1])
    return u


def nldiff_u0(n: int) -> np.ndarray:
    g = np.arange(n) / n
    X, Y = np.meshgrid(g, g)
    return np.sin(2.0 * np.pi * X) * np.sin(2.0 * np.pi * Y)


def nldiff_random_u0(n: int, seed: int, amplitude: float = 1.0) -> np.ndarray:
    """Smooth seeded field (a few low Fourier modes) for parity cases that
    should not coincide with the manufactured solution."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.arange(n) / n
    u = np.zeros((n, n))
    for _ in range(6):
        kx, ky = rng.integers(1, 4, size=2)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=2)
        a = rng.uniform(-1.0, 1.0)
        # separable mode a sin(2 pi kx x + ph0) cos(2 pi ky y + ph1), evaluated
        # from 1-D factors (same values as the 2-D evaluation, O(n) sin/cos)
        sx = np.sin(2 * np.pi * kx * g + ph[0])
        cy = np.cos(2 * np.pi * ky * g + ph[1])
        u += (a * sx)[None, :] * cy[:, None]
    return amplitude * u / max(1.0, float(np.abs(u).max()))


def vsf_omega0(n: int, seed: int = 0, n_vortices: int = 32) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, 1.0, size=(n_vortices, 2))
    radii = rng.uniform(0.02, 0.05, size=n_vortices)
    strength = rng.uniform(1.0, 5.0, size=n_vortices) * rng.choice([-1.0, 1.0], size=n_vortices)
    g = np.arange(n) / n
    X, Y = np.meshgrid(g, g)
    om = np.zeros((n, n))
    for (cx, cy), r, sg in zip(centres, radii, strength):
        dx = X - cx
        dy = Y - cy
        dx -= np.round(dx)
        dy -= np.round(dy)
        om += sg * np.exp(-(dx * dx + dy * dy) / (r * r))
    return om


def vsf_psi0(omega: np.ndarray) -> np.ndarray:
    """Consistent streamfunction for the 5-point periodic Laplacian."""
    n = omega.shape[0]
    h = 1.0 / n
    k = np.arange(n)
    sym1 = (4.0 / (h * h)) * np.sin(np.pi * k / n) ** 2   # symbol of -D2 per axis
    sym = sym1[:, None] + sym1[None, :]
    w = np.fft.fft2(omega - omega.mean())
    sym[0, 0] = 1.0
    p = w / sym
    p[0, 0] = 0.0
    return np.real(np.fft.ifft2(p))


def vsf_state0(n: int, seed: int = 0, n_vortices: int = 32) -> np.ndarray:
    """Stacked (omega0, psi0), shape (2, n, n)."""
    om = vsf_omega0(n, seed, n_vortices)
    return np.stack([om, vsf_psi0(om)])


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float        # seconds after the stream starts
    n: int                # grid side
    family: str           # "gauss" | "radau"
    s: int
    dt: float
    nsteps: int
    seed: int


def serving_requests(count: int, rate: float, seed: int = 0,
                     sides=(128, 256, 512, 1024), stages=(2, 3, 4),
                     nsteps: int = 10) -> list:
    """Seeded request stream: Poisson arrivals at ``rate`` per second, grid
    side uniform over ``sides`` (uniform in log2), family and s uniform,
    dt log-uniform on [1e-3, 1e-2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=count) if rate > 0 else np.zeros(count)
    t = np.cumsum(gaps)
    out = []
    for r in range(count):
        out.append(Request(
            rid=r,
            arrival=float(t[r]),
            n=int(rng.choice(sides)),
            family=str(rng.choice(["gauss", "radau"])),
            s=int(rng.choice(stages)),
            dt=float(np.exp(rng.uniform(np.log(1e-3), np.log(1e-2)))),
            nsteps=nsteps,
            seed=int(rng.integers(0, 2 ** 31 - 1)),
        ))
    return out
