"""Seeded synthetic inputs (initial wave functions and parameter draws).

This module holds no arithmetic of the SSCN method: it only draws the seeded
initial conditions that both the CPU oracle and the GPU library are fed with.
Arrays are complex128 numpy arrays of shape (3, ny, nx), components ordered
m = +1, 0, -1, x fastest; random draws are taken component-major, then y, then
x, from ``numpy.random.default_rng(seed)``.
"""
import math

import numpy as np


def grid(n: int, d: float, origin: float | None = None) -> np.ndarray:
    """Grid coordinates origin + i d (default origin -n d / 2)."""
    o = -n * d / 2.0 if origin is None else origin
    return o + d * np.arange(n, dtype=np.float64)


def _unit_norm(psi: np.ndarray, dx: float, dy: float) -> np.ndarray:
    return psi / math.sqrt(dx * dy * float(np.sum(np.abs(psi) ** 2)))


def gaussian(nx: int, ny: int, dx: float, dy: float, x0: float | None = None, y0: float | None = None,
             populations=(0.25, 0.5, 0.25), phase_noise: float = 0.1, seed: int = 1,
             windings=(0, 0, 0), center=(0.0, 0.0), full_phase: bool = False) -> np.ndarray:
    """psi_m = sqrt(p_m) pi^{-1/2} exp(-(x^2 + y^2)/2) (x + i s y)^{|l_m|} exp(i theta_m),
    theta_m i.i.d. uniform in [-phase_noise, phase_noise] (or [-pi, pi) when
    ``full_phase``), normalised to dx dy sum |psi|^2 = 1.  ``windings`` seeds
    a central vortex of winding l_m (sign s = sign(l_m)) in component m."""
    x = grid(nx, dx, x0) - center[0]
    y = grid(ny, dy, y0) - center[1]
    X, Y = np.meshgrid(x, y)  # (ny, nx)
    rng = np.random.default_rng(seed)
    if full_phase:
        theta = rng.uniform(-math.pi, math.pi, size=(3, ny, nx))
    else:
        theta = rng.uniform(-phase_noise, phase_noise, size=(3, ny, nx))
    env = np.exp(-(X ** 2 + Y ** 2) / 2.0) / math.sqrt(math.pi)
    psi = np.empty((3, ny, nx), dtype=np.complex128)
    for m in range(3):
        l = int(windings[m])
        vort = (X + 1j * math.copysign(1.0, l) * Y) ** abs(l) if l != 0 else 1.0
        psi[m] = math.sqrt(populations[m]) * env * vort * np.exp(1j * theta[m])
    return _unit_norm(psi, dx, dy)


def add_noise(psi: np.ndarray, dx: float, dy: float, amplitude: float = 1e-3, seed: int = 3) -> np.ndarray:
    """psi + amplitude (xi_1 + i xi_2)/sqrt2, xi ~ N(0, 1) i.i.d., then unit norm."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(size=(2,) + psi.shape)
    out = psi + amplitude * (xi[0] + 1j * xi[1]) / math.sqrt(2.0)
    return _unit_norm(out, dx, dy)


def random_state(nx: int, ny: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Unstructured complex Gaussian field (for substep tests on random input)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(size=(2, 3, ny, nx))
    return scale * (z[0] + 1j * z[1])


def params(nx: int, ny: int, dx: float, dy: float | None = None, dt: float = 5e-4, c0: float = 0.0,
           c2: float = 0.0, gamma: float = 0.0, eta: int = 1, rabi: float = 0.0, omega: float = 0.0,
           x0: float | None = None, y0: float | None = None, gx: float = 1.0, gy: float = 1.0, split: int = 0,
           fix_m: int = 0, magnetization: float = 0.0) -> dict:
    """Plain parameter mapping understood by both the oracle and the library binding
    (gx, gy: trap frequencies; split: 0 Lie, 1 Strang; fix_m, magnetization:
    imaginary-time projection to a fixed magnetisation)."""
    dy = dx if dy is None else dy
    return {"nx": int(nx), "ny": int(ny), "dx": float(dx), "dy": float(dy),
            "x0": float(-nx * dx / 2.0 if x0 is None else x0), "y0": float(-ny * dy / 2.0 if y0 is None else y0),
            "dt": float(dt), "c0": float(c0), "c2": float(c2), "gamma": float(gamma), "eta": int(eta),
            "rabi": float(rabi), "omega": float(omega), "gx": float(gx), "gy": float(gy), "split": int(split),
            "fix_m": int(fix_m), "magnetization": float(magnetization)}


# The five workloads, as concrete seeded inputs.
def config_c1() -> dict:
    """128x128, dx = 0.1, [-6.4, 6.4), dt = 5e-4, 200 imaginary steps; c0 = 50,
    c2 = -1, Rashba gamma = 0.5, Rabi 0, Omega = 0.5; Gaussian, +-0.1 rad, seed 1."""
    return params(128, 128, 0.1, dt=5e-4, c0=50.0, c2=-1.0, gamma=0.5, eta=1, rabi=0.0, omega=0.5)


def config_c2() -> dict:
    """512x512, dx = 0.05, dt = 1e-4 real time; Dresselhaus gamma = 1, Rabi 0.2,
    Omega = 0.9, c0 = 200, c2 = +5."""
    return params(512, 512, 0.05, dt=1e-4, c0=200.0, c2=5.0, gamma=1.0, eta=-1, rabi=0.2, omega=0.9)


def config_c3(n: int = 4096) -> dict:
    """n x n (2048 or 4096), dx = 0.02, dt = 0.1 dx^2 imaginary; Rashba gamma = 0.75,
    Omega = 0.95, c0 = 1000, c2 = -20, Rabi 0."""
    return params(n, n, 0.02, dt=0.1 * 0.02 ** 2, c0=1000.0, c2=-20.0, gamma=0.75, eta=1, rabi=0.0, omega=0.95)


def batch_scan(n_condensates: int = 256, seed: int = 5) -> list:
    """Parameter scan: N = 32 k, k ~ U{4..16}; box [-12.8, 12.8); dt = 0.1 dx^2;
    Omega ~ U[0, 0.95], gamma ~ U[0, 1], c0 ~ U[10, 500], c2 ~ U[-20, 20],
    Rabi ~ U[0, 0.5], eta = +-1 with probability 1/2."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_condensates):
        n = 32 * int(rng.integers(4, 17))
        dx = 25.6 / n
        out.append(params(n, n, dx, dt=0.1 * dx * dx, c0=float(rng.uniform(10, 500)),
                          c2=float(rng.uniform(-20, 20)), gamma=float(rng.uniform(0, 1)),
                          eta=1 if rng.random() < 0.5 else -1, rabi=float(rng.uniform(0, 0.5)),
                          omega=float(rng.uniform(0, 0.95))))
    return out


def serving_trace(n_requests: int = 2000, rate: float = 200.0, seed: int = 6) -> list:
    """Poisson arrivals of rate ``rate`` per second; N in {128, 256, 512, 1024}
    with probability {0.4, 0.3, 0.2, 0.1} on the box [-12.8, 12.8) (dx = 25.6/N);
    couplings drawn as in ``batch_scan``; steps ~ U{500..5000}; imaginary or
    real time with probability 1/2, dt = 0.1 dx^2 (imaginary) or 0.025 dx^2
    (real).  Returns dicts with arrival, params, nsteps, mode, seed (the
    initial-state seed 10^6 + k)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice([128, 256, 512, 1024], p=[0.4, 0.3, 0.2, 0.1]))
        dx = 25.6 / n
        imag = bool(rng.random() < 0.5)
        p = params(n, n, dx, dt=(0.1 if imag else 0.025) * dx * dx, c0=float(rng.uniform(10, 500)),
                   c2=float(rng.uniform(-20, 20)), gamma=float(rng.uniform(0, 1)),
                   eta=1 if rng.random() < 0.5 else -1, rabi=float(rng.uniform(0, 0.5)),
                   omega=float(rng.uniform(0, 0.95)))
        out.append({"arrival": t, "params": p, "nsteps": int(rng.integers(500, 5001)),
                    "mode": "imag" if imag else "real", "seed": 10 ** 6 + k})
    return out
