"""Seeded synthetic initial fields (rho, u) for the benchmark workloads.

This module holds no lattice Boltzmann arithmetic: it only produces the
macroscopic density and velocity fields that both the GPU library and the CPU
oracle start from (each side builds its own populations from them).  Every
generator is deterministic given its arguments.

Field layout: rho[z, y, x] and u[a, z, y, x] (x fastest), float64.  Node
coordinates are the integer site indices.
"""
from __future__ import annotations

import os

import numpy as np

# Seeds of the two randomised workloads.
TURBULENCE_SEED = 2002025030
BATCH_SEED = 2002025034


def _grid(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def taylor_green_2d(n: int, u0: float, T0: float, D: int = 2):
    """Taylor-Green vortex on an n x n periodic box with wavenumber k = 2 pi / n:

        u_x = -u0 cos(kx) sin(ky),   u_y = u0 sin(kx) cos(ky),
        rho = 1 - (u0^2 / 4 T0) (cos 2kx + cos 2ky)

    (the pressure field of the vortex with p = rho T0).  Returns rho (1, n, n)
    and u (D, 1, n, n)."""
    x, y, _ = _grid(n, n, 1)
    k = 2.0 * np.pi / n
    u = np.zeros((D, 1, n, n))
    u[0] = -u0 * np.cos(k * x) * np.sin(k * y)
    u[1] = u0 * np.sin(k * x) * np.cos(k * y)
    rho = 1.0 - (u0 * u0 / (4.0 * T0)) * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho, u


def shear_wave(dims, amplitude: float, U=(0.0, 0.0, 0.0), D: int = 3):
    """Transverse shear wave along x on a uniform background U:

        u = U + amplitude * sin(2 pi x / nx) * e_y,   rho = 1."""
    nx, ny, nz = dims
    x, _, _ = _grid(nx, ny, nz)
    u = np.zeros((D,) + x.shape)
    for a in range(D):
        u[a] = U[a]
    u[1] += amplitude * np.sin(2.0 * np.pi * x / nx)
    return np.ones(x.shape), u


def turbulence(n: int, k0: float = 4.0, u_rms: float = 0.04, seed: int = TURBULENCE_SEED):
    """Random-phase solenoidal velocity field on an n^3 periodic box.

    Fourier components live on integer wavevectors k with every |k_a| <= kc,
    kc = min(n // 2 - 1, 8 k0) (beyond 8 k0 the amplitude is below 1e-26 of its
    peak).  Each component gets amplitude |k| exp(-|k|^2 / k0^2) and an
    independent uniform phase per velocity component, drawn in C order over
    (component, kz, ky, kx) from numpy's default generator with `seed`, so the
    shell energy spectrum is proportional to k^4 exp(-2 k^2 / k0^2).  The field
    is projected onto k . u_hat = 0, the real part of its inverse FFT is taken,
    and it is scaled so that the per-component rms velocity sqrt(<|u|^2> / 3)
    equals u_rms.  rho = 1."""
    import scipy.fft as sfft

    rng = np.random.default_rng(seed)
    kc = int(min(n // 2 - 1, 8 * k0))
    m = 2 * kc + 1
    kk = np.arange(-kc, kc + 1, dtype=np.float64)
    kz, ky, kx = np.meshgrid(kk, kk, kk, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    amp = np.sqrt(k2) * np.exp(-k2 / (k0 * k0))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(3, m, m, m))
    uh = amp * np.exp(1j * phase)
    k2s = np.where(k2 == 0, 1.0, k2)
    kdotu = kx * uh[0] + ky * uh[1] + kz * uh[2]
    uh[0] -= kx * kdotu / k2s
    uh[1] -= ky * kdotu / k2s
    uh[2] -= kz * kdotu / k2s
    idx = np.arange(-kc, kc + 1) % n  # FFT storage positions of the kept modes
    u = np.zeros((3, n, n, n))
    workers = os.cpu_count() or 1
    full = np.zeros((n, n, n), dtype=np.complex128)
    for a in range(3):
        full[...] = 0.0
        full[np.ix_(idx, idx, idx)] = uh[a]
        u[a] = np.real(sfft.ifftn(full, workers=workers))
    scale = u_rms / np.sqrt(np.mean(np.sum(u * u, axis=0)) / 3.0)
    u *= scale
    return np.ones((n, n, n)), u


def batch_boxes(nbox: int = 256, side_lo: int = 16, side_hi: int = 64, tau_lo: float = 0.52,
                tau_hi: float = 1.0, u_max: float = 0.1, seed: int = BATCH_SEED):
    """Parameters of the batched workload: per box, each side drawn uniformly
    from the integers [side_lo, side_hi], tau uniform in [tau_lo, tau_hi], and a
    background velocity U uniform in the ball |U| <= u_max.  Returns a list of
    dicts with keys dims (nx, ny, nz), tau, U."""
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(nbox):
        dims = tuple(int(v) for v in rng.integers(side_lo, side_hi + 1, size=3))
        tau = float(rng.uniform(tau_lo, tau_hi))
        while True:
            U = rng.uniform(-u_max, u_max, size=3)
            if np.dot(U, U) <= u_max * u_max:
                break
        boxes.append({"dims": dims, "tau": tau, "U": tuple(float(v) for v in U)})
    return boxes


def taylor_green_box(dims, U, T0: float, amplitude: float = 0.05):
    """Taylor-Green vortex in the x-y plane of an (nx, ny, nz) box, on a
    uniform background U, with kx = 2 pi / nx and ky = 2 pi / ny:

        u_x = U_x - A cos(kx x) sin(ky y)
        u_y = U_y + A (kx / ky) sin(kx x) cos(ky y)
        u_z = U_z
        rho = 1 - (A^2 / 4 T0) [cos(2 kx x) + (kx / ky)^2 cos(2 ky y)]

    with A = amplitude / max(1, kx / ky), so that the largest velocity
    perturbation is `amplitude`.  The field is divergence free."""
    nx, ny, nz = dims
    x, y, _ = _grid(nx, ny, nz)
    kx, ky = 2.0 * np.pi / nx, 2.0 * np.pi / ny
    r = kx / ky
    A = amplitude / max(1.0, r)
    u = np.zeros((3,) + x.shape)
    u[0] = U[0] - A * np.cos(kx * x) * np.sin(ky * y)
    u[1] = U[1] + A * r * np.sin(kx * x) * np.cos(ky * y)
    u[2] = U[2]
    rho = 1.0 - (A * A / (4.0 * T0)) * (np.cos(2 * kx * x) + r * r * np.cos(2 * ky * y))
    return rho, u
