"""Helpers shared by the GPU tests: running the library and the oracle on the
same seeded inputs, and sampled oracle values at full size through the light
cone (oracle.lightcone_samples)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2002_02503_amd import lbm

# The library's stated error bounds per storage type (max |du| over max |u|
# against the FP64 oracle): 1e-12 (FP64), 1e-5 (FP32), 5e-3 (FP16), 5e-2 (BF16).
BOUND = dict(lbm.STATED_BOUNDS)


def rel_u(u, u_ref) -> float:
    return float(np.abs(u - u_ref).max() / np.abs(u_ref).max())


def rel_rho(r, r_ref) -> float:
    return float(np.abs(r - r_ref).max() / np.abs(r_ref).max())


def run_gpu(lattice, dims, tau, dtype, rho, u, steps, K=None, **kw):
    with lbm.Simulation(lattice, dims, tau, dtype=dtype, K=K, **kw) as sim:
        sim.init(rho, u).step(steps)
        return sim.moments()


def run_oracle(lattice, dims, tau, rho, u, steps, K=None, mode="literal", **kw):
    sim = oracle.Sim(lattice, dims, tau, K=K, mode=mode, **kw).init(rho, u)
    sim.step(steps)
    return sim.moments()


def lightcone_samples(lattice, rho0, u0, tau, steps, points, K=None, mode="closed", **kw):
    """Oracle (rho, u) at `points` after `steps` steps (oracle.lightcone_samples)."""
    return oracle.lightcone_samples(lattice, rho0, u0, tau, steps, points, K=K, mode=mode, **kw)


def sample_points(shape, n, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    pts = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (0, ny - 1, 0), (nz - 1, 0, nx - 1)]
    for _ in range(n - len(pts)):
        pts.append((int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))))
    return pts
