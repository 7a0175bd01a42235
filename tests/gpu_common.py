"""Helpers shared by the GPU tests: running the library and the oracle on the
same seeded inputs, and computing sampled oracle values at full size.

Light-cone sampling: the populations at site x after s steps depend only on
the initial fields within R*s sites of x (R = largest velocity component).
Running the oracle on a periodic box of side 2*R*s + 1 centred on x (cut out
of the full initial field) therefore gives the exact value at its centre: the
wrap-around of the small box contaminates only layers closer than R*s to its
faces."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2002_02503_amd import lbm

# Stated error bounds of the reduced-precision storage modes (max |du| over
# max |u| against the FP64 oracle).  FP64 and FP32 use the tolerances of the
# method's specification: 1e-12 and 1e-5 relative.
BOUND = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 5e-3, "bf16": 5e-2}


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
    """Oracle (rho, u) at `points` (list of (z, y, x)) after `steps` steps of a
    run started from (rho0, u0) on the full periodic box.  Further keywords
    (kind, theta) go to the oracle's Sim."""
    L = oracle.lattice(lattice)
    D = L["D"]
    R = int(np.abs(L["c"]).max())
    r = R * steps
    nz, ny, nx = rho0.shape
    side = 2 * r + 1
    rho_out, u_out = [], []
    for z, y, x in points:
        ix = (x + np.arange(-r, r + 1)) % nx
        iy = (y + np.arange(-r, r + 1)) % ny
        iz = (z + np.arange(-r, r + 1)) % nz if D == 3 else np.array([0])
        sub_r = rho0[np.ix_(iz, iy, ix)]
        sub_u = u0[(slice(None),) + np.ix_(iz, iy, ix)]
        dims = (side, side, side if D == 3 else 1)
        sim = oracle.Sim(lattice, dims, tau, K=K, mode=mode, **kw).init(sub_r, sub_u).step(steps)
        rr, uu = sim.moments()
        cz = r if D == 3 else 0
        rho_out.append(rr[cz, r, r])
        u_out.append(uu[:, cz, r, r])
    return np.array(rho_out), np.array(u_out).T


def sample_points(shape, n, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    pts = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (0, ny - 1, 0), (nz - 1, 0, nx - 1)]
    for _ in range(n - len(pts)):
        pts.append((int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx))))
    return pts
