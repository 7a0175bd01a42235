"""The staged batched step (a wave's tile of whole rows collected in LDS and
written as one contiguous run) against the batched step with direct stores:
the same bits for every row length, lattice, storage type, collision kind and
launch shape, and parity of the staged batch with the oracle."""
import numpy as np
import pytest

from gpu_common import BOUND, rel_rho, rel_u, run_oracle

pytestmark = pytest.mark.gpu

# Row lengths around the tiling rules: rows of 1, 2, 16, 20, 33, 40 and 64
# sites (whole rows per tile, several rows or one), 65 and 100 (64-site pieces
# of a longer row, written directly in both kernels).
MIXED = [(1, 3, 4), (2, 5, 3), (16, 7, 3), (20, 6, 5), (33, 4, 3), (40, 5, 2), (64, 3, 3), (65, 2, 3),
         (100, 3, 2)]


def _batch_fields(D, dims, seed):
    rng = np.random.default_rng(seed)
    n = sum(a * b * c for a, b, c in dims)
    return 1.0 + rng.uniform(-0.01, 0.01, n), rng.uniform(-0.05, 0.05, (D, n))


def _run(lattice, dims, taus, dtype, rho, u, steps, **kw):
    from paper_2002_02503_amd import lbm

    with lbm.Simulation(lattice, dims, taus, dtype=dtype, **kw) as sim:
        sim.init(rho, u).step(steps)
        return sim.moments()


CASES = [
    ("D3Q19", "fp32", {}),
    ("D3Q19", "fp16", {}),
    ("D3Q19", "bf16", {"collision": "bgk"}),
    ("D3Q19", "fp64", {"theta": 0.5}),
    ("D3Q15", "fp32", {}),
    ("D3Q39", "fp32", {"K": 5}),
    ("D3Q39", "fp64", {}),  # 39 * 64 * 8 B per wave: at most three waves per block
]


@pytest.mark.parametrize("lattice,dtype,kw", CASES)
@pytest.mark.parametrize("block", [64, 256])
def test_staged_equals_direct_batch(lattice, dtype, kw, block):
    taus = list(np.linspace(0.55, 0.95, len(MIXED)))
    rho, u = _batch_fields(3, MIXED, seed=block + len(lattice))
    a = _run(lattice, MIXED, taus, dtype, rho, u, 9, kernel="staged", block=block, **kw)
    b = _run(lattice, MIXED, taus, dtype, rho, u, 9, kernel="scalar", block=block, **kw)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_staged_d2q9_and_persistent_grid():
    """D2Q9 boxes (one plane), and a grid smaller than the tile count, so
    that each wave walks several tiles and reuses its LDS slice."""
    dims = [(d[0], d[1], 1) for d in MIXED]
    taus = [0.6] * len(dims)
    rho, u = _batch_fields(2, dims, seed=4)
    a = _run("D2Q9", dims, taus, "fp32", rho, u, 11, kernel="staged", block=128, grid=3)
    b = _run("D2Q9", dims, taus, "fp32", rho, u, 11, kernel="scalar")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    rho3, u3 = _batch_fields(3, MIXED, seed=5)
    a = _run("D3Q19", MIXED, taus, "fp32", rho3, u3, 11, kernel="staged", block=256, grid=2)
    b = _run("D3Q19", MIXED, taus, "fp32", rho3, u3, 11, kernel="scalar")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_staged_batch_in_graphs():
    dims = MIXED[:6]
    taus = [0.6, 0.7, 0.8, 0.9, 0.65, 0.75]
    rho, u = _batch_fields(3, dims, seed=6)
    a = _run("D3Q19", dims, taus, "fp32", rho, u, 23, kernel="staged", graph_chunk=4)
    b = _run("D3Q19", dims, taus, "fp32", rho, u, 23, kernel="scalar", graph_chunk=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_staged_batch_matches_oracle():
    """Each box of a staged batch against the oracle run of that box alone."""
    from paper_2002_02503_amd import lbm

    dims = [(20, 6, 5), (16, 4, 4), (40, 3, 4)]
    taus = [0.6, 0.7, 0.85]
    rho, u = _batch_fields(3, dims, seed=7)
    with lbm.Simulation("D3Q19", dims, taus, dtype="fp32", kernel="staged") as sim:
        sim.init(rho, u).step(17)
        r, uu = sim.moments()
        rb, ub = sim.split_boxes(r), sim.split_boxes(uu)
    off = 0
    for k, (nx, ny, nz) in enumerate(dims):
        n = nx * ny * nz
        r0 = rho[off:off + n].reshape(nz, ny, nx)
        u0 = u[:, off:off + n].reshape(3, nz, ny, nx)
        off += n
        r_ref, u_ref = run_oracle("D3Q19", (nx, ny, nz), taus[k], r0, u0, 17, mode="closed")
        assert rel_u(ub[k], u_ref) < BOUND["fp32"] and rel_rho(rb[k], r_ref) < BOUND["fp32"]


def test_staged_is_rejected_for_a_single_box():
    from paper_2002_02503_amd import lbm

    with pytest.raises(lbm.LBMError) as e:
        lbm.Simulation("D3Q19", (32, 8, 8), 0.6, kernel="staged")
    assert e.value.name == "LBM_EINVAL"
