"""GPU parity: the HIP fused step against the FP64 CPU oracle, element by
element on the same seeded inputs, for every lattice, storage type and
Hermite order, on boxes that span several blocks and end in a ragged tail,
and on degenerate boxes shorter than the largest lattice velocity."""
import numpy as np
import pytest

from gpu_common import BOUND, rel_rho, rel_u, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

def _random_fields(D, dims, amp=0.05, drho=0.01, seed=0):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    u = rng.uniform(-amp, amp, size=(D,) + shape)
    rho = 1.0 + rng.uniform(-drho, drho, size=shape)
    return rho, u


# (lattice, dims, K values): nx spans two 256-wide blocks with a ragged tail
CASES = [
    ("D2Q9", (300, 7, 1), [2, 3]),
    ("D3Q19", (300, 5, 4), [2, 3]),
    ("D3Q19", (70, 9, 6), [3]),
    ("D3Q39", (260, 5, 4), [2, 3, 4, 5]),
]


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("lattice,dims,Ks", CASES)
def test_step_matches_oracle(lattice, dims, Ks, dtype):
    D = 2 if lattice == "D2Q9" else 3
    rho, u = _random_fields(D, dims, seed=int(np.prod(dims)) + D)
    steps = 40
    for K in Ks:
        r_ref, u_ref = run_oracle(lattice, dims, 0.57, rho, u, steps, K=K, mode="closed" if K <= 4 else "literal")
        r, uu = run_gpu(lattice, dims, 0.57, dtype, rho, u, steps, K=K)
        eu, er = rel_u(uu, u_ref), rel_rho(r, r_ref)
        print(f"{lattice} {dims} K={K} {dtype}: u {eu:.2e} rho {er:.2e}", flush=True)
        assert eu < BOUND[dtype], (K, eu)
        assert er < BOUND[dtype], (K, er)


@pytest.mark.parametrize("lattice,dims", [
    ("D2Q9", (1, 1, 1)), ("D2Q9", (2, 3, 1)), ("D3Q19", (1, 2, 3)), ("D3Q19", (2, 2, 2)),
    ("D3Q39", (1, 1, 1)), ("D3Q39", (2, 1, 5)), ("D3Q39", (5, 3, 2)), ("D3Q39", (4, 4, 4)),
])
def test_degenerate_boxes_shorter_than_velocities(lattice, dims):
    """Periodic wrap when a side is shorter than |c_i| (D3Q39 reaches 3)."""
    D = 2 if lattice == "D2Q9" else 3
    rho, u = _random_fields(D, dims, seed=3)
    r_ref, u_ref = run_oracle(lattice, dims, 0.7, rho, u, 25)
    for dtype in ["fp64", "fp32"]:
        r, uu = run_gpu(lattice, dims, 0.7, dtype, rho, u, 25)
        assert rel_u(uu, u_ref) < BOUND[dtype]
        assert rel_rho(r, r_ref) < BOUND[dtype]


@pytest.mark.parametrize("block", [64, 128, 256])
def test_launch_shapes_agree_bitwise(block):
    """Every block size computes the same bits (the per-site arithmetic does
    not depend on the launch shape)."""
    dims = (200, 6, 5)
    rho, u = _random_fields(3, dims, seed=5)
    r0, u0 = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, 10)
    r1, u1 = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, 10, block=block)
    assert np.array_equal(r0, r1) and np.array_equal(u0, u1)


def test_zero_steps_returns_initial_moments():
    dims = (33, 7, 5)
    rho, u = _random_fields(3, dims, seed=9)
    r, uu = run_gpu("D3Q19", dims, 0.6, "fp64", rho, u, 0)
    assert np.abs(r - rho).max() < 1e-14
    assert np.abs(uu - u).max() < 1e-14


# (lattice, dims, dtype): nx = 4 V lanes ... 64 lanes per row, several rows
# per wave, a ragged last wave, odd ny and nz
ROW_WAVE_CASES = [
    ("D3Q19", (256, 5, 3), "fp32"), ("D3Q19", (64, 7, 3), "fp16"), ("D3Q19", (16, 9, 5), "bf16"),
    ("D3Q19", (4, 6, 5), "fp32"), ("D3Q19", (128, 3, 7), "fp64"), ("D3Q19", (2, 9, 4), "fp64"),
    ("D2Q9", (64, 11, 1), "fp32"), ("D2Q9", (8, 13, 1), "fp64"),
    ("D3Q39", (192, 4, 3), "fp32"), ("D3Q39", (12, 7, 5), "bf16"), ("D3Q39", (256, 3, 3), "fp16"),
]


@pytest.mark.parametrize("lattice,dims,dtype", ROW_WAVE_CASES)
def test_row_wave_kernel_matches_scalar_and_oracle(lattice, dims, dtype):
    """The row-wave step (V sites per lane, x-neighbours by lane shuffle)
    computes exactly the bits of the one-site-per-thread step, and both match
    the oracle."""
    D = 2 if lattice == "D2Q9" else 3
    rho, u = _random_fields(D, dims, seed=sum(dims))
    steps = 25
    rw = run_gpu(lattice, dims, 0.62, dtype, rho, u, steps, kernel="row_wave")
    sc = run_gpu(lattice, dims, 0.62, dtype, rho, u, steps, kernel="scalar")
    assert np.array_equal(rw[0], sc[0]) and np.array_equal(rw[1], sc[1])
    r_ref, u_ref = run_oracle(lattice, dims, 0.62, rho, u, steps, mode="closed")
    assert rel_u(rw[1], u_ref) < BOUND[dtype] and rel_rho(rw[0], r_ref) < BOUND[dtype]


def test_row_wave_is_rejected_where_it_does_not_apply():
    from paper_2002_02503_amd import lbm

    for lattice, dims, dtype in [("D3Q19", (260, 4, 4), "fp32"), ("D3Q19", (6, 4, 4), "fp32"),
                                 ("D3Q39", (64, 4, 4), "fp64"), ("D3Q19", (512, 2, 2), "fp32")]:
        with pytest.raises(lbm.LBMError) as e:
            lbm.Simulation(lattice, dims, 0.6, dtype=dtype, kernel="row_wave")
        assert e.value.name == "LBM_EINVAL"
