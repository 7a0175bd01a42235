"""The two-step kernel (k_step2: two time steps per launch, the first step's
state kept in LDS) against the one-site step: the same bits after any number
of steps (an odd count ends with one one-site step), for every storage type,
collision kind and Hermite order of D3Q15 and D3Q19, over several column
tiles, with grids that leave blocks idle or split columns, in captured graphs
of odd and even chunks; its fit rules; tuning and kernel switches around it;
and parity with the oracle."""
import numpy as np
import pytest

from gpu_common import BOUND, rel_rho, rel_u, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _fields(dims, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    return 1.0 + rng.uniform(-0.01, 0.01, size=shape), rng.uniform(-amp, amp, size=(3,) + shape)


# boxes of 1 x 1 to 3 x 5 columns (64 x 8 sites; 64 x 4 for FP64), nz from 1
CASES = [
    ("D3Q19", (128, 16, 5), "fp32", {}),
    ("D3Q19", (64, 8, 1), "fp32", {}),
    ("D3Q19", (64, 8, 2), "fp32", {"K": 2}),
    ("D3Q19", (64, 16, 5), "fp32", {"theta": 0.5}),
    ("D3Q19", (192, 24, 7), "fp16", {"collision": "bgk"}),
    ("D3Q19", (64, 32, 3), "bf16", {}),
    ("D3Q19", (128, 12, 6), "fp64", {"theta": 0.5}),
    ("D3Q19", (64, 4, 9), "fp64", {}),
    ("D3Q15", (64, 32, 4), "fp32", {}),
    ("D3Q15", (64, 20, 3), "fp64", {"K": 2}),
    ("D3Q15", (192, 16, 2), "fp16", {"theta": 0.3}),
]


@pytest.mark.parametrize("lattice,dims,dtype,kw", CASES)
@pytest.mark.parametrize("steps", [1, 2, 7, 40])
def test_two_step_equals_one_site_step(lattice, dims, dtype, kw, steps):
    rho, u = _fields(dims, seed=steps + sum(dims))
    a = run_gpu(lattice, dims, 0.6, dtype, rho, u, steps, kernel="two_step", **kw)
    b = run_gpu(lattice, dims, 0.6, dtype, rho, u, steps, kernel="scalar", **kw)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("grid", [1, 3, 8, 13, 64, 2048])
def test_two_step_any_grid(grid):
    """Blocks take runs of column-planes: a run may span columns (small
    grids), a grid not a multiple of 8 takes the plain block order, and blocks
    past the last column-plane stay idle."""
    dims = (192, 16, 11)  # 6 columns x 11 planes = 66 column-planes
    rho, u = _fields(dims, seed=grid)
    a = run_gpu("D3Q19", dims, 0.57, "fp32", rho, u, 14, kernel="two_step", grid=grid)
    b = run_gpu("D3Q19", dims, 0.57, "fp32", rho, u, 14, kernel="scalar")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("chunk", [1, 2, 3, 32])
def test_two_step_graph_chunks(chunk):
    """A captured graph of an odd chunk ends with a one-site step, so the
    buffer parity and the time advance differently; 77 steps in all."""
    dims = (64, 16, 6)
    rho, u = _fields(dims, seed=chunk)
    a = run_gpu("D3Q19", dims, 0.57, "fp32", rho, u, 77, kernel="two_step", graph_chunk=chunk)
    b = run_gpu("D3Q19", dims, 0.57, "fp32", rho, u, 77, kernel="scalar")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("lattice,dims,dtype", [("D2Q9", (64, 32, 1), "fp32"), ("D3Q39", (64, 32, 4), "fp32"),
                                                ("D3Q19", (96, 32, 4), "fp32"), ("D3Q19", (64, 12, 4), "fp32"),
                                                ("D3Q19", (64, 6, 4), "fp64"), ("D3Q15", (32, 8, 4), "fp16")])
def test_two_step_fit_rules(lattice, dims, dtype):
    from paper_2002_02503_amd import lbm

    with pytest.raises(lbm.LBMError) as e:
        lbm.Simulation(lattice, dims, 0.6, dtype=dtype, kernel="two_step")
    assert e.value.name == "LBM_EINVAL"
    with pytest.raises(lbm.LBMError) as e:
        lbm.Simulation("D3Q19", [(64, 8, 4), (64, 8, 4)], [0.6, 0.7], kernel="two_step")
    assert e.value.name == "LBM_EINVAL"


def test_two_step_fits_fp64_tile():
    """ny a multiple of 4 but not 8 fits the FP64 tile only."""
    from paper_2002_02503_amd import lbm

    dims = (64, 12, 3)
    rho, u = _fields(dims, seed=5)
    a = run_gpu("D3Q19", dims, 0.6, "fp64", rho, u, 6, kernel="two_step")
    b = run_gpu("D3Q19", dims, 0.6, "fp64", rho, u, 6, kernel="scalar")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    with pytest.raises(lbm.LBMError):
        lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel="two_step")


@pytest.mark.parametrize("kernel", ["two_step", "twist", "scalar"])
@pytest.mark.parametrize("t0", [3, 4])
def test_tuning_with_two_step_keeps_the_state(kernel, t0):
    """The tuner (whose candidates include the two-step kernel here) starts
    from any kernel at an odd or even time; afterwards the run continues bit
    for bit, whichever kernel it chose."""
    from paper_2002_02503_amd import lbm

    dims = (64, 32, 5)
    rho, u = _fields(dims, seed=8)
    ref = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, t0 + 11, kernel="scalar")
    mid = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, t0, kernel="scalar")
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel=kernel) as sim:
        sim.init(rho, u).step(t0)
        sim.tune(steps=4)
        assert sim.t == t0
        r0, u0 = sim.moments()
        sim.step(11)
        r, uu = sim.moments()
    assert np.array_equal(r0, mid[0]) and np.array_equal(u0, mid[1])
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])


def test_switching_to_and_from_two_step_mid_run():
    from paper_2002_02503_amd import lbm

    dims = (64, 16, 5)
    rho, u = _fields(dims, seed=21)
    ref = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, 26, kernel="scalar")
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel="two_step", torch_memory=False) as sim:
        sim.init(rho, u).step(3)
        for kernel, n in [("twist", 3), ("two_step", 4), ("in_place", 1), ("two_step", 5), ("scalar", 1),
                          ("two_step", 2), ("twist", 2), ("two_step", 5)]:
            assert lbm.STATUS[sim.lib.lbm_set_kernel(sim.h, lbm.KERNELS[kernel])] == "LBM_OK"
            sim.step(n)
        assert sim.t == 26
        r, uu = sim.moments()
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])


def test_two_step_checkpoint_resumes_in_any_kernel():
    from paper_2002_02503_amd import lbm

    dims = (64, 8, 7)
    rho, u = _fields(dims, seed=31)
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel="two_step") as a, \
            lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel="scalar") as b:
        a.init(rho, u).step(5)
        b.init(rho, u).step(5)
        ck = a.get_state()
        assert np.array_equal(ck, b.get_state())
        b.step(6)
        ref = b.moments()
    for kernel in ["two_step", "twist", "scalar"]:
        with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel=kernel) as other:
            other.set_state(ck)
            other.step(6)
            r, uu = other.moments()
        assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1]), kernel


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp16"])
def test_two_step_matches_the_oracle(dtype):
    """Direct parity with the oracle on a box of several columns and a ragged
    step count (the last step one-site)."""
    dims, tau, steps = (64, 32, 6), 0.55, 21
    rho, u = _fields(dims, seed=44, amp=0.04)
    r, uu = run_gpu("D3Q19", dims, tau, dtype, rho, u, steps, kernel="two_step")
    r_ref, u_ref = run_oracle("D3Q19", dims, tau, rho, u, steps)
    eu, er = rel_u(uu, u_ref), rel_rho(r, r_ref)
    print(f"two-step D3Q19 {dims} {dtype} {steps} steps: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < BOUND[dtype] and er < BOUND[dtype]


@pytest.mark.parametrize("dims,fits", [((64, 16, 5), True), ((96, 6, 5), False)])
def test_cached_two_step_choice(tmp_path, dims, fits):
    """A tune-cache line naming the two-step kernel is taken for a box it
    fits and replaced by the one-site step for one it does not (nx not a
    multiple of 64, ny not of 8); either way the run gives the reference bits."""
    from paper_2002_02503_amd import lbm

    rho, u = _fields(dims, seed=17)
    ref = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, 9, kernel="scalar")
    cache = tmp_path / "tune.txt"
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32") as sim:
        sim.init(rho, u).tune(steps=2, cache=str(cache))
    key = open(cache).read().splitlines()[-1].split(" | ")[0]
    with open(cache, "a") as f:
        f.write(key + f" | {lbm.KERNELS['two_step']} 0 0\n")
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32") as sim:
        sim.init(rho, u).tune(steps=2, cache=str(cache))
        kernel = sim.info()["kernel"]
        sim.step(9)
        r, uu = sim.moments()
    assert kernel == (lbm.KERNELS["two_step"] if fits else lbm.KERNELS["scalar"])
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])


def _random_cases(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        dtype = ["fp32", "fp64", "fp16", "bf16"][rng.integers(4)]
        ty = 4 if dtype == "fp64" else 8
        lattice = ["D3Q19", "D3Q15"][rng.integers(2)]
        dims = (64 * int(rng.integers(1, 4)), ty * int(rng.integers(1, 6)), int(rng.integers(1, 10)))
        kw = [{}, {"collision": "bgk"}, {"K": 2}, {"theta": 0.4}][rng.integers(4)]
        out.append((lattice, dims, dtype, kw, int(rng.integers(1, 24)), int(rng.choice([0, 1, 5, 8, 24, 4096]))))
    return out


@pytest.mark.parametrize("lattice,dims,dtype,kw,steps,grid", _random_cases(16, 2002))
def test_two_step_random_shapes(lattice, dims, dtype, kw, steps, grid):
    """Seeded random boxes (several columns, nz from 1), step counts, grids
    (0: one block per compute unit), storage types and collision kinds: the
    two-step kernel gives the one-site step's bits."""
    rho, u = _fields(dims, seed=steps * 7 + sum(dims))
    a = run_gpu(lattice, dims, 0.58, dtype, rho, u, steps, kernel="two_step", grid=grid, **kw)
    b = run_gpu(lattice, dims, 0.58, dtype, rho, u, steps, kernel="scalar", **kw)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
