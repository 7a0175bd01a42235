"""The in-place steps (one buffer, two alternating layouts of the state: the
swapped form k_step_ip and the twisted form k_step_tw) against the two-buffer
step: the same bits after any number of steps, whatever the graph chunking;
readers (moments, totals, residual, checkpoints) see the natural layout at
odd and even times; and parity with the oracle."""
import numpy as np
import pytest

from gpu_common import BOUND, rel_rho, rel_u, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _fields(D, dims, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    return 1.0 + rng.uniform(-0.01, 0.01, size=shape), rng.uniform(-amp, amp, size=(D,) + shape)


CASES = [
    ("D3Q19", (256, 5, 4), "fp32", {}),
    ("D3Q19", (70, 9, 6), "fp16", {}),
    ("D3Q19", (37, 6, 5), "bf16", {"collision": "bgk"}),
    ("D3Q19", (64, 7, 3), "fp64", {"theta": 0.5}),
    ("D3Q15", (300, 4, 3), "fp32", {}),
    ("D2Q9", (300, 7, 1), "fp32", {}),
    ("D3Q39", (260, 5, 4), "fp32", {}),
    ("D3Q39", (40, 6, 7), "fp16", {"K": 5}),
]


IN_PLACE = ["in_place", "twist"]


@pytest.mark.parametrize("kernel", IN_PLACE)
@pytest.mark.parametrize("lattice,dims,dtype,kw", CASES)
@pytest.mark.parametrize("steps", [1, 2, 7, 40])
def test_in_place_equals_two_buffer_step(lattice, dims, dtype, kw, steps, kernel):
    D = 2 if lattice == "D2Q9" else 3
    rho, u = _fields(D, dims, seed=steps + sum(dims))
    a = run_gpu(lattice, dims, 0.6, dtype, rho, u, steps, kernel=kernel, **kw)
    b = run_gpu(lattice, dims, 0.6, dtype, rho, u, steps, kernel="scalar", **kw)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("kernel", IN_PLACE)
@pytest.mark.parametrize("chunk", [1, 3, 32])
def test_in_place_graph_chunks(chunk, kernel):
    """Odd and even graph chunks alternate the layout inside a captured graph."""
    dims = (96, 5, 6)
    rho, u = _fields(3, dims, seed=chunk)
    a = run_gpu("D3Q19", dims, 0.57, "fp32", rho, u, 77, kernel=kernel, graph_chunk=chunk)
    b = run_gpu("D3Q19", dims, 0.57, "fp32", rho, u, 77, kernel="scalar")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("kernel", IN_PLACE)
@pytest.mark.parametrize("lattice,dims", [("D3Q19", (1, 2, 3)), ("D3Q19", (2, 2, 2)), ("D3Q39", (1, 1, 1)),
                                          ("D3Q39", (2, 1, 5)), ("D3Q39", (5, 3, 2)), ("D2Q9", (2, 3, 1))])
def test_in_place_degenerate_boxes(lattice, dims, kernel):
    """Boxes shorter than the velocities: every element is still read and
    written by exactly one thread."""
    D = 2 if lattice == "D2Q9" else 3
    rho, u = _fields(D, dims, seed=3)
    r_ref, u_ref = run_oracle(lattice, dims, 0.7, rho, u, 25)
    for dtype in ["fp64", "fp32"]:
        r, uu = run_gpu(lattice, dims, 0.7, dtype, rho, u, 25, kernel=kernel)
        assert rel_u(uu, u_ref) < BOUND[dtype] and rel_rho(r, r_ref) < BOUND[dtype]
        r2, u2 = run_gpu(lattice, dims, 0.7, dtype, rho, u, 25, kernel="scalar")
        assert np.array_equal(r, r2) and np.array_equal(uu, u2)


@pytest.mark.parametrize("kernel", IN_PLACE)
def test_in_place_matches_oracle(kernel):
    dims = (200, 6, 5)
    rho, u = _fields(3, dims, seed=11)
    r_ref, u_ref = run_oracle("D3Q19", dims, 0.55, rho, u, 31, mode="closed")
    for dtype in ["fp64", "fp32", "fp16", "bf16"]:
        r, uu = run_gpu("D3Q19", dims, 0.55, dtype, rho, u, 31, kernel=kernel)
        assert rel_u(uu, u_ref) < BOUND[dtype] and rel_rho(r, r_ref) < BOUND[dtype]


@pytest.mark.parametrize("kernel", IN_PLACE)
def test_readers_at_odd_and_even_times(kernel):
    """Moments, totals, residual and checkpoints after odd and even step
    counts equal those of the two-buffer step, and a checkpoint taken at an odd
    time resumes bit for bit in every kernel."""
    from paper_2002_02503_amd import lbm

    dims = (64, 9, 7)
    rho, u = _fields(3, dims, seed=5)
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel=kernel) as ip, \
            lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel="scalar") as sc:
        ip.init(rho, u)
        sc.init(rho, u)
        for n in [1, 1, 3, 2]:
            ip.step(n)
            sc.step(n)
            r1, u1 = ip.moments()
            r2, u2 = sc.moments()
            assert np.array_equal(r1, r2) and np.array_equal(u1, u2)
            assert np.array_equal(ip.totals(), sc.totals())
            assert ip.residual(r2, u2) == sc.residual(r2, u2)
            assert np.array_equal(ip.get_state(), sc.get_state())
            # reading does not disturb the state: stepping on gives the same bits
        assert ip.t == 7
        ck = ip.get_state()
        ip.step(5)
        sc.step(5)
        ref = sc.moments()
        for other_kernel in ["in_place", "twist", "scalar"]:
            with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel=other_kernel) as other:
                other.set_state(ck)
                assert other.t == 7
                other.step(5)
                r, uu = other.moments()
                assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])


@pytest.mark.parametrize("kernel", IN_PLACE)
def test_in_place_is_rejected_for_batches(kernel):
    from paper_2002_02503_amd import lbm

    with pytest.raises(lbm.LBMError) as e:
        lbm.Simulation("D3Q19", [(8, 8, 8), (9, 9, 9)], [0.6, 0.7], kernel=kernel)
    assert e.value.name == "LBM_EINVAL"


@pytest.mark.parametrize("kernel", IN_PLACE + ["scalar"])
@pytest.mark.parametrize("t0", [3, 4])
def test_tuning_across_layouts_keeps_the_state(kernel, t0):
    """The tuner switches between the in-place, twisted and two-buffer
    kernels with the state at an odd or even time; afterwards the run
    continues bit for bit, whichever kernel it chose."""
    from paper_2002_02503_amd import lbm

    dims = (128, 6, 5)
    rho, u = _fields(3, dims, seed=8)
    ref = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, t0 + 10, kernel="scalar")
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel=kernel) as sim:
        sim.init(rho, u).step(t0)
        sim.tune(steps=4)
        assert sim.t == t0
        r0, u0 = sim.moments()
        sim.step(10)
        r, uu = sim.moments()
    mid = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, t0, kernel="scalar")
    assert np.array_equal(r0, mid[0]) and np.array_equal(u0, mid[1])
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])


@pytest.mark.parametrize("kernel", IN_PLACE)
def test_in_place_holds_one_buffer(kernel):
    """With library-owned memory the in-place steps allocate one population
    buffer; reading at odd times (moments, totals, residual, checkpoint) needs
    no second one, and the results equal the two-buffer step's."""
    import torch

    from paper_2002_02503_amd import lbm

    dims = (128, 128, 64)  # 128^2 * 64 * 19 * 4 B = 80 MiB per buffer
    rho, u = _fields(3, dims, seed=12, amp=0.03)
    ref = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, 9, kernel="scalar")
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel=kernel, torch_memory=False) as sim:
        nbytes = sim.info()["state_bytes"]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        sim.init(rho, u).step(9)
        r, uu = sim.moments()
        tot = sim.totals()
        ck = sim.get_state()
        torch.cuda.synchronize()
        used = free0 - torch.cuda.mem_get_info()[0]
        print(f"{kernel}: {used / 2**20:.1f} MiB allocated for a {nbytes / 2**20:.1f} MiB state", flush=True)
        assert used < 1.5 * nbytes
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel="scalar") as other:
        other.set_state(ck)
        assert np.array_equal(other.totals(), tot)
        r2, u2 = other.moments()
        assert np.array_equal(r2, ref[0]) and np.array_equal(u2, ref[1])


TWO_ROW_CASES = [
    ("D3Q19", (256, 6, 4), "fp32", {}),
    ("D3Q19", (70, 10, 6), "fp16", {"collision": "bgk"}),
    ("D3Q19", (64, 2, 3), "fp64", {"theta": 0.5}),
    ("D3Q15", (300, 4, 3), "bf16", {}),
    ("D2Q9", (300, 8, 1), "fp32", {}),
    ("D3Q39", (40, 6, 7), "fp32", {"K": 5}),
    ("D3Q39", (9, 2, 5), "fp32", {}),
]


@pytest.mark.parametrize("lattice,dims,dtype,kw", TWO_ROW_CASES)
def test_two_row_equals_scalar_step(lattice, dims, dtype, kw):
    """Two sites per thread (rows 2j and 2j + 1) compute the bits of the
    one-site step."""
    D = 2 if lattice == "D2Q9" else 3
    rho, u = _fields(D, dims, seed=sum(dims) + 1)
    a = run_gpu(lattice, dims, 0.6, dtype, rho, u, 13, kernel="two_row", **kw)
    b = run_gpu(lattice, dims, 0.6, dtype, rho, u, 13, kernel="scalar", **kw)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_two_row_needs_even_ny():
    from paper_2002_02503_amd import lbm

    with pytest.raises(lbm.LBMError) as e:
        lbm.Simulation("D3Q19", (32, 7, 4), 0.6, kernel="two_row")
    assert e.value.name == "LBM_EINVAL"


def test_switching_kernels_mid_run_keeps_the_bits():
    """lbm_set_kernel on an initialised handle, at odd and even times, between
    the in-place and two-buffer forms: the run continues bit for bit."""
    from paper_2002_02503_amd import lbm

    dims = (64, 6, 5)
    rho, u = _fields(3, dims, seed=21)
    ref = run_gpu("D3Q19", dims, 0.6, "fp32", rho, u, 19, kernel="scalar")
    with lbm.Simulation("D3Q19", dims, 0.6, dtype="fp32", kernel="in_place", torch_memory=False) as sim:
        sim.init(rho, u).step(3)
        for kernel, n in [("scalar", 2), ("twist", 3), ("in_place", 2), ("twist", 2), ("two_row", 3), ("twist", 1),
                          ("twist", 2), ("in_place", 1)]:
            assert lbm.STATUS[sim.lib.lbm_set_kernel(sim.h, lbm.KERNELS[kernel])] == "LBM_OK"
            sim.step(n)
        assert sim.t == 19
        r, uu = sim.moments()
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])


@pytest.mark.parametrize("kernel", IN_PLACE)
@pytest.mark.parametrize("lattice,dims", [("D3Q39", (40, 6, 5)), ("D2Q9", (50, 7, 1)), ("D3Q15", (33, 5, 4)),
                                          ("D3Q39", (2, 1, 5))])
def test_odd_time_checkpoint_every_lattice(lattice, dims, kernel):
    """A checkpoint taken after an odd number of in-place steps (the state is
    then swapped, and lbm_get_state rearranges it on the host) equals the
    two-buffer step's bytes, and resumes bit for bit in either kernel."""
    from paper_2002_02503_amd import lbm

    D = 2 if lattice == "D2Q9" else 3
    rho, u = _fields(D, dims, seed=31)
    with lbm.Simulation(lattice, dims, 0.6, dtype="fp32", kernel=kernel) as ip, \
            lbm.Simulation(lattice, dims, 0.6, dtype="fp32", kernel="scalar") as sc:
        ip.init(rho, u).step(3)
        sc.init(rho, u).step(3)
        ck = ip.get_state()
        assert np.array_equal(ck, sc.get_state())
        sc.step(4)
        ref = sc.moments()
    for other_kernel in IN_PLACE + ["scalar"]:
        with lbm.Simulation(lattice, dims, 0.6, dtype="fp32", kernel=other_kernel) as other:
            other.set_state(ck)
            other.step(4)
            r, uu = other.moments()
        assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1]), other_kernel
