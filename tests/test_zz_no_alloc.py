"""GPU test of the allocation-free residual (lbm_residual_noalloc) against
lbm_residual, called through the C ABI on two handles in a row, the second
smaller than the first and in the in-place step's swapped layout."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(lattice, dims, tau, dtype, steps, kernel="auto", seed=0):
    import torch

    from paper_2002_02503_amd import lbm

    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    D = 2 if lattice == "D2Q9" else 3
    u0 = rng.uniform(-0.05, 0.05, size=(D, nz, ny, nx))
    r0 = 1.0 + rng.uniform(-0.01, 0.01, size=(nz, ny, nx))
    with lbm.Simulation(lattice, dims, tau, dtype=dtype, kernel=kernel) as sim:
        sim.init(r0, u0).step(steps)
        ref_r = torch.from_numpy(r0).cuda()
        ref_u = torch.from_numpy(u0).cuda()
        want = sim.residual(ref_r, ref_u)
        out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        sim.residual_noalloc(ref_r, ref_u, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    print(f"noalloc {lattice} {dims} {dtype} {kernel} t={steps}: {got.tolist()} vs {list(want.values())}", flush=True)
    w = np.array([want["u_max"], want["u_l2"], want["rho_max"], want["rho_l2"]])
    assert np.all(w > 0)
    # the maxima are the same reduction in the same order: equal bits; the L2
    # norms take the square root on the GPU instead of the host
    assert got[0] == w[0] and got[2] == w[2]
    assert np.all(np.abs(got[[1, 3]] - w[[1, 3]]) <= 2e-16 * w[[1, 3]])


def test_noalloc_residual_matches_residual_on_two_handles():
    # several reduction chunks with a ragged last one, then a smaller box whose
    # in-place state is in the swapped layout (odd step count)
    _case("D3Q19", (48, 40, 36), 0.6, "fp32", 7, seed=1)
    _case("D3Q19", (20, 12, 9), 0.8, "fp16", 5, kernel="in_place", seed=2)
    _case("D2Q9", (33, 17, 1), 0.7, "fp64", 4, seed=3)


def test_noalloc_residual_refuses_handles_beyond_its_scratch():
    from paper_2002_02503_amd import lbm

    # 2^28 + 4096 sites: 65537 reduction chunks, one more than the scratch holds
    import ctypes

    # no population memory is allocated: the handle is never initialised, and
    # the size check comes before anything else is looked at
    with lbm.Simulation("D3Q19", (4096, 4097, 16), 0.6, dtype="fp16", torch_memory=False) as sim:
        dummy = ctypes.c_void_p(256)
        with pytest.raises(lbm.LBMError) as e:
            lbm._check(sim.lib.lbm_residual_noalloc(sim.h, dummy, dummy, dummy))
        assert e.value.name == "LBM_EINVAL" and "scratch" in str(e.value)
