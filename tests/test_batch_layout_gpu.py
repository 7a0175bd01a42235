"""The batched step in its blocked layout (64-site blocks of each box, any
row length) against the same boxes run alone in the row-tiled single-box
layout: the same bits for every box shape, lattice, storage type, collision
kind and launch shape; graphs, checkpoints and poisoned buffers; the
documented layout decoded on the host; and parity with the oracle."""
import numpy as np
import pytest

from gpu_common import BOUND, rel_rho, rel_u, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

# Box shapes around the blocking rules: rows of 1, 2, 16, 20, 33, 40, 64, 65
# and 100 sites; boxes shorter than one block (1 x 3 x 4, 2 x 5 x 3) and
# boxes whose size is not a multiple of 64 (the last block is partial).
MIXED = [(1, 3, 4), (2, 5, 3), (16, 7, 3), (20, 6, 5), (33, 4, 3), (40, 5, 2), (64, 3, 3), (65, 2, 3),
         (100, 3, 2)]

STORED_SCALE = {"D2Q9": 36, "D3Q15": 72, "D3Q19": 36, "D3Q39": 6480}
NP_DTYPE = {"fp64": np.float64, "fp32": np.float32, "fp16": np.float16}


def _batch_fields(D, dims, seed):
    rng = np.random.default_rng(seed)
    n = sum(a * b * c for a, b, c in dims)
    return 1.0 + rng.uniform(-0.01, 0.01, n), rng.uniform(-0.05, 0.05, (D, n))


def _box_fields(dims, rho, u, k):
    off = sum(a * b * c for a, b, c in dims[:k])
    nx, ny, nz = dims[k]
    n = nx * ny * nz
    return rho[off:off + n].reshape(nz, ny, nx), u[:, off:off + n].reshape(-1, nz, ny, nx)


def _run_batch(lattice, dims, taus, dtype, rho, u, steps, **kw):
    from paper_2002_02503_amd import lbm

    with lbm.Simulation(lattice, dims, taus, dtype=dtype, **kw) as sim:
        sim.init(rho, u).step(steps)
        r, uu = sim.moments()
        return sim.split_boxes(r), sim.split_boxes(uu)


CASES = [
    ("D3Q19", "fp32", {}),
    ("D3Q19", "fp16", {}),
    ("D3Q19", "bf16", {"collision": "bgk"}),
    ("D3Q19", "fp64", {"theta": 0.5}),
    ("D3Q15", "fp32", {}),
    ("D3Q39", "fp32", {"K": 5}),
    ("D3Q39", "fp64", {}),
]


@pytest.mark.parametrize("lattice,dtype,kw", CASES)
@pytest.mark.parametrize("block", [64, 256])
def test_batch_equals_boxes_run_alone(lattice, dtype, kw, block):
    taus = list(np.linspace(0.55, 0.95, len(MIXED)))
    rho, u = _batch_fields(3, MIXED, seed=block + len(lattice))
    rb, ub = _run_batch(lattice, MIXED, taus, dtype, rho, u, 9, block=block, **kw)
    for k, d in enumerate(MIXED):
        r0, u0 = _box_fields(MIXED, rho, u, k)
        r1, u1 = run_gpu(lattice, d, taus[k], dtype, r0, u0, 9, **kw)
        assert np.array_equal(rb[k], r1) and np.array_equal(ub[k], u1), d


def test_d2q9_batch_and_persistent_grid():
    """D2Q9 boxes (one plane), and grids smaller than the tile count, so that
    each wave walks several tiles."""
    dims = [(d[0], d[1], 1) for d in MIXED]
    taus = [0.6] * len(dims)
    rho, u = _batch_fields(2, dims, seed=4)
    ref = _run_batch("D2Q9", dims, taus, "fp32", rho, u, 11)
    for block, grid in [(128, 3), (64, 1), (256, 1024)]:
        got = _run_batch("D2Q9", dims, taus, "fp32", rho, u, 11, block=block, grid=grid)
        for k in range(len(dims)):
            assert np.array_equal(got[0][k], ref[0][k]) and np.array_equal(got[1][k], ref[1][k])
    for k, d in enumerate(dims):
        r0, u0 = _box_fields(dims, rho, u, k)
        r1, u1 = run_gpu("D2Q9", d, taus[k], "fp32", r0, u0, 11)
        assert np.array_equal(ref[0][k], r1) and np.array_equal(ref[1][k], u1), d


def test_aligned_rows_batch():
    """Every box with nx a multiple of 64 (the launch that streams the c_x = 0
    populations non-temporally) equals its boxes run alone."""
    dims = [(64, 3, 4), (128, 2, 3), (64, 5, 1)]
    taus = [0.6, 0.7, 0.8]
    rho, u = _batch_fields(3, dims, seed=9)
    rb, ub = _run_batch("D3Q19", dims, taus, "fp32", rho, u, 10)
    for k, d in enumerate(dims):
        r0, u0 = _box_fields(dims, rho, u, k)
        r1, u1 = run_gpu("D3Q19", d, taus[k], "fp32", r0, u0, 10)
        assert np.array_equal(rb[k], r1) and np.array_equal(ub[k], u1), d


def test_batch_in_graphs():
    dims = MIXED[:6]
    taus = [0.6, 0.7, 0.8, 0.9, 0.65, 0.75]
    rho, u = _batch_fields(3, dims, seed=6)
    a = _run_batch("D3Q19", dims, taus, "fp32", rho, u, 23, graph_chunk=4)
    b = _run_batch("D3Q19", dims, taus, "fp32", rho, u, 23, graph_chunk=1)
    for k in range(len(dims)):
        assert np.array_equal(a[0][k], b[0][k]) and np.array_equal(a[1][k], b[1][k])


def test_batch_matches_oracle():
    """Each box of a batch against the oracle run of that box alone."""
    dims = [(20, 6, 5), (16, 4, 4), (40, 3, 4), (7, 9, 3)]
    taus = [0.6, 0.7, 0.85, 0.55]
    rho, u = _batch_fields(3, dims, seed=7)
    rb, ub = _run_batch("D3Q19", dims, taus, "fp32", rho, u, 17)
    for k, d in enumerate(dims):
        r0, u0 = _box_fields(dims, rho, u, k)
        r_ref, u_ref = run_oracle("D3Q19", d, taus[k], r0, u0, 17, mode="closed")
        assert rel_u(ub[k], u_ref) < BOUND["fp32"] and rel_rho(rb[k], r_ref) < BOUND["fp32"]


def test_batch_checkpoint_and_poisoned_buffers():
    """Both buffers filled with NaN bytes before init: the results and the
    checkpoint bytes (padding included) equal those of a clean run; a batch
    checkpoint resumes bit for bit; its size counts whole 64-site blocks."""
    from paper_2002_02503_amd import lbm

    dims = MIXED
    taus = list(np.linspace(0.55, 0.95, len(dims)))
    rho, u = _batch_fields(3, dims, seed=8)
    with lbm.Simulation("D3Q19", dims, taus, dtype="fp32") as clean:
        clean.init(rho, u).step(7)
        ck = clean.get_state()
        clean.step(5)
        ref = clean.moments()
    padded = sum(-(-(a * b * c) // 64) * 64 for a, b, c in dims)
    assert ck.size == 64 + 19 * 4 * padded
    with lbm.Simulation("D3Q19", dims, taus, dtype="fp32") as dirty:
        for b in dirty._bufs:
            b.fill_(0xFF)
        dirty.init(rho, u).step(7)
        assert np.array_equal(dirty.get_state(), ck)
        dirty.step(5)
        r, uu = dirty.moments()
    assert np.isfinite(r).all() and np.isfinite(uu).all()
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])
    with lbm.Simulation("D3Q19", dims, taus, dtype="fp32") as other:
        for b in other._bufs:
            b.fill_(0xFF)
        other.set_state(ck)
        assert other.t == 7
        other.step(5)
        r, uu = other.moments()
        ck2 = other.get_state()
    assert np.array_equal(r, ref[0]) and np.array_equal(uu, ref[1])
    payload = ck2[64:].view(np.float32)
    assert np.isfinite(payload).all()


@pytest.mark.parametrize("lattice,dtype", [("D3Q19", "fp32"), ("D3Q39", "fp64"), ("D2Q9", "fp16"),
                                           ("D3Q15", "fp32")])
def test_checkpoint_layout_as_documented(lattice, dtype):
    """Decode a batch checkpoint with the layout stated in the header (blocks
    of 64 sites, Q runs of 64 per block in tile-row order, boxes padded to
    whole blocks, stored values S (f_i - w_i)): its density and velocity equal
    the library's moments, and the padding is zero."""
    from paper_2002_02503_amd import lbm

    tab = lbm.lattice_table(lattice)
    D, Q, c = tab["D"], tab["Q"], tab["c"]
    c3 = np.zeros((Q, 3), dtype=np.int64)
    c3[:, :D] = c
    order = sorted(range(Q), key=lambda i: (c3[i, 2], c3[i, 1], c3[i, 0]))
    mrow = np.empty(Q, dtype=np.int64)
    mrow[order] = np.arange(Q)
    dims = [(d[0], d[1], 1) for d in MIXED] if D == 2 else MIXED
    taus = [0.7] * len(dims)
    rho, u = _batch_fields(D, dims, seed=10)
    with lbm.Simulation(lattice, dims, taus, dtype=dtype) as sim:
        sim.init(rho, u).step(3)
        ck = sim.get_state()
        r_lib, u_lib = sim.moments()
    vals = ck[64:].view(NP_DTYPE[dtype]).astype(np.float64)
    S = STORED_SCALE[lattice]
    base = 0
    rho_dec, j_dec = [], []
    for nx, ny, nz in dims:
        n = nx * ny * nz
        nblk = -(-n // 64)
        box = vals[base:base + nblk * 64 * Q].reshape(nblk, Q, 64)
        base += nblk * 64 * Q
        l = np.arange(n)
        G = box[l // 64, :, l % 64][:, mrow]  # G[s, i]: population i of site s
        pad_l = np.arange(n, nblk * 64)
        assert np.all(box[pad_l // 64, :, pad_l % 64] == 0)
        rho_dec.append(1.0 + G.sum(axis=1) / S)
        j_dec.append((G @ c3[:, :D]).T / S)
    assert base == vals.size
    r_dec = np.concatenate(rho_dec)
    u_dec = np.concatenate(j_dec, axis=1) / r_dec
    assert np.allclose(r_dec, r_lib, rtol=0, atol=1e-13)
    assert np.allclose(u_dec, u_lib.reshape(D, -1), rtol=0, atol=1e-13)


def test_batch_box_limits():
    """A batch box longer than 2^21 sites along x is rejected before any
    device work (the batched step's site split is exact below that)."""
    from paper_2002_02503_amd import lbm

    with pytest.raises(lbm.LBMError) as e:
        lbm.Simulation("D3Q19", [(2 ** 21 + 1, 1, 1), (8, 8, 8)], [0.6, 0.7])
    assert e.value.name == "LBM_EINVAL"
    dims = [(2 ** 21, 1, 1), (3, 2, 2)]
    rho, u = _batch_fields(3, dims, seed=12)
    rb, ub = _run_batch("D3Q19", dims, [0.6, 0.7], "fp32", rho, u, 3)
    for k, d in enumerate(dims):
        r0, u0 = _box_fields(dims, rho, u, k)
        r1, u1 = run_gpu("D3Q19", d, [0.6, 0.7][k], "fp32", r0, u0, 3)
        assert np.array_equal(rb[k], r1) and np.array_equal(ub[k], u1), d


def test_size_limits_are_refused_before_allocation():
    """The documented limits of lbm_create / lbm_create_batch, each refused
    with LBM_EINVAL before any device memory is touched: ny and nz at most
    65535 with ny * nz below 2^31 (32-bit row indices), a population row
    below 2 GiB (32-bit lane offsets), at most 2^36 sites, and less than 2 GiB
    of populations per batch box (the batched kernel's 32-bit offsets)."""
    from paper_2002_02503_amd import lbm

    cases = [
        ("D3Q19", (1, 65536, 1), "fp32"),               # ny > 65535
        ("D3Q19", (1, 1, 65536), "fp32"),               # nz > 65535
        ("D3Q19", (1, 65535, 65535), "fp32"),           # ny * nz >= 2^31
        ("D2Q9", (2 ** 28, 1, 1), "fp64"),              # 2 GiB population rows
        ("D3Q19", (2 ** 20, 256, 65535), "fp16"),       # more than 2^36 sites
    ]
    for lattice, dims, dtype in cases:
        with pytest.raises(lbm.LBMError) as e:
            lbm.Simulation(lattice, dims, 0.6, dtype=dtype, torch_memory=False)
        assert e.value.name == "LBM_EINVAL", dims
    big = (1024, 1024, 14)  # 14.7 M sites * 19 * 8 B = 2.2 GiB in FP64
    with pytest.raises(lbm.LBMError) as e:
        lbm.Simulation("D3Q19", [big, (8, 8, 8)], [0.6, 0.7], dtype="fp64")
    assert e.value.name == "LBM_EINVAL" and "2 GiB" in str(e.value)
    # accepted, nothing allocated yet: the same box alone (64-bit row
    # offsets), a 2^31-site box and a 2^28-site row in FP32
    for dims, dtype in [(big, "fp64"), ((2 ** 11, 2 ** 10, 2 ** 10), "fp32"), ((2 ** 28, 1, 1), "fp32")]:
        lattice = "D2Q9" if dims[1:] == (1, 1) else "D3Q19"
        with lbm.Simulation(lattice, dims, 0.6, dtype=dtype, torch_memory=False) as sim:
            assert sim.info()["nsites"] == dims[0] * dims[1] * dims[2]


@pytest.mark.parametrize("kernel", ["in_place", "twist", "two_step"])
def test_box_of_more_than_2_31_sites(kernel):
    """A single D3Q19 box of 2^31 + 2^20 sites (1024 x 1024 x 2049), FP16, in
    place (82 GB of populations, fields on the device), or with the two-step
    kernel (two buffers, 164 GB; its z-planes start past 4 GiB).  The field
    varies along x and z (u_x along z, u_y along x), so a site index that
    wrapped at 32 bits would land on a site with other values: after the steps
    the field is y-independent bit for bit and equals the 1024 x 1 x 2049 box's
    run (one-site step for the two-step case, whose tile needs ny >= 8), and the
    FP64 totals are ny times that box's."""
    import torch

    from paper_2002_02503_amd import lbm

    nx, ny, nz = 1024, 1024, 2049
    U, tau, steps = (0.05, 0.02, -0.03), 0.6, 5

    def fields(ny_, dev):
        lib = torch if dev else np
        kw = {"dtype": torch.float64, "device": "cuda"} if dev else {}
        x = lib.arange(nx, **kw) if dev else np.arange(nx, dtype=np.float64)
        z = lib.arange(nz, **kw) if dev else np.arange(nz, dtype=np.float64)
        shape = (nz, ny_, nx)
        rho = torch.ones(shape, **kw) if dev else np.ones(shape)
        u = torch.empty((3,) + shape, **kw) if dev else np.empty((3,) + shape)
        u[0] = U[0] + 0.01 * lib.sin(2 * np.pi * z / nz)[:, None, None]
        u[1] = U[1] + 0.01 * lib.sin(2 * np.pi * x / nx)[None, None, :]
        u[2] = U[2]
        return rho, u

    with lbm.Simulation("D3Q19", (nx, ny, nz), tau, dtype="fp16", kernel=kernel, torch_memory=False) as sim:
        assert sim.info()["nsites"] > 2 ** 31
        rho, u = fields(ny, True)
        sim.init(rho, u)  # synchronises: the fields can go before the outputs are made
        del rho, u
        torch.cuda.empty_cache()
        sim.step(steps)
        tot = sim.totals()[0]
        r, uu = sim.moments(device=True)
    assert torch.equal(uu, uu[:, :, :1, :].expand_as(uu))
    assert torch.equal(r, r[:, :1, :].expand_as(r))
    slab_u, slab_r = uu[:, :, 0, :].cpu().numpy(), r[:, 0, :].cpu().numpy()
    del r, uu
    torch.cuda.empty_cache()
    rho1, u1 = fields(1, False)
    with lbm.Simulation("D3Q19", (nx, 1, nz), tau, dtype="fp16",
                        kernel="scalar" if kernel == "two_step" else kernel) as one:
        one.init(rho1, u1).step(steps)
        tot1 = one.totals()[0]
        r1, uu1 = one.moments()
    assert np.array_equal(slab_u, uu1[:, :, 0, :]) and np.array_equal(slab_r, r1[:, 0, :])
    # the reductions over 2^31 + 2^20 sites: ny copies of the slab's totals
    assert abs(tot[0] / (ny * tot1[0]) - 1) < 1e-12
    assert np.all(np.abs(tot[1:] - ny * tot1[1:]) <= 1e-12 * tot[0])
