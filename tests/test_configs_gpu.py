"""GPU parity on the five benchmark workloads, at their full sizes.

Where the oracle cannot run the full box, an exact reduction is used:
  * x-only shear waves equal the oracle's nx x 1 x 1 run (pinned on the CPU);
  * x-y Taylor-Green boxes equal the oracle's nx x ny x 1 run;
  * the turbulent box is compared on sampled sites after a few steps through
    the light cone, and over the full 500 steps on the same recipe at 32^3.
"""
import numpy as np
import pytest

import oracle
from gpu_common import BOUND, lightcone_samples, rel_rho, rel_u, run_oracle, sample_points
from lbm_analysis import fit_decay, mode_amplitude
from paper_2002_02503_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def test_d2q9_taylor_green_fp64():
    """D2Q9, 64 x 64, FP64, tau = 0.8, Taylor-Green u0 = 0.05, 1000 steps."""
    n, tau, steps = 64, 0.8, 1000
    rho, u = inputs.taylor_green_2d(n, 0.05, 1.0 / 3.0)
    r_ref, u_ref = run_oracle("D2Q9", (n, n, 1), tau, rho, u, steps)
    with lbm.Simulation("D2Q9", (n, n, 1), tau, dtype="fp64") as sim:
        sim.init(rho, u).step(steps)
        r, uu = sim.moments()
    eu, er = rel_u(uu, u_ref), rel_rho(r, r_ref)
    print(f"D2Q9 TG fp64: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < 1e-12 and er < 1e-12
    k = 2 * np.pi / n
    ratio = np.sqrt(np.mean(uu * uu)) / np.sqrt(np.mean(u * u))
    assert abs(ratio / np.exp(-2 * (tau - 0.5) / 3 * k * k * steps) - 1) < 2e-3


def _shear_gpu(lattice, dims, tau, U, steps, dtype="fp32", every=100, K=None, **kw):
    nx = dims[0]
    rho, u = inputs.shear_wave(dims, 0.01, U)
    ts, amps = [0], [mode_amplitude(u[1, 0, 0] - U[1], nx, axis=0)]
    with lbm.Simulation(lattice, dims, tau, dtype=dtype, K=K, **kw) as sim:
        sim.init(rho, u)
        for t in range(every, steps + 1, every):
            sim.step(every)
            r, uu = sim.moments()
            ts.append(t)
            amps.append(mode_amplitude(uu[1, 0, 0] - U[1], nx, axis=0))
    return r, uu, np.array(ts), np.array(amps)


def _shear_oracle_rate(lattice, nx, tau, U, steps, every=100, K=None):
    sim = oracle.Sim(lattice, (nx, 1, 1), tau, K=K)
    rho, u = inputs.shear_wave((nx, 1, 1), 0.01, U)
    sim.init(rho, u)
    ts, amps = [0], [mode_amplitude(u[1, 0, 0] - U[1], nx, axis=0)]
    for t in range(every, steps + 1, every):
        sim.step(every)
        _, uu = sim.moments()
        ts.append(t)
        amps.append(mode_amplitude(uu[1, 0, 0] - U[1], nx, axis=0))
    return fit_decay(ts, amps)


def test_d3q19_shear_wave_128_fp32():
    """D3Q19, 128^3, FP32, tau = 0.55, shear wave 0.01 on U = (0.1, 0.05, 0),
    2000 steps: parity with the oracle, x-only structure kept bit for bit, the
    decay rate equal to the oracle's, and the Galilean test at full size: the
    paper's operator (K = 3) keeps the decay rate of the U = 0 run far better
    than the zero-velocity filter (K = 2) and than BGK with the second-order
    equilibrium; BGK with the third-order equilibrium is close to the paper's
    operator on this flow (the oracle gives 1.2e-5 against 8.6e-6).  (The
    absolute Galilean error of the paper's operator, ~1e-5, is pinned on the
    oracle; over this horizon the wave decays by only 8%, so FP32 rounding
    limits a rate fit to ~1e-4.)"""
    n, tau, steps, U = 128, 0.55, 2000, (0.1, 0.05, 0.0)
    r, uu, ts, amps = _shear_gpu("D3Q19", (n, n, n), tau, U, steps)
    # the field depends on x only, bit for bit
    assert np.array_equal(uu, np.broadcast_to(uu[:, :1, :1, :], uu.shape))
    assert np.array_equal(r, np.broadcast_to(r[:1, :1, :], r.shape))
    rho1, u1 = inputs.shear_wave((n, 1, 1), 0.01, U)
    r_ref, u_ref = run_oracle("D3Q19", (n, 1, 1), tau, rho1, u1, steps)
    eu, er = rel_u(uu[:, :1, :1, :], u_ref), rel_rho(r[:1, :1, :], r_ref)
    print(f"D3Q19 128^3 shear fp32: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < 1e-5 and er < 1e-5
    g_gpu = fit_decay(ts, amps)
    g_ora = _shear_oracle_rate("D3Q19", n, tau, U, steps)
    print(f"decay rate GPU {g_gpu:.6e} oracle {g_ora:.6e}", flush=True)
    assert abs(g_gpu / g_ora - 1) < 1e-3
    gal = {}
    for key, K, coll in [(3, 3, "filtered"), (2, 2, "filtered"), ("bgk3", 3, "bgk"), ("bgk2", 2, "bgk")]:
        if key == 3:
            tU, aU = ts, amps
        else:
            _, _, tU, aU = _shear_gpu("D3Q19", (n, n, n), tau, U, steps, K=K, collision=coll)
        _, _, t0, a0 = _shear_gpu("D3Q19", (n, n, n), tau, (0.0, 0.0, 0.0), steps, K=K, collision=coll)
        gal[key] = abs(fit_decay(tU, aU) / fit_decay(t0, a0) - 1)
    print(f"Galilean error on the GPU, U = (0.1, 0.05, 0): K=3 {gal[3]:.2e}, K=2 (old filter) {gal[2]:.2e}, "
          f"BGK K=3 {gal['bgk3']:.2e}, BGK K=2 {gal['bgk2']:.2e}", flush=True)
    assert gal[2] > 1e-2 and gal["bgk2"] > 1e-2
    assert gal[3] < 1e-3 and gal[3] < gal[2] / 20
    assert gal["bgk3"] < 1e-3


@pytest.mark.parametrize("dtype", ["fp16", "bf16"])
def test_d3q19_shear_wave_128_16bit(dtype):
    """The 128^3 shear wave on U = (0.1, 0.05, 0), tau = 0.55, 2000 steps, in
    16-bit storage against the oracle's 128 x 1 x 1 run: within the stated
    bound (max |du| over max |u|); also states the error against the wave
    itself, max |du| over max |u_ref - U|."""
    n, tau, steps, U = 128, 0.55, 2000, (0.1, 0.05, 0.0)
    rho, u = inputs.shear_wave((n, n, n), 0.01, U)
    with lbm.Simulation("D3Q19", (n, n, n), tau, dtype=dtype) as sim:
        sim.init(rho, u).step(steps)
        r, uu = sim.moments()
    rho1, u1 = inputs.shear_wave((n, 1, 1), 0.01, U)
    r_ref, u_ref = run_oracle("D3Q19", (n, 1, 1), tau, rho1, u1, steps, mode="closed")
    du = np.abs(uu - u_ref).max()
    wave = np.abs(u_ref - np.asarray(U).reshape(3, 1, 1, 1)).max()
    eu, er = rel_u(uu, np.broadcast_to(u_ref, uu.shape)), rel_rho(r, np.broadcast_to(r_ref, r.shape))
    print(f"D3Q19 128^3 shear {dtype}, 2000 steps: u {eu:.2e} (to the wave {du / wave:.2e}) rho {er:.2e}",
          flush=True)
    assert eu < BOUND[dtype] and er < BOUND[dtype]


def test_d3q19_galilean_128_fp64():
    """The Galilean test of the shear wave on U = (0.1, 0.05, 0) at 128^3 in
    FP64, where rounding no longer limits the rate fit: the paper's operator
    (K = 3) and the zero-velocity filter (K = 2) change the decay rate by the
    same relative amounts as the oracle's runs of the same flow, about 1e-5
    against 3e-2."""
    n, tau, steps, U = 128, 0.55, 2000, (0.1, 0.05, 0.0)
    gal_gpu, gal_ora = {}, {}
    for K in (3, 2):
        _, _, tU, aU = _shear_gpu("D3Q19", (n, n, n), tau, U, steps, dtype="fp64", K=K)
        _, _, t0, a0 = _shear_gpu("D3Q19", (n, n, n), tau, (0.0, 0.0, 0.0), steps, dtype="fp64", K=K)
        gal_gpu[K] = fit_decay(tU, aU) / fit_decay(t0, a0) - 1
        gal_ora[K] = (_shear_oracle_rate("D3Q19", n, tau, U, steps, K=K)
                      / _shear_oracle_rate("D3Q19", n, tau, (0.0, 0.0, 0.0), steps, K=K) - 1)
    print(f"Galilean error FP64 128^3: K=3 GPU {gal_gpu[3]:.3e} oracle {gal_ora[3]:.3e}; "
          f"K=2 GPU {gal_gpu[2]:.3e} oracle {gal_ora[2]:.3e}", flush=True)
    for K in (3, 2):
        assert abs(gal_gpu[K] - gal_ora[K]) < 1e-8, K
    assert abs(gal_gpu[3]) < 3e-5 and abs(gal_gpu[2]) > 1e-2


def test_d3q39_shear_wave_192_fp32():
    """D3Q39 (K = 4), 192^3, FP32, tau = 0.6, shear wave on U = (0.2, 0, 0),
    1000 steps: parity with the oracle, and a smaller Galilean error than
    D3Q19 on the same flow."""
    n, tau, steps, U = 192, 0.6, 1000, (0.2, 0.0, 0.0)
    r, uu, ts, amps = _shear_gpu("D3Q39", (n, n, n), tau, U, steps)
    assert np.array_equal(uu, np.broadcast_to(uu[:, :1, :1, :], uu.shape))
    rho1, u1 = inputs.shear_wave((n, 1, 1), 0.01, U)
    r_ref, u_ref = run_oracle("D3Q39", (n, 1, 1), tau, rho1, u1, steps, mode="closed")
    eu, er = rel_u(uu[:, :1, :1, :], u_ref), rel_rho(r[:1, :1, :], r_ref)
    print(f"D3Q39 192^3 shear fp32: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < 1e-5 and er < 1e-5
    gal = {}
    for lat in ["D3Q39", "D3Q19"]:
        if lat == "D3Q39":
            tU, aU = ts, amps
        else:
            _, _, tU, aU = _shear_gpu(lat, (n, n, n), tau, U, steps)
        _, _, t0, a0 = _shear_gpu(lat, (n, n, n), tau, (0.0, 0.0, 0.0), steps)
        gal[lat] = abs(fit_decay(tU, aU) / fit_decay(t0, a0) - 1)
    print(f"Galilean error at U_x = 0.2: D3Q39 {gal['D3Q39']:.2e}, D3Q19 {gal['D3Q19']:.2e}", flush=True)
    assert gal["D3Q39"] < gal["D3Q19"]


@pytest.mark.parametrize("kernel", ["scalar", "in_place", "twist"])
def test_d3q39_k5_shear_wave_192_fp32(kernel):
    """D3Q39 at K = 5 (the benchmark's variant), 192^3, FP32, shear wave on
    U = (0.2, 0, 0), 200 steps, in the launch the tuner picks for it (the
    in-place step, one x-row per block) and the one-site step: the field stays
    x-only bit for bit and matches the oracle's 192 x 1 x 1 run."""
    n, tau, steps, U = 192, 0.6, 200, (0.2, 0.0, 0.0)
    rho, u = inputs.shear_wave((n, n, n), 0.01, U)
    with lbm.Simulation("D3Q39", (n, n, n), tau, dtype="fp32", K=5, kernel=kernel) as sim:
        sim.init(rho, u).step(steps)
        r, uu = sim.moments()
    assert np.array_equal(uu, np.broadcast_to(uu[:, :1, :1, :], uu.shape))
    rho1, u1 = inputs.shear_wave((n, 1, 1), 0.01, U)
    r_ref, u_ref = run_oracle("D3Q39", (n, 1, 1), tau, rho1, u1, steps, K=5)
    eu, er = rel_u(uu[:, :1, :1, :], u_ref), rel_rho(r[:1, :1, :], r_ref)
    print(f"D3Q39 K=5 192^3 shear fp32 {kernel}: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < 1e-5 and er < 1e-5


@pytest.fixture(scope="module")
def turbulence_256():
    return inputs.turbulence(256)


@pytest.mark.parametrize("dtype", ["fp32", "fp16", "bf16", "fp64"])
def test_turbulence_256_sampled_parity(turbulence_256, dtype):
    """D3Q19, 256^3, tau = 0.51, random-phase turbulence: after 3 steps at full
    size, 48 sampled sites match the oracle's light-cone values."""
    rho, u = turbulence_256
    steps, tau = 3, 0.51
    pts = sample_points(rho.shape, 48, seed=1)
    r_ref, u_ref = lightcone_samples("D3Q19", rho, u, tau, steps, pts)
    with lbm.Simulation("D3Q19", (256, 256, 256), tau, dtype=dtype) as sim:
        sim.init(rho, u).step(steps)
        r, uu = sim.moments()
    idx = tuple(np.array(pts).T)
    got_u = uu[(slice(None),) + idx]
    eu = float(np.abs(got_u - u_ref).max() / np.abs(u).max())
    er = float(np.abs(r[idx] - r_ref).max())
    print(f"turbulence 256^3 {dtype}, {steps} steps, sampled: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < BOUND[dtype] and er < BOUND[dtype]


# the benchmark's variants on the headline box: (lattice, library keywords, oracle keywords)
VARIANT_CASES = [
    ("D3Q19", {"collision": "bgk"}, {"kind": "bgk"}),
    ("D3Q19", {"theta": 0.5}, {"theta": 0.5, "mode": "literal"}),
    ("D3Q19", {"K": 2}, {"K": 2}),
    ("D3Q15", {}, {}),
]


@pytest.mark.parametrize("kernel", ["scalar", "in_place", "twist", "two_step"])
@pytest.mark.parametrize("lattice,lib_kw,ora_kw", VARIANT_CASES)
def test_turbulence_256_sampled_parity_variants(turbulence_256, lattice, lib_kw, ora_kw, kernel):
    """The benchmark's other collision kinds and D3Q15 on the full 256^3
    turbulence box, FP32, in the launches the tuner picks for them: after 3
    steps, 24 sampled sites match the oracle's light-cone values."""
    rho, u = turbulence_256
    steps, tau = 3, 0.51
    pts = sample_points(rho.shape, 24, seed=2)
    r_ref, u_ref = lightcone_samples(lattice, rho, u, tau, steps, pts, **ora_kw)
    with lbm.Simulation(lattice, (256, 256, 256), tau, dtype="fp32", kernel=kernel, **lib_kw) as sim:
        sim.init(rho, u).step(steps)
        r, uu = sim.moments()
    idx = tuple(np.array(pts).T)
    eu = float(np.abs(uu[(slice(None),) + idx] - u_ref).max() / np.abs(u).max())
    er = float(np.abs(r[idx] - r_ref).max())
    print(f"{lattice} {lib_kw} {kernel} 256^3, {steps} steps, sampled: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < BOUND["fp32"] and er < BOUND["fp32"]


@pytest.fixture(scope="module")
def turbulence_256_samples(turbulence_256):
    rho, u = turbulence_256
    pts = sample_points(rho.shape, 48, seed=1)
    r_ref, u_ref = lightcone_samples("D3Q19", rho, u, 0.51, 3, pts)
    return pts, r_ref, u_ref


@pytest.mark.parametrize("kernel", ["in_place", "two_row", "twist", "two_step"])
@pytest.mark.parametrize("dtype", ["fp32", "fp16", "bf16", "fp64"])
def test_turbulence_256_sampled_parity_other_kernels(turbulence_256, turbulence_256_samples, kernel, dtype):
    """The same full-size check for the kernel forms the tuner may pick for the
    benchmark (after 3 steps the in-place state is in its swapped layout)."""
    rho, u = turbulence_256
    pts, r_ref, u_ref = turbulence_256_samples
    with lbm.Simulation("D3Q19", (256, 256, 256), 0.51, dtype=dtype, kernel=kernel) as sim:
        sim.init(rho, u).step(3)
        r, uu = sim.moments()
    idx = tuple(np.array(pts).T)
    eu = float(np.abs(uu[(slice(None),) + idx] - u_ref).max() / np.abs(u).max())
    er = float(np.abs(r[idx] - r_ref).max())
    print(f"turbulence 256^3 {dtype} {kernel}, 3 steps, sampled: u {eu:.2e} rho {er:.2e}", flush=True)
    assert eu < BOUND[dtype] and er < BOUND[dtype]


def test_turbulence_256_full_horizon_invariants(turbulence_256):
    """500 steps at full size in FP32: global mass and momentum conserved
    (FP64 totals on the GPU), kinetic energy decays monotonically."""
    rho, u = turbulence_256
    with lbm.Simulation("D3Q19", (256, 256, 256), 0.51, dtype="fp32") as sim:
        sim.init(rho, u)
        t0 = sim.totals()[0]
        energies = []
        for _ in range(5):
            sim.step(100)
            _, uu = sim.moments()
            energies.append(float(np.mean(uu * uu)))
        t1 = sim.totals()[0]
    mass = t0[0]
    print(f"mass drift {abs(t1[0] - t0[0]) / mass:.2e}, momentum drift "
          f"{np.abs(t1[1:] - t0[1:]).max() / mass:.2e}, energies {energies}", flush=True)
    # conserved to single-precision round-off (FP32 epsilon 6e-8)
    assert abs(t1[0] - t0[0]) / mass < 1e-8
    assert np.abs(t1[1:] - t0[1:]).max() / mass < 1e-8
    assert all(b < a for a, b in zip(energies, energies[1:]))


@pytest.mark.parametrize("dtype", ["fp32", "fp16", "bf16"])
def test_turbulence_recipe_32_full_horizon(dtype):
    """The same turbulence recipe (k0 = 4, u_rms = 0.04, tau = 0.51) at 32^3
    for the full 500 steps against the oracle; states the storage error."""
    rho, u = inputs.turbulence(32)
    r_ref, u_ref = run_oracle("D3Q19", (32, 32, 32), 0.51, rho, u, 500, mode="closed")
    with lbm.Simulation("D3Q19", (32, 32, 32), 0.51, dtype=dtype) as sim:
        sim.init(rho, u).step(500)
        r, uu = sim.moments()
    eu, er = rel_u(uu, u_ref), rel_rho(r, r_ref)
    l2 = float(np.sqrt(np.sum((uu - u_ref) ** 2) / np.sum(u_ref ** 2)))
    print(f"turbulence 32^3 500 steps {dtype}: u max {eu:.2e} u L2 {l2:.2e} rho {er:.2e}", flush=True)
    assert eu < BOUND[dtype] and er < BOUND[dtype]


def test_batched_256_boxes_fp32():
    """256 independent D3Q19 boxes (sides 16..64, own tau and U), Taylor-Green
    in x-y, FP32, 1000 steps as graph launches: every box keeps its z-invariance
    bit for bit and conserves mass and momentum; 16 boxes match the oracle's
    nx x ny x 1 runs; a batched box equals the same box run alone, bit for
    bit."""
    boxes = inputs.batch_boxes()
    T0, steps = 1.0 / 3.0, 1000
    dims = [b["dims"] for b in boxes]
    taus = [b["tau"] for b in boxes]
    fields = [inputs.taylor_green_box(b["dims"], b["U"], T0) for b in boxes]
    rho = np.concatenate([f[0].ravel() for f in fields])
    u = np.concatenate([f[1].reshape(3, -1) for f in fields], axis=1)
    with lbm.Simulation("D3Q19", dims, taus, dtype="fp32") as sim:
        sim.init(rho, u)
        tot0 = sim.totals()
        sim.step(steps)
        tot1 = sim.totals()
        r, uu = sim.moments()
    rb = sim.split_boxes(r)
    ub = sim.split_boxes(uu)
    for k in range(len(boxes)):
        assert np.array_equal(ub[k], np.broadcast_to(ub[k][:, :1], ub[k].shape)), k
    mass = tot0[:, 0]
    dm = np.abs(tot1[:, 0] - mass) / mass
    dp = np.abs(tot1[:, 1:] - tot0[:, 1:]).max(axis=1) / mass
    print(f"batched: worst mass drift {dm.max():.2e}, momentum drift {dp.max():.2e}", flush=True)
    # Single-precision round-off only: each step rounds every stored value to
    # FP32 (epsilon 6e-8); even if all of it added up, 1000 steps at |u| <= 0.2
    # would drift by steps * epsilon * 0.2 = 1.2e-5.  A collision that broke
    # conservation would drift by O(|u|^2) = 1e-3 or more.
    assert np.all(dm < 1e-6) and np.all(dp < 1e-6)
    worst = 0.0
    for k in range(0, len(boxes), 16):
        nx, ny, nz = boxes[k]["dims"]
        r1, u1 = inputs.taylor_green_box((nx, ny, 1), boxes[k]["U"], T0)
        r_ref, u_ref = run_oracle("D3Q19", (nx, ny, 1), boxes[k]["tau"], r1, u1, steps, mode="closed")
        worst = max(worst, rel_u(ub[k][:, :1], u_ref), rel_rho(rb[k][:1], r_ref))
    print(f"batched: worst box error vs oracle {worst:.2e}", flush=True)
    assert worst < 1e-5
    for k in [0, 100, 255]:
        with lbm.Simulation("D3Q19", boxes[k]["dims"], boxes[k]["tau"], dtype="fp32") as one:
            one.init(fields[k][0], fields[k][1]).step(steps)
            r1, u1 = one.moments()
        # the batched and single-box kernels compute the same bits
        assert np.array_equal(u1, ub[k]) and np.array_equal(r1, rb[k]), k


def _progress(capfd, msg: str) -> None:
    """A progress line written past pytest's output capture, so that a long
    host-side run keeps printing while it works."""
    with capfd.disabled():
        print(msg, flush=True)


def test_turbulence_256_full_horizon_error(turbulence_256, capfd):
    """The headline workload at its own configuration: D3Q19, 256^3, tau =
    0.51, decaying turbulence, 500 steps, every storage type against the
    oracle's full 256^3 run (closed mode, pinned equal to the literal mode, on
    all host threads).  States max and L2 errors of u and rho (max |du| over
    max |u|, ||du||_2 over ||u||_2, max |drho|, ||drho||_2 over ||rho||_2) and
    asserts the stated bound of each storage type on the velocity and density
    maxima.  The two-step kernel (which the tuner picks for FP64 and FP32 on
    this box) gives the same bits over the 500 steps."""
    rho, u = turbulence_256
    tau, steps, every = 0.51, 500, 25
    got = {}
    for dtype in ["fp64", "fp32", "fp16", "bf16"]:
        with lbm.Simulation("D3Q19", (256, 256, 256), tau, dtype=dtype) as sim:
            sim.init(rho, u).step(steps)
            got[dtype] = sim.moments()
        _progress(capfd, f"full-horizon error: GPU {dtype} 500 steps done")
        if dtype in ("fp64", "fp32"):
            with lbm.Simulation("D3Q19", (256, 256, 256), tau, dtype=dtype, kernel="two_step") as sim:
                sim.init(rho, u).step(steps)
                r2, u2 = sim.moments()
            assert np.array_equal(r2, got[dtype][0]) and np.array_equal(u2, got[dtype][1]), dtype
            _progress(capfd, f"full-horizon error: GPU {dtype} two-step kernel bit-identical")
    sim = oracle.Sim("D3Q19", (256, 256, 256), tau, mode="closed").init(rho, u)
    for t in range(every, steps + 1, every):
        sim.step(every)
        _progress(capfd, f"full-horizon error: oracle at step {t} of {steps} ({oracle.get_threads()} threads)")
    r_ref, u_ref = sim.moments()
    del sim
    umax = np.abs(u_ref).max()
    u_l2 = np.sqrt(np.sum(u_ref * u_ref))
    r_l2 = np.sqrt(np.sum(r_ref * r_ref))
    bad = []
    for dtype, (r, uu) in got.items():
        du = uu - u_ref
        dr = r - r_ref
        e = {"u_max": float(np.abs(du).max() / umax), "u_l2": float(np.sqrt(np.sum(du * du)) / u_l2),
             "rho_max": float(np.abs(dr).max()), "rho_l2": float(np.sqrt(np.sum(dr * dr)) / r_l2)}
        print(f"FULL HORIZON 256^3 500 steps {dtype}: u max {e['u_max']:.3e} u L2 {e['u_l2']:.3e} "
              f"rho max {e['rho_max']:.3e} rho L2 {e['rho_l2']:.3e} (bound {BOUND[dtype]:g})", flush=True)
        _progress(capfd, f"full-horizon error {dtype}: {e}")
        if not (e["u_max"] < BOUND[dtype] and e["rho_max"] < BOUND[dtype]):
            bad.append(dtype)
    assert not bad, bad
