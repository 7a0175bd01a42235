#!/usr/bin/env python3
"""Benchmark of the fused stream + filtered-collision step on one MI355X.

Workload (the headline): D3Q19, 256^3 periodic box, tau = 0.51, decaying
turbulence from a seeded random-phase field (k0 = 4, u_rms = 0.04), FP32
storage; FP16 and BF16 storage of the deviations, the batched form (256 boxes)
and D3Q39 (192^3) are reported beside it.  A "step" is one application of the
lattice Boltzmann equation to every site; the two-step kernel, where the tuner
picks it, takes two steps per launch, and per-launch figures (roofline bytes,
counter traffic) then count both.  Inputs are resident in HBM before
the timed region.  Each measurement sets the handle's graph chunk to
min(K, 4096) and builds its step graphs beforehand, so the K timed steps are
one captured-graph launch (K <= 4096); the W warm-up steps before them, fewer
than one chunk, are direct launches.  The timed region is bracketed by device
synchronisation and timed with HIP events on the stream the kernels run on.
Every measurement records its graph chunk and how many graph and direct
launches its timed steps took.

Error statements (errors, and "error" in each variant) compare the GPU's
fields with the FP64 oracle's on the same seeded inputs, on the full box where
the oracle can run it in the time budget, else on exact reductions of the flow
(x-only shear waves as nx x 1 x 1 runs, x-y Taylor-Green boxes as nx x ny x 1
runs) or on light-cone samples.  Norms: max |du| / max |u_ref|, ||du||_2 /
||u_ref||_2, max |drho|, ||drho||_2 / ||rho_ref||_2, and for waves on a
background U also max |du| / max |u_ref - U|.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline, D3Q19 256³ FP32 vs FP16-storage at stated error"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak
def traffic_file(kernel: str, workload: str = "turbulence256", dtype: str = "fp32") -> str:
    """Committed counter summary of the step for one kernel variant, on the
    headline box (in one storage type), the 256-box batch or the D3Q39 box."""
    if workload == "batch256":
        return os.path.join(ROOT, "profiles", f"traffic_batch256_{dtype}.json")
    if workload == "d3q39_192":
        return os.path.join(ROOT, "profiles", f"traffic_d3q39_192_fp32_{kernel}.json")
    return os.path.join(ROOT, "profiles", f"traffic_d3q19_256_{dtype}_{kernel}.json")
# what decides the step kernel's machine code: its sources and the compiler flags
def _kernel_sources() -> list:
    """Every source that goes into the device code (all of csrc/ except the
    host-only C-ABI and host-helper files), and the build flags."""
    csrc = os.path.join(ROOT, "paper_2002_02503_amd", "csrc")
    names = sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".hpp")) and n not in ("api.hip", "host.hpp"))
    return [f"csrc/{n}" for n in names] + ["build.py"]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the kernel sources and build flags, to tell whether stored
    counters still apply."""
    h = hashlib.sha256()
    for name in _kernel_sources():
        with open(os.path.join(ROOT, "paper_2002_02503_amd", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def timed_steps(sim, steps: int, warmup: int) -> float:
    """Milliseconds per step over `steps` steps after `warmup` untimed ones."""
    import torch

    sim.prepare()
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


KERNEL_NAMES = {1: "scalar", 2: "row_wave", 3: "in_place", 4: "two_row", 5: "twist", 6: "two_step"}
KERNEL_SYMBOLS = {"scalar": "k_step", "row_wave": "k_step_vec", "in_place": "k_step_ip", "two_row": "k_step_pair",
                  "twist": "k_step_tw", "two_step": "k_step2"}
# time steps one launch of a kernel takes (the two-step kernel: two; per-launch
# figures count both)
STEPS_PER_LAUNCH = {"two_step": 2}
STORAGE_CTYPE = {"fp64": "double", "fp32": "float", "fp16": "_Float16", "bf16": "bf16_t"}


MAX_GRAPH_CHUNK = 4096


GRAPH_CHUNK = None  # --graph-chunk: steps per captured graph (None: min(steps, 4096))


def measure_box(lattice, dims, tau, dtype, rho, u, steps, warmup, tune=True, **kw):
    """Create, initialise, autotune the launch (outside the timed region, state
    restored), then time `steps` steps, issued as graphs of min(steps, 4096)
    steps.  The FP64 totals (lbm_totals) before and after give the mass and
    momentum drift over all the steps taken."""
    import numpy as np

    from paper_2002_02503_amd import lbm

    chunk = min(steps, MAX_GRAPH_CHUNK) if GRAPH_CHUNK is None else GRAPH_CHUNK
    with lbm.Simulation(lattice, dims, tau, dtype=dtype, graph_chunk=chunk, **kw) as sim:
        t0 = time.perf_counter()
        sim.init(rho, u)  # host fields in, synchronises
        init_ms = (time.perf_counter() - t0) * 1e3
        tot0 = sim.totals()
        if tune:
            sim.tune(steps=20)
        ms = timed_steps(sim, steps, warmup)
        tot1 = sim.totals()
        t0 = time.perf_counter()
        sim.moments()  # host fields out, synchronises
        moments_ms = (time.perf_counter() - t0) * 1e3
        info = sim.info()
    mass = tot0[:, 0]
    conservation = {"steps": int(info["t"]),
                    "mass_rel_max": float(np.max(np.abs(tot1[:, 0] - mass) / mass)),
                    "momentum_rel_max": float(np.max(np.abs(tot1[:, 1:] - tot0[:, 1:]).max(axis=1) / mass))}
    bytes_site = info["bytes_per_site_update"]
    nsites = info["nsites"]
    mlups = nsites / (ms * 1e-3) / 1e6
    gbs = bytes_site * nsites / (ms * 1e-3) / 1e9
    kernel = KERNEL_NAMES[info["kernel"]]
    return {"value": mlups, "unit": "MLUPS", "ms_per_step": ms, "steps": steps,
            "bytes_per_site_update": bytes_site, "nsites": nsites, "achieved_GBs": gbs,
            "roofline_frac": gbs / PEAK_HBM_GBS, "kernel": kernel,
            "steps_per_launch": STEPS_PER_LAUNCH.get(kernel, 1),
            "block": info["block"], "grid": info["grid"], "conservation": conservation,
            "launches": {"graph_chunk": int(info["graph_chunk"]), "graph_launches": steps // int(info["graph_chunk"]),
                         "direct_launches": steps % int(info["graph_chunk"]), "warmup_direct_launches": warmup},
            "host_io_ms": {"init": init_ms, "moments": moments_ms}}


def pcie_inclusive(m) -> dict:
    """Throughput when the K timed steps are charged with lbm_init from host
    fields and lbm_moments back to host (FP64 rho and u over PCIe): context
    for callers that hand over host buffers, never the reported value."""
    total_ms = m["host_io_ms"]["init"] + m["steps"] * m["ms_per_step"] + m["host_io_ms"]["moments"]
    return {"value": m["nsites"] * m["steps"] / (total_ms * 1e-3) / 1e6, "unit": "MLUPS",
            "steps": m["steps"], "init_ms": m["host_io_ms"]["init"], "moments_ms": m["host_io_ms"]["moments"],
            "note": "lbm_init from host float64 rho, u + timed steps + lbm_moments to host"}


def traffic_per_launch(kernel: str, workload: str = "turbulence256", dtype: str = "fp32"):
    """HBM bytes per launch of the FP32 256^3 step of a kernel variant from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the
    copy-kernel calibration), or None when absent or taken on other kernel
    sources.  For the in-place variant a launch is one of its two alternating
    forms, averaged over both."""
    path = traffic_file(kernel, workload, dtype)
    if not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash():
        return None, "kernel changed since the counters were taken"
    return float(t["traffic_bytes_per_launch"]), "rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated"


def counted_rate(m, traffic):
    """HBM bytes the counters saw per second of the kernel's own time (traffic
    per launch over the time one launch takes), and that as a fraction of the
    peak; None without a counter summary.  For a kernel that moves fewer bytes
    than the algorithmic ones (the two-step kernel) this is the bandwidth it
    really draws, below `achieved`."""
    if not traffic:
        return None, None
    gbs = traffic / (m["ms_per_step"] * m["steps_per_launch"] * 1e-3) / 1e9
    return gbs, gbs / PEAK_HBM_GBS


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def err_norms(r, uu, r_ref, u_ref, U=None) -> dict:
    """Error norms of (rho, u) against the oracle's fields (see the module
    docstring); U: the background velocity of a wave."""
    import numpy as np

    du, dr = uu - u_ref, r - r_ref
    e = {"u_max_rel": float(np.abs(du).max() / np.abs(u_ref).max()),
         "u_l2_rel": float(np.sqrt(np.sum(du * du) / np.sum(u_ref * u_ref))),
         "rho_max": float(np.abs(dr).max()),
         "rho_l2_rel": float(np.sqrt(np.sum(dr * dr) / np.sum(r_ref * r_ref)))}
    if U is not None:
        Ub = np.asarray(U, dtype=np.float64)[: u_ref.shape[0]].reshape((-1,) + (1,) * (u_ref.ndim - 1))
        e["u_max_rel_to_wave"] = float(np.abs(du).max() / np.abs(u_ref - Ub).max())
    return e


def cpu_baseline_leg(rho, u, tau, budget_s: float, dtypes):
    """The FP64 oracle as it stands, on the full 256^3 box, for as many steps as
    fit in about `budget_s` seconds of host time -- timed as the CPU baseline.
    Its fields after those steps, and a 500-step oracle run of the same recipe
    at 32^3, are the references for the error statement of every storage type
    (max and L2 error of u and rho).  The 500-step error at 256^3 itself takes
    minutes of host time and is measured by the GPU test suite
    (test_turbulence_256_full_horizon_error)."""
    import oracle
    from paper_2002_02503_amd import inputs, lbm

    t0 = time.perf_counter()
    sim = oracle.Sim("D3Q19", (256, 256, 256), tau)
    sim.init(rho, u)
    t_init = time.perf_counter() - t0
    t1 = time.perf_counter()
    sim.step(1)
    one = time.perf_counter() - t1
    extra = max(0, min(19, int(budget_s / max(one, 1e-3)) - 1))
    t2 = time.perf_counter()
    sim.step(extra)
    steps = 1 + extra
    wall = one + (time.perf_counter() - t2)
    nsites = 256 ** 3
    base = {"value": nsites * steps / wall / 1e6, "unit": "MLUPS", "cores": oracle.get_threads(), "kind": "oracle",
            "sample": f"{steps} step(s) of the full 256^3 D3Q19 turbulence box, FP64 oracle "
                      f"(literal Hermite-tensor mode, OpenMP), {wall:.1f} s stepping + {t_init:.1f} s init",
            "cpu_model": cpu_model()}
    r_ref, u_ref = sim.moments()
    del sim
    errors = {"bounds": dict(lbm.STATED_BOUNDS),
              "bound_norm": "max |u - u_oracle| / max |u_oracle| and max |rho - rho_oracle|",
              f"full_256cubed_{steps}_steps": {}, "recipe_32cubed_500_steps": {}}
    for dt in dtypes:
        log(f"error statement {dt}: 256^3 after {steps} steps")
        with lbm.Simulation("D3Q19", (256, 256, 256), tau, dtype=dt) as g:
            g.init(rho, u).step(steps)
            r, uu = g.moments()
        errors[f"full_256cubed_{steps}_steps"][dt] = err_norms(r, uu, r_ref, u_ref)
        del r, uu
    del r_ref, u_ref
    log("error statement: 32^3 same recipe, 500 steps")
    srho, su = inputs.turbulence(32)
    ref = oracle.Sim("D3Q19", (32, 32, 32), tau, mode="closed").init(srho, su).step(500)
    r_ref, u_ref = ref.moments()
    for dt in dtypes:
        with lbm.Simulation("D3Q19", (32, 32, 32), tau, dtype=dt) as g:
            g.init(srho, su).step(500)
            r, uu = g.moments()
        errors["recipe_32cubed_500_steps"][dt] = err_norms(r, uu, r_ref, u_ref)
    return base, errors


def _row_amplitude(u_row, U_y: float) -> complex:
    """Complex amplitude of the first Fourier mode of u_y - U_y along one x-row."""
    import numpy as np

    n = u_row.shape[0]
    return complex(np.mean((u_row - U_y) * np.exp(-2j * np.pi * np.arange(n) / n)))


def _decay_rate(ts, amps) -> float:
    """Least-squares slope of -log|amplitude| over the last 80% of the run."""
    import numpy as np

    ts = np.asarray(ts, dtype=np.float64)
    a = np.log(np.abs(np.asarray(amps)))
    sel = ts >= 0.2 * ts.max()
    return -float(np.polyfit(ts[sel], a[sel], 1)[0])


def shear_run_gpu(lattice, n, tau, U, steps, dtype="fp32", every=100, **kw):
    """GPU shear wave (amplitude 0.01 along y on background U) on an n^3 box:
    decay rate of its fundamental mode and the final fields (one x-row each,
    the field being x-only bit for bit)."""
    import torch

    from paper_2002_02503_amd import inputs, lbm

    rho, u = inputs.shear_wave((n, n, n), 0.01, U)
    ts, amps = [0], [_row_amplitude(u[1, 0, 0], U[1])]
    with lbm.Simulation(lattice, (n, n, n), tau, dtype=dtype, graph_chunk=every, **kw) as sim:
        sim.init(rho, u)
        for t in range(every, steps + 1, every):
            sim.step(every)
            r, uu = sim.moments(device=True)
            ts.append(t)
            amps.append(_row_amplitude(uu[1, 0, 0].cpu().numpy(), U[1]))
        x_only = bool(torch.equal(uu, uu[:, :1, :1, :].expand_as(uu)))
        row = (r[0, 0].cpu().numpy()[None, None, :], uu[:, 0, 0].cpu().numpy()[:, None, None, :])
    return _decay_rate(ts, amps), row, x_only


def shear_run_oracle(lattice, n, tau, U, steps, every=100, **kw):
    """The oracle's run of the same x-only wave on an n x 1 x 1 box."""
    import oracle
    from paper_2002_02503_amd import inputs

    rho, u = inputs.shear_wave((n, 1, 1), 0.01, U)
    sim = oracle.Sim(lattice, (n, 1, 1), tau, mode="closed", **kw).init(rho, u)
    ts, amps = [0], [_row_amplitude(u[1, 0, 0], U[1])]
    for t in range(every, steps + 1, every):
        sim.step(every)
        _, uu = sim.moments()
        ts.append(t)
        amps.append(_row_amplitude(uu[1, 0, 0], U[1]))
    return _decay_rate(ts, amps), sim.moments()


def galilean_leg():
    """The Galilean test of configs with a background flow, on the GPU beside
    the oracle: the relative change of a shear wave's decay rate when the
    uniform flow U is added, |gamma_U / gamma_0 - 1|.  D3Q19 128^3, tau = 0.55,
    U = (0.1, 0.05, 0), 2000 steps, the paper's operator (K = 3) against the
    zero-velocity filter (K = 2), in FP32 and FP64; D3Q39 (K = 4) against
    D3Q19 at 192^3, tau = 0.6, U = (0.2, 0, 0), 1000 steps, in FP32 and FP64.
    In FP32 the rate fit bottoms out near 1e-4 (the wave decays by only a few
    per cent over the run); the FP64 runs resolve the operator's own ~1e-5.
    Also the shear waves' own errors against the oracle at the last step."""
    out = {}
    cases = [("d3q19_128_U0.1_0.05", "D3Q19", 128, 0.55, (0.1, 0.05, 0.0), 2000, "fp32", {}),
             ("d3q19_128_U0.1_0.05_fp64", "D3Q19", 128, 0.55, (0.1, 0.05, 0.0), 2000, "fp64", {}),
             ("d3q19_128_U0.1_0.05_k2", "D3Q19", 128, 0.55, (0.1, 0.05, 0.0), 2000, "fp32", {"K": 2}),
             ("d3q39_192_U0.2", "D3Q39", 192, 0.6, (0.2, 0.0, 0.0), 1000, "fp32", {}),
             ("d3q19_192_U0.2", "D3Q19", 192, 0.6, (0.2, 0.0, 0.0), 1000, "fp32", {}),
             ("d3q39_192_U0.2_fp64", "D3Q39", 192, 0.6, (0.2, 0.0, 0.0), 1000, "fp64", {}),
             ("d3q19_192_U0.2_fp64", "D3Q19", 192, 0.6, (0.2, 0.0, 0.0), 1000, "fp64", {})]
    for name, lat, n, tau, U, steps, dt, kw in cases:
        log(f"Galilean test {name}: {lat} {n}^3 {dt}, {steps} steps, U and U = 0")
        gU, (rU, uU), x_only = shear_run_gpu(lat, n, tau, U, steps, dtype=dt, **kw)
        g0, _, _ = shear_run_gpu(lat, n, tau, (0.0, 0.0, 0.0), steps, dtype=dt, **kw)
        oU, (r_ref, u_ref) = shear_run_oracle(lat, n, tau, U, steps, **kw)
        o0, _ = shear_run_oracle(lat, n, tau, (0.0, 0.0, 0.0), steps, **kw)
        out[name] = {"lattice": lat, "n": n, "tau": tau, "U": list(U), "steps": steps, "dtype": dt,
                     "hermite_order": kw.get("K", 4 if lat == "D3Q39" else 3),
                     "galilean_rel_rate_change_gpu": gU / g0 - 1, "galilean_rel_rate_change_oracle": oU / o0 - 1,
                     "decay_rate_gpu": gU, "decay_rate_oracle": oU, "x_only_bitwise": x_only,
                     "error_at_last_step": err_norms(rU, uU, r_ref, u_ref, U=U)}
    return out


def variant_error_leg():
    """Error statements of the benchmark's variants against the oracle:
    the 256-box batch (every 16th box against its nx x ny x 1 reduction after
    1000 steps), D3Q39 192^3 at K = 5 (300 steps, 192 x 1 x 1 reduction), and
    the collision kinds and D3Q15 on the 256^3 turbulence box (24 light-cone
    samples after 3 steps).  The D3Q39 K = 4 and FP64 statements come from the
    Galilean leg and the CPU baseline leg."""
    import numpy as np

    import oracle
    from paper_2002_02503_amd import inputs, lbm

    out = {}
    log("error statement: 256-box batch (FP32, FP16), 1000 steps, 16 boxes against the oracle")
    boxes = inputs.batch_boxes()
    dims, taus, rho, u = batch_fields()
    fields = {}
    for dt in ["fp32", "fp16"]:
        with lbm.Simulation("D3Q19", dims, taus, dtype=dt, graph_chunk=1000) as sim:
            sim.init(rho, u).step(1000)
            r, uu = sim.moments()
            fields[dt] = (sim.split_boxes(r), sim.split_boxes(uu))
    del rho, u
    worst = {"fp32": {}, "fp16": {}}
    for k in range(0, len(boxes), 16):
        nx, ny, _ = boxes[k]["dims"]
        r1, u1 = inputs.taylor_green_box((nx, ny, 1), boxes[k]["U"], 1.0 / 3.0)
        ref = oracle.Sim("D3Q19", (nx, ny, 1), boxes[k]["tau"], mode="closed").init(r1, u1).step(1000)
        r_ref, u_ref = ref.moments()
        for dt, (rb, ub) in fields.items():
            e = err_norms(rb[k][:1], ub[k][:, :1], r_ref, u_ref)
            # most vortices have decayed to round-off by t = 1000: relate the
            # error to the initial vortex amplitude instead of the final one
            Ub = np.asarray(boxes[k]["U"]).reshape(3, 1, 1, 1)
            e["u_max_rel_to_initial_wave"] = float(np.abs(ub[k][:, :1] - u_ref).max() / np.abs(u1 - Ub).max())
            for key, v in e.items():
                worst[dt][key] = max(worst[dt].get(key, 0.0), v)
    for dt in ["fp32", "fp16"]:
        out[f"batched_{dt}"] = dict(worst[dt], horizon_steps=1000, bound=lbm.STATED_BOUNDS[dt],
                                    note="worst of boxes 0, 16, ..., 240 (per-box norms) against their "
                                         "nx x ny x 1 oracle runs")
    log("error statement: D3Q39 192^3 K = 5, 300 steps")
    U = (0.2, 0.0, 0.0)
    srho, su = inputs.shear_wave((192, 192, 192), 0.01, U)
    with lbm.Simulation("D3Q39", (192, 192, 192), 0.6, dtype="fp32", K=5) as sim:
        sim.init(srho, su).step(300)
        r, uu = sim.moments()
    del srho, su
    r1, u1 = inputs.shear_wave((192, 1, 1), 0.01, U)
    # the closed forms are printed up to K = 4: the literal Hermite-tensor mode
    r_ref, u_ref = oracle.Sim("D3Q39", (192, 1, 1), 0.6, K=5, mode="literal").init(r1, u1).step(300).moments()
    out["d3q39_k5_fp32_192"] = dict(err_norms(r[:1, :1], uu[:, :1, :1], r_ref, u_ref, U=U), horizon_steps=300,
                                    x_only_bitwise=bool(np.array_equal(uu, np.broadcast_to(uu[:, :1, :1], uu.shape))))
    del r, uu
    log("error statement: collision kinds and D3Q15 on the 256^3 turbulence box, 24 light-cone samples, 3 steps")
    rho, u = inputs.turbulence(256)
    rng = np.random.default_rng(2)
    pts = [(0, 0, 0), (255, 255, 255)] + [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(22)]
    idx = tuple(np.array(pts).T)
    for name, lat, lib_kw, ora_kw in [("d3q19_bgk_fp32_256", "D3Q19", {"collision": "bgk"}, {"kind": "bgk"}),
                                      ("d3q19_theta0.5_fp32_256", "D3Q19", {"theta": 0.5},
                                       {"theta": 0.5, "mode": "literal"}),
                                      ("d3q19_k2_fp32_256", "D3Q19", {"K": 2}, {"K": 2}),
                                      ("d3q15_fp32_256", "D3Q15", {}, {})]:
        r_ref, u_ref = oracle.lightcone_samples(lat, rho, u, 0.51, 3, pts, **ora_kw)
        with lbm.Simulation(lat, (256, 256, 256), 0.51, dtype="fp32", **lib_kw) as sim:
            sim.init(rho, u).step(3)
            r, uu = sim.moments()
        out[name] = dict(err_norms(r[idx], uu[(slice(None),) + idx], r_ref, u_ref), horizon_steps=3,
                         note="24 sampled sites, light-cone oracle values")
        del r, uu
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-variants", action="store_true", help="headline FP32 measurement only")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline timing and error statements)")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the variants' error statements and the Galilean test (oracle on reductions)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle stepping")
    ap.add_argument("--graph-chunk", type=int, default=None,
                    help="steps per captured graph (default min(steps, 4096); 1 = direct launches, as counter "
                         "collection needs)")
    ap.add_argument("--kernel", choices=["tune", "scalar", "row_wave", "in_place", "two_row", "twist", "two_step"],
                    default="tune",
                    help="headline step kernel: autotuned (default) or pinned")
    ap.add_argument("--block", type=int, default=256, help="threads per block when --kernel is pinned")
    ap.add_argument("--dtype", choices=["fp32", "fp16", "bf16", "fp64"], default="fp32",
                    help="storage type of the headline box or of --workload batch256 (fp32 is the headline; the others "
                         "are profiling aids; the batch takes fp32, fp16 or bf16)")
    ap.add_argument("--workload", choices=["turbulence256", "batch256", "d3q39_192"], default="turbulence256",
                    help="turbulence256: the headline box (default); batch256: only the 256-box FP32 batch; "
                         "d3q39_192: only the D3Q39 192^3 FP32 shear wave; the last two print their own roofline "
                         "(profiling aids)")
    args = ap.parse_args()
    if args.workload == "batch256" and args.dtype == "fp64":
        ap.error("--workload batch256 takes --dtype fp32, fp16 or bf16")
    global GRAPH_CHUNK
    if args.graph_chunk is not None:
        if not 1 <= args.graph_chunk <= MAX_GRAPH_CHUNK:
            ap.error("--graph-chunk must be in [1, 4096]")
        GRAPH_CHUNK = args.graph_chunk
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the slab decomposition over xGMI is a design, not code). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2002_02503_amd import inputs, lbm

    torch.cuda.set_device(0)
    lbm.load_library()
    if args.workload == "batch256":
        batch_only(args)
        return
    if args.workload == "d3q39_192":
        d3q39_only(args)
        return
    tau = 0.51
    log("generating the 256^3 turbulence field")
    rho, u = inputs.turbulence(256)

    hd = args.dtype
    log(f"{hd.upper()} 256^3: {args.warmup} warm-up + {args.steps} timed steps")
    if args.kernel == "tune":
        head = measure_box("D3Q19", (256, 256, 256), tau, hd, rho, u, args.steps, args.warmup)
    else:
        pin = {"kernel": args.kernel, "block": args.block if args.kernel != "row_wave" else 0}
        head = measure_box("D3Q19", (256, 256, 256), tau, hd, rho, u, args.steps, args.warmup, tune=False, **pin)
    log(f"headline: {head['value']:.0f} MLUPS with the {head['kernel']} step, block {head['block']}")
    nsites = head["nsites"]
    traffic, traffic_src = traffic_per_launch(head["kernel"], "turbulence256", hd)
    spl = head["steps_per_launch"]
    roofline = {"bound": "hbm", "achieved": head["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": head["achieved_GBs"] / PEAK_HBM_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": head["bytes_per_site_update"] * nsites * spl,
                "steps_per_launch": spl,
                "kernel": KERNEL_SYMBOLS[head["kernel"]] + "<D3Q19, " + STORAGE_CTYPE[hd] + ", K=3>",
                "launch": {"kernel": head["kernel"], "block": head["block"], "grid": head["grid"]},
                "traffic_source": traffic_src}
    roofline["traffic_GBs"], roofline["traffic_frac"] = counted_rate(head, traffic)
    if spl == 2:
        roofline["note"] = ("achieved counts 2*Q*S bytes per site update, one read and one write of every "
                            "population per step; this kernel reads and writes the state once per two steps, "
                            "so its HBM traffic (traffic, counters: one write and about 1.7 reads of the state "
                            "per launch) is well below that and achieved can exceed a copy's rate; traffic_GBs "
                            "is the bandwidth it draws")

    log("copy probe at the same footprint")
    copy_bytes = head["bytes_per_site_update"] // 2 * nsites
    copy_ms = lbm.copy_probe(copy_bytes, reps=10)
    copy_gbs = 2 * copy_bytes / (copy_ms * 1e-3) / 1e9

    variants = {}
    if not args.no_variants:
        for dt in ["fp16", "bf16"]:
            log(f"{dt} storage 256^3")
            variants[dt] = measure_box("D3Q19", (256, 256, 256), tau, dt, rho, u, args.steps, args.warmup)
        log("fp64 storage 256^3, 300 steps")
        variants["fp64"] = measure_box("D3Q19", (256, 256, 256), tau, "fp64", rho, u, 300, args.warmup)
        log("batched: 256 D3Q19 boxes, 1000 steps")
        bdims, btaus, brho, bu = batch_fields()
        variants["batched_fp32"] = measure_box("D3Q19", bdims, btaus, "fp32", brho, bu, 1000, args.warmup)
        variants["batched_fp32"]["config"] = "256 boxes, sides 16..64, tau 0.52..1, |U| <= 0.1, Taylor-Green"
        log("batched: 256 D3Q19 boxes in FP16 storage, 1000 steps")
        variants["batched_fp16"] = measure_box("D3Q19", bdims, btaus, "fp16", brho, bu, 1000, args.warmup)
        variants["batched_fp16"]["config"] = variants["batched_fp32"]["config"] + ", FP16 storage of S(f_i - w_i)"
        del brho, bu
        log("D3Q39 192^3 FP32, 1000 steps")
        srho, su = inputs.shear_wave((192, 192, 192), 0.01, (0.2, 0.0, 0.0))
        variants["d3q39_fp32_192"] = measure_box("D3Q39", (192, 192, 192), 0.6, "fp32", srho, su, 1000,
                                                 args.warmup)
        log("D3Q39 192^3 FP32 at K = 5, 300 steps")
        variants["d3q39_k5_fp32_192"] = measure_box("D3Q39", (192, 192, 192), 0.6, "fp32", srho, su, 300,
                                                    args.warmup, K=5)
        del srho, su
        # the other collision kinds and lattices on the headline workload
        log("BGK, the energy-flux kind and K = 2 on the 256^3 FP32 turbulence box, 300 steps each")
        variants["d3q19_bgk_fp32_256"] = measure_box("D3Q19", (256, 256, 256), tau, "fp32", rho, u, 300,
                                                     args.warmup, collision="bgk")
        # theta inside D3Q19's bound |1 - 1/tau| theta 3/2 < 1 at tau = 0.51
        variants["d3q19_theta0.5_fp32_256"] = measure_box("D3Q19", (256, 256, 256), tau, "fp32", rho, u, 300,
                                                          args.warmup, theta=0.5)
        # the zero-velocity filter (K = 2), the operator the paper improves on
        variants["d3q19_k2_fp32_256"] = measure_box("D3Q19", (256, 256, 256), tau, "fp32", rho, u, 300,
                                                    args.warmup, K=2)
        log("D3Q15 on the 256^3 turbulence box, FP32, 300 steps")
        variants["d3q15_fp32_256"] = measure_box("D3Q15", (256, 256, 256), tau, "fp32", rho, u, 300, args.warmup)

    # measured HBM traffic of the variants whose launch has a committed counter summary
    for name, wl, dt in [("fp16", "turbulence256", "fp16"), ("bf16", "turbulence256", "bf16"),
                         ("fp64", "turbulence256", "fp64"),
                         ("batched_fp32", "batch256", "fp32"), ("batched_fp16", "batch256", "fp16"),
                         ("d3q39_fp32_192", "d3q39_192", "fp32")]:
        if name in variants:
            v = variants[name]
            tb, src = traffic_per_launch(v["kernel"], wl, dt)
            alg = v["bytes_per_site_update"] * v["nsites"] * v["steps_per_launch"]
            v["traffic_over_algorithmic"] = tb / alg if tb else None
            v["traffic_source"] = src

    galilean = None
    if not args.no_errors and not args.no_variants:
        galilean = galilean_leg()
        verr = variant_error_leg()
        for name, e in verr.items():
            variants[name]["error"] = e
        variants["d3q39_fp32_192"]["error"] = dict(galilean["d3q39_192_U0.2"]["error_at_last_step"],
                                                   horizon_steps=1000)

    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        log("CPU baseline leg: FP64 oracle on the host cores, and the error statements")
        dts = ["fp32", "fp16", "bf16", "fp64"] if not args.no_variants else ["fp32"]
        cpu, errors = cpu_baseline_leg(rho, u, tau, args.cpu_budget, dts)
        full = [k for k in errors if k.startswith("full_256cubed_")]
        for dt in ["fp16", "bf16", "fp64"]:
            if full and dt in variants and dt in errors[full[0]]:
                variants[dt]["error"] = dict(errors[full[0]][dt], horizon_steps=int(full[0].split("_")[2]),
                                             bound=errors["bounds"][dt])

    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D3Q19 256^3 periodic, decaying turbulence (k0=4, u_rms=0.04, seeded), "
                               f"tau=0.51, {hd.upper()} storage of S(f_i - w_i), Hermite order 3",
                   "lattice": "D3Q19", "dims": [256, 256, 256], "tau": tau, "hermite_order": 3},
        "roofline": roofline,
        "conservation": head["conservation"],
        "pcie_inclusive": pcie_inclusive(head),
        "cpu_baseline": cpu,
        "copy_probe": {"bytes_moved": 2 * copy_bytes, "GB_s": copy_gbs, "frac_of_peak": copy_gbs / PEAK_HBM_GBS},
        "frac_of_copy": head["achieved_GBs"] / copy_gbs,
        "launches": head["launches"],
        "variants": variants,
        "errors": errors,
        "galilean": galilean,
    }
    print(json.dumps(line), flush=True)


def batch_fields():
    """The 256-box workload: box parameters and Taylor-Green fields."""
    import numpy as np

    from paper_2002_02503_amd import inputs

    boxes = inputs.batch_boxes()
    fields = [inputs.taylor_green_box(b["dims"], b["U"], 1.0 / 3.0) for b in boxes]
    rho = np.concatenate([f[0].ravel() for f in fields])
    u = np.concatenate([f[1].reshape(3, -1) for f in fields], axis=1)
    return [b["dims"] for b in boxes], [b["tau"] for b in boxes], rho, u


def batch_only(args):
    """--workload batch256: time the batched step alone and print one JSON line
    with its roofline (the batched kernel is then the dominant one)."""
    from paper_2002_02503_amd import lbm

    dims, taus, rho, u = batch_fields()
    dt = args.dtype
    log(f"batched {dt.upper()}, 256 boxes: {args.warmup} warm-up + {args.steps} timed steps")
    if args.kernel == "tune":
        m = measure_box("D3Q19", dims, taus, dt, rho, u, args.steps, args.warmup)
    elif args.kernel == "scalar":
        m = measure_box("D3Q19", dims, taus, dt, rho, u, args.steps, args.warmup, tune=False, block=args.block)
    else:
        raise SystemExit("a batch runs the batched kernel: --kernel tune or scalar (block pinned)")
    nsites = m["nsites"]
    traffic, traffic_src = traffic_per_launch(m["kernel"], "batch256", dt)
    roofline = {"bound": "hbm", "achieved": m["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": m["achieved_GBs"] / PEAK_HBM_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": m["bytes_per_site_update"] * nsites,
                "kernel": "k_step_batch<D3Q19, " + {"fp32": "float", "fp16": "_Float16", "bf16": "bf16_t"}[dt] + ", K=3>", "launch": {"kernel": m["kernel"], "block": m["block"]},
                "traffic_source": traffic_src}
    copy_bytes = m["bytes_per_site_update"] // 2 * nsites
    copy_ms = lbm.copy_probe(copy_bytes, reps=10)
    copy_gbs = 2 * copy_bytes / (copy_ms * 1e-3) / 1e9
    roofline["traffic_GBs"], roofline["traffic_frac"] = counted_rate(m, traffic)
    line = {"metric": f"MLUPS & % HBM roofline, 256-box D3Q19 batch {dt.upper()}", "value": m["value"], "unit": "MLUPS",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "256 D3Q19 boxes, sides 16..64, tau 0.52..1, |U| <= 0.1, Taylor-Green, "
                                   f"{dt.upper()} storage, Hermite order 3, one launch per step", "nsites": nsites},
            "roofline": roofline, "conservation": m["conservation"], "cpu_baseline": None,
            "copy_probe": {"bytes_moved": 2 * copy_bytes, "GB_s": copy_gbs, "frac_of_peak": copy_gbs / PEAK_HBM_GBS},
            "frac_of_copy": m["achieved_GBs"] / copy_gbs}
    print(json.dumps(line), flush=True)


def d3q39_only(args):
    """--workload d3q39_192: time the D3Q39 192^3 FP32 step (K = 4) alone and
    print one JSON line with its roofline."""
    from paper_2002_02503_amd import inputs, lbm

    srho, su = inputs.shear_wave((192, 192, 192), 0.01, (0.2, 0.0, 0.0))
    log(f"D3Q39 192^3 FP32: {args.warmup} warm-up + {args.steps} timed steps")
    if args.kernel == "tune":
        m = measure_box("D3Q39", (192, 192, 192), 0.6, "fp32", srho, su, args.steps, args.warmup)
    else:
        pin = {"kernel": args.kernel, "block": args.block if args.kernel != "row_wave" else 0}
        m = measure_box("D3Q39", (192, 192, 192), 0.6, "fp32", srho, su, args.steps, args.warmup, tune=False, **pin)
    nsites = m["nsites"]
    traffic, traffic_src = traffic_per_launch(m["kernel"], "d3q39_192")
    roofline = {"bound": "hbm", "achieved": m["achieved_GBs"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": m["achieved_GBs"] / PEAK_HBM_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": m["bytes_per_site_update"] * nsites,
                "kernel": KERNEL_SYMBOLS[m["kernel"]] + "<D3Q39, float, K=4>",
                "launch": {"kernel": m["kernel"], "block": m["block"]}, "traffic_source": traffic_src}
    copy_bytes = m["bytes_per_site_update"] // 2 * nsites
    copy_ms = lbm.copy_probe(copy_bytes, reps=10)
    copy_gbs = 2 * copy_bytes / (copy_ms * 1e-3) / 1e9
    roofline["traffic_GBs"], roofline["traffic_frac"] = counted_rate(m, traffic)
    line = {"metric": "MLUPS & % HBM roofline, D3Q39 192^3 FP32", "value": m["value"], "unit": "MLUPS",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "D3Q39 192^3 periodic shear wave 0.01 on U = (0.2, 0, 0), tau = 0.6, "
                                   "FP32 storage, Hermite order 4", "nsites": nsites},
            "roofline": roofline, "conservation": m["conservation"], "cpu_baseline": None,
            "copy_probe": {"bytes_moved": 2 * copy_bytes, "GB_s": copy_gbs, "frac_of_peak": copy_gbs / PEAK_HBM_GBS},
            "frac_of_copy": m["achieved_GBs"] / copy_gbs}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
