"""Build liblbm.so (the HIP library behind include/lbm.h) for gfx950.

Every HIP source is compiled with hipcc for gfx950 only, without fast-math,
and with packed FP32 instructions disabled.  Multiply-adds are fused only
where one source expression writes a * b + c (-ffp-contract=on), never across
statements in the backend, so every kernel form of the step (one site per
lane, several sites per lane, batched) rounds the same expressions the same
way and computes the same bits.  The translation units are
compiled in parallel and linked into ``paper_2002_02503_amd/liblbm.so``.  The
step kernels' template instances are spread over small generated units (see
INSTANCE_GROUPS) so that the build runs in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = ["kernels.hip", "api.hip", "host.cpp"]
STORAGE = ["double", "float", "_Float16", "bf16_t"]
# Step-kernel instances, one translation unit per group (lattice, storage
# types): the large D3Q39 instances get a unit per storage type so that the
# units compile in parallel in similar times.
INSTANCE_GROUPS = ([("D2Q9", STORAGE), ("D3Q15", STORAGE), ("D3Q19", STORAGE)]
                   + [("D3Q39", [s]) for s in STORAGE])
# Two-step kernel instances (lattices with a one-site ring), one unit per
# (lattice, storage type): each instance holds two collisions.
STEP2_GROUPS = [(lat, [s]) for lat in ("D3Q15", "D3Q19") for s in STORAGE]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-Wall", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str, obj: str) -> None:
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns about the device-only target feature; drop that noise
    noise = ("packed-fp32-ops", "warning: unknown target feature", "1 warning generated")
    err = "\n".join(l for l in res.stderr.splitlines() if not any(n in l for n in noise))
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")


def _instance_units(gendir: str) -> list:
    """Write the step-kernel instance units: each includes step.hpp (single
    box), step_batch.hpp (batch) or step2.hpp (two steps per launch) and
    instantiates the launchers of one group of (lattice, storage type)
    pairs."""
    units = []
    families = [("step", "step.hpp", "LBM_DECLARE_STEP_INSTANCES", INSTANCE_GROUPS),
                ("batch", "step_batch.hpp", "LBM_DECLARE_BATCH_INSTANCES", INSTANCE_GROUPS),
                ("step2", "step2.hpp", "LBM_DECLARE_STEP2_INSTANCES", STEP2_GROUPS)]
    for family, header, macro, groups in families:
        for lat, types in groups:
            tag = lat.lower() + ("" if len(types) > 1 else "_" + types[0].strip("_").lower())
            path = os.path.join(gendir, f"{family}_{tag}.hip")
            lines = [f"// {family} kernels of {lat} ({', '.join(types)}); written by build.py",
                     f'#include "{header}"', "namespace lbm {"]
            lines += [f"{macro}(, {lat}, {t})" for t in types]
            lines += ["}  // namespace lbm", ""]
            text = "\n".join(lines)
            old = open(path).read() if os.path.exists(path) else None
            if old != text:
                with open(path, "w") as f:
                    f.write(text)
            units.append(path)
    return units


def build(out: str = LIB) -> str:
    objdir = os.path.join(PKG, "_build")
    gendir = os.path.join(objdir, "gen")
    os.makedirs(gendir, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + _instance_units(gendir)
    objs = [os.path.join(objdir, os.path.splitext(os.path.basename(s))[0] + ".o") for s in srcs]
    workers = min(len(srcs), max(1, os.cpu_count() or 1), 16)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(_compile, srcs, objs))
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
