"""CPU tests of the C ABI: the library loads, exports every symbol declared in
include/lbm.h, describes the same lattices as the oracle, and rejects bad
arguments on the host (before any device call).  No compute call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2002_02503_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    return lbm.load_library()


def _has_gpu():
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def test_every_declared_symbol_is_exported(lib):
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(lbm.EXPORTS) == declared


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15", "D3Q19", "D3Q39"])
def test_library_lattice_matches_oracle(lib, oracle_mod, name):
    """Same velocity set (as a set of (c, w) pairs), T0 and 2N as the oracle's
    independently typed tables."""
    got = lbm.lattice_table(name)
    ref = oracle_mod.lattice(name)
    assert (got["D"], got["Q"], got["two_n"]) == (ref["D"], ref["Q"], ref["two_n"])
    assert got["T0"] == ref["T0"]
    a = sorted((tuple(c), w) for c, w in zip(got["c"].tolist(), got["w"].tolist()))
    b = sorted((tuple(c), w) for c, w in zip(ref["c"].tolist(), ref["w"].tolist()))
    assert len(a) == len(b)
    for (ca, wa), (cb, wb) in zip(a, b):
        assert ca == cb and abs(wa - wb) < 1e-16


def _create(lib, lattice, dims, tau, dtype):
    h = ctypes.c_void_p()
    d = (ctypes.c_int64 * 3)(*dims)
    rc = lib.lbm_create(ctypes.byref(h), lattice, d, tau, dtype)
    return rc, h


@pytest.mark.parametrize("args,why", [
    ((1, (8, 8, 8), 0.5, 1), "tau == 1/2"),
    ((1, (8, 8, 8), 0.3, 1), "tau < 1/2"),
    ((1, (8, 8, 8), float("nan"), 1), "tau NaN"),
    ((1, (8, 8, 8), float("inf"), 1), "tau inf"),
    ((7, (8, 8, 8), 0.6, 1), "unknown lattice"),
    ((1, (8, 8, 8), 0.6, 9), "unknown dtype"),
    ((1, (0, 8, 8), 0.6, 1), "zero dim"),
    ((1, (8, -1, 8), 0.6, 1), "negative dim"),
    ((0, (8, 8, 2), 0.6, 1), "2-D lattice with nz != 1"),
    ((1, (1 << 20, 1 << 20, 1), 0.6, 1), "too many sites"),
    ((1, (1, 65536, 1), 0.6, 1), "ny > 65535"),
    ((1, (1, 1, 65536), 0.6, 1), "nz > 65535"),
    ((1, (1, 65535, 65535), 0.6, 1), "ny * nz >= 2^31"),
    ((0, (1 << 28, 1, 1), 0.6, 0), "population row of 2 GiB"),
    ((1, (1 << 20, 256, 65535), 0.6, 2), "more than 2^36 sites"),
])
def test_create_rejects_bad_arguments_on_host(lib, args, why):
    lattice, dims, tau, dtype = args
    rc, h = _create(lib, lattice, dims, tau, dtype)
    assert rc == -1, why
    assert not h.value
    assert lib.lbm_last_error().decode()


def test_create_null_out(lib):
    d = (ctypes.c_int64 * 3)(8, 8, 8)
    assert lib.lbm_create(None, 1, d, 0.6, 1) == -1


def test_batch_rejects_bad_box(lib):
    h = ctypes.c_void_p()
    dims = np.array([[8, 8, 8], [8, 0, 8]], dtype=np.int64)
    tau = np.array([0.6, 0.7])
    rc = lib.lbm_create_batch(ctypes.byref(h), 1, 2, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1)
    assert rc == -1
    assert "box 1" in lib.lbm_last_error().decode()
    rc = lib.lbm_create_batch(ctypes.byref(h), 1, 0, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1)
    assert rc == -1


def _create_batch(lib, lattice, dims, taus, dtype):
    h = ctypes.c_void_p()
    d = np.ascontiguousarray(dims, dtype=np.int64)
    t = np.ascontiguousarray(taus, dtype=np.float64)
    rc = lib.lbm_create_batch(ctypes.byref(h), lattice, len(t), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dtype)
    return rc, h


@pytest.mark.parametrize("dims,dtype,needle", [
    ([[1024, 1024, 14], [8, 8, 8]], 0, "2 GiB"),          # 14.7 M sites * 19 * 8 B in one batch box
    ([[(1 << 21) + 1, 1, 1], [8, 8, 8]], 0, "2^21"),      # float-reciprocal site split of the batched step
    ([[8, 65536, 1], [8, 8, 8]], 1, "65535"),
])
def test_batch_size_limits_are_host_checks(lib, dims, dtype, needle):
    """Every documented limit of lbm_create_batch is an argument check made on
    the host before any device call: LBM_EINVAL with or without a GPU."""
    rc, h = _create_batch(lib, 1, dims, [0.6] * len(dims), dtype)
    assert rc == -1
    assert not h.value
    assert needle in lib.lbm_last_error().decode()


def test_null_handle_calls_are_rejected(lib):
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_sync(None) == -1
    assert lib.lbm_set_hermite_order(None, 3) == -1
    assert lib.lbm_destroy(None) == 0


def test_copy_probe_validates(lib):
    ms = ctypes.c_double()
    assert lib.lbm_copy_probe(None, None, 16, 1, None, ctypes.byref(ms)) == -1


@pytest.mark.skipif(_has_gpu(), reason="checks the no-GPU path")
def test_valid_create_without_gpu_reports_enodev(lib):
    rc, h = _create(lib, 1, (8, 8, 8), 0.6, 1)
    assert rc == -4
    assert not h.value


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(lbm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lbm, "_lib", None)
    with pytest.raises(ImportError):
        lbm.load_library()


def test_binding_shares_torchs_hip_runtime():
    """Loaded through the binding first, the library still binds to the HIP
    runtime torch ships (same soname), so the process maps exactly one."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2002_02503_amd import lbm; lbm.load_library(); import torch; "
            "print(len(lbm._hip_runtimes_mapped()))")
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
