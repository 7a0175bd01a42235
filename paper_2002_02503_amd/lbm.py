"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the method runs in the HIP library.  PyTorch supplies device
memory (the two population buffers are torch tensors bound with
lbm_bind_state) and the stream (torch's current stream).  If the library is
not built, importing the binding's entry points raises immediately: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LATTICES = {"D2Q9": 0, "D3Q19": 1, "D3Q39": 2, "D3Q15": 3}
DTYPES = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
DTYPE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}
KERNELS = {"auto": 0, "scalar": 1, "row_wave": 2, "in_place": 3, "two_row": 4, "twist": 5, "two_step": 6}
COLLISIONS = {"filtered": 0, "bgk": 1}
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_ENODEV",
          -5: "LBM_ESTATE", -6: "LBM_ENUMERIC"}

# Every entry point declared in include/lbm.h.
EXPORTS = ["lbm_create", "lbm_create_batch", "lbm_set_hermite_order", "lbm_set_collision", "lbm_set_stream",
           "lbm_state_bytes",
           "lbm_bind_state", "lbm_init", "lbm_step", "lbm_prepare", "lbm_set_graph_chunk", "lbm_set_launch",
           "lbm_set_kernel", "lbm_tune", "lbm_moments", "lbm_totals", "lbm_residual", "lbm_residual_noalloc", "lbm_checkpoint_bytes", "lbm_get_state",
           "lbm_set_state", "lbm_get_info", "lbm_sync", "lbm_destroy", "lbm_last_error", "lbm_lattice_table",
           "lbm_copy_probe"]


# Stated error bounds of each storage type: the largest velocity error
# max |u - u_oracle| / max |u_oracle| (and density error max |rho -
# rho_oracle|) against the FP64 oracle on the same seeded inputs.  FP64 and
# FP32 are the method's tolerances; FP16 and BF16 store S (f_i - w_i) with 11
# and 8 significant bits and are bounded by what the 500-step 256^3
# turbulence run and the 2000-step shear waves measure, with margin.
STATED_BOUNDS = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 5e-3, "bf16": 5e-2}


class LBMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class lbm_info(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("dtype", ctypes.c_int32), ("D", ctypes.c_int32),
                ("Q", ctypes.c_int32), ("two_n", ctypes.c_int32), ("K", ctypes.c_int32),
                ("T0", ctypes.c_double), ("nbox", ctypes.c_int32), ("dims", ctypes.c_int64 * 3),
                ("nsites", ctypes.c_int64), ("t", ctypes.c_int64), ("bytes_per_site_update", ctypes.c_int64),
                ("state_bytes", ctypes.c_uint64), ("block", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("graph_chunk", ctypes.c_int32), ("kernel", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("theta", ctypes.c_double)]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load liblbm.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950). There is no CPU fallback.")
    # PyTorch ships its own HIP runtime under the soname libamdhip64.so.7, the
    # one liblbm.so links.  With torch loaded first the dynamic linker binds
    # liblbm.so to torch's copy and the process has one HIP runtime; loaded the
    # other way round, torch would bring a second runtime that sees no devices
    # and whose streams and events liblbm.so could not use.
    _torch()
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are mapped into this process (" + ", ".join(sorted(runtimes)) +
                          "); import torch before anything that loads libamdhip64")
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "lbm_create": [ctypes.POINTER(vp), ctypes.c_int32, i64p, ctypes.c_double, ctypes.c_int32],
        "lbm_create_batch": [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32, i64p, dp, ctypes.c_int32],
        "lbm_set_hermite_order": [vp, ctypes.c_int32],
        "lbm_set_collision": [vp, ctypes.c_int32, ctypes.c_double],
        "lbm_set_stream": [vp, vp],
        "lbm_state_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_bind_state": [vp, vp, vp, ctypes.c_size_t],
        "lbm_init": [vp, vp, vp, ctypes.c_int32],
        "lbm_step": [vp, ctypes.c_int64],
        "lbm_prepare": [vp],
        "lbm_set_graph_chunk": [vp, ctypes.c_int32],
        "lbm_set_launch": [vp, ctypes.c_int32, ctypes.c_int32],
        "lbm_set_kernel": [vp, ctypes.c_int32],
        "lbm_tune": [vp, ctypes.c_int32, ctypes.c_char_p],
        "lbm_moments": [vp, vp, vp, ctypes.c_int32],
        "lbm_totals": [vp, dp],
        "lbm_residual": [vp, vp, vp, ctypes.c_int32, dp],
        "lbm_residual_noalloc": [vp, vp, vp, vp],
        "lbm_checkpoint_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_get_state": [vp, vp, ctypes.c_size_t],
        "lbm_set_state": [vp, vp, ctypes.c_size_t],
        "lbm_get_info": [vp, ctypes.POINTER(lbm_info)],
        "lbm_sync": [vp],
        "lbm_destroy": [vp],
        "lbm_last_error": [],
        "lbm_lattice_table": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                              dp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), dp],
        "lbm_copy_probe": [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp, dp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "lbm_last_error" else ctypes.c_int
    _lib = lib
    return lib


def _hip_runtimes_mapped() -> set:
    """Files named libamdhip64* mapped into this process (Linux)."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1] if len(line.split()) >= 6 else ""
                if "libamdhip64" in os.path.basename(path):
                    found.add(os.path.realpath(path))
    except OSError:
        pass
    return found


def _check(rc: int):
    if rc != 0:
        msg = load_library().lbm_last_error().decode(errors="replace")
        raise LBMError(rc, msg)


def lattice_table(name: str) -> dict:
    """The library's own lattice descriptor (D, Q, T0, 2N, c, w)."""
    lib = load_library()
    D, Q, two_n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    T0 = ctypes.c_double()
    c = (ctypes.c_int32 * (39 * 3))()
    w = (ctypes.c_double * 39)()
    _check(lib.lbm_lattice_table(LATTICES[name], ctypes.byref(D), ctypes.byref(Q), ctypes.byref(T0),
                                 ctypes.byref(two_n), c, w))
    q = Q.value
    cc = np.array(c[: 3 * q], dtype=np.int64).reshape(q, 3)[:, : D.value]
    return {"D": D.value, "Q": q, "T0": T0.value, "two_n": two_n.value, "c": cc, "w": np.array(w[:q])}


def _torch():
    import torch  # noqa: PLC0415  (imported lazily: the binding itself needs only ctypes)

    return torch


def _ptr_of(a):
    """(pointer, on_device) for a numpy array or a torch CUDA tensor of float64."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise TypeError("host arrays must be C-contiguous float64")
        return ctypes.c_void_p(a.ctypes.data), 0
    torch = _torch()
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or not a.is_contiguous() or not a.is_cuda:
            raise TypeError("device tensors must be contiguous float64 CUDA tensors")
        return ctypes.c_void_p(a.data_ptr()), 1
    raise TypeError(f"unsupported array type {type(a)!r}")


class Simulation:
    """One periodic box, or a batch of boxes, advanced by the HIP library.

    Parameters follow lbm_create / lbm_create_batch: lattice name, dims
    (nx, ny, nz) or a list of them for a batch, tau (one value or one per
    box), storage dtype ("fp64", "fp32", "fp16", "bf16"), optional Hermite
    order K, collision operator ("filtered" or "bgk") with the energy-flux
    weight theta (lbm_set_collision), launch shape (block, grid) and steps per
    captured graph.  kernel picks the single-box step (lbm_set_kernel; a key of
    KERNELS: "scalar", "row_wave", "in_place", "two_row", "twist" or
    "two_step", the last taking two steps per launch); "auto" leaves the
    choice to the library, and tune() to measurement.
    """

    def __init__(self, lattice: str, dims, tau, dtype: str = "fp32", K: int | None = None,
                 block: int = 0, grid: int = 0, graph_chunk: int | None = None, torch_memory: bool = True,
                 stream=None, kernel: str = "auto", collision: str = "filtered", theta: float = 0.0):
        self.lib = load_library()
        self.lattice = lattice
        self.dtype = dtype
        self.h = ctypes.c_void_p()
        dims_arr = np.atleast_2d(np.asarray(dims, dtype=np.int64))
        self.nbox = dims_arr.shape[0]
        self.box_dims = [tuple(int(v) for v in d) for d in dims_arr]
        taus = np.broadcast_to(np.asarray(tau, dtype=np.float64), (self.nbox,)).copy()
        d = np.ascontiguousarray(dims_arr)
        if self.nbox == 1 and np.ndim(dims) == 1:
            _check(self.lib.lbm_create(ctypes.byref(self.h), LATTICES[lattice],
                                       d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), float(taus[0]),
                                       DTYPES[dtype]))
        else:
            _check(self.lib.lbm_create_batch(ctypes.byref(self.h), LATTICES[lattice], self.nbox,
                                             d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                             taus.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             DTYPES[dtype]))
        self._bufs = None
        try:
            if K is not None:
                _check(self.lib.lbm_set_hermite_order(self.h, int(K)))
            if collision != "filtered" or theta != 0.0:
                _check(self.lib.lbm_set_collision(self.h, COLLISIONS[collision], float(theta)))
            if block or grid:
                _check(self.lib.lbm_set_launch(self.h, int(block), int(grid)))
            if graph_chunk is not None:
                _check(self.lib.lbm_set_graph_chunk(self.h, int(graph_chunk)))
            if kernel != "auto":
                _check(self.lib.lbm_set_kernel(self.h, KERNELS[kernel]))
            torch = _torch()
            if stream is None:
                stream = torch.cuda.current_stream()
            self.stream = stream
            _check(self.lib.lbm_set_stream(self.h, ctypes.c_void_p(int(stream.cuda_stream))))
            if torch_memory:
                nbytes = ctypes.c_size_t()
                _check(self.lib.lbm_state_bytes(self.h, ctypes.byref(nbytes)))
                self._bufs = [torch.empty(nbytes.value, dtype=torch.uint8, device="cuda") for _ in range(2)]
                _check(self.lib.lbm_bind_state(self.h, ctypes.c_void_p(self._bufs[0].data_ptr()),
                                               ctypes.c_void_p(self._bufs[1].data_ptr()), nbytes.value))
        except Exception:
            self.close()
            raise
        info = self.info()
        self.D, self.Q, self.nsites = info["D"], info["Q"], info["nsites"]

    # -- lifetime -------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.lbm_destroy(self.h)
            self.h = ctypes.c_void_p()
        self._bufs = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state ------------------------------------------------------------
    def _field_shapes(self):
        if self.nbox == 1:
            nx, ny, nz = self.box_dims[0]
            return (nz, ny, nx), (self.D, nz, ny, nx)
        return (self.nsites,), (self.D, self.nsites)

    def init(self, rho, u):
        """f := f^eq_K(rho, u); rho and u as numpy float64 (host) or CUDA tensors."""
        rs, us = self._field_shapes()
        if isinstance(rho, np.ndarray):
            rho = np.ascontiguousarray(np.broadcast_to(rho, rs), dtype=np.float64)
            u = np.ascontiguousarray(u, dtype=np.float64).reshape(us)
        pr, dev_r = _ptr_of(rho)
        pu, dev_u = _ptr_of(u)
        if dev_r != dev_u:
            raise TypeError("rho and u must both be host arrays or both be device tensors")
        _check(self.lib.lbm_init(self.h, pr, pu, dev_r))
        return self

    def step(self, n: int = 1):
        _check(self.lib.lbm_step(self.h, int(n)))
        return self

    def prepare(self):
        _check(self.lib.lbm_prepare(self.h))
        return self

    def tune(self, steps: int = 20, cache: str | None = None):
        """Time the candidate launch shapes / step kernels and keep the fastest
        (the state is restored afterwards); `cache` is an optional text file."""
        _check(self.lib.lbm_tune(self.h, int(steps), cache.encode() if cache else None))
        return self

    def sync(self):
        _check(self.lib.lbm_sync(self.h))
        return self

    def moments(self, device: bool = False):
        """(rho, u) of the current state in float64: numpy arrays, or CUDA
        tensors when device=True."""
        rs, us = self._field_shapes()
        if device:
            torch = _torch()
            rho = torch.empty(rs, dtype=torch.float64, device="cuda")
            u = torch.empty(us, dtype=torch.float64, device="cuda")
        else:
            rho, u = np.empty(rs), np.empty(us)
        pr, dev = _ptr_of(rho)
        pu, _ = _ptr_of(u)
        _check(self.lib.lbm_moments(self.h, pr, pu, dev))
        return rho, u

    def split_boxes(self, field: np.ndarray) -> list:
        """Split a concatenated batch field (last axis = sites) into per-box
        arrays of shape (..., nz, ny, nx)."""
        out, off = [], 0
        for nx, ny, nz in self.box_dims:
            n = nx * ny * nz
            out.append(field[..., off:off + n].reshape(field.shape[:-1] + (nz, ny, nx)))
            off += n
        return out

    def totals(self) -> np.ndarray:
        """(nbox, 4): [sum rho, sum rho u_x, sum rho u_y, sum rho u_z] per box."""
        out = np.zeros(4 * self.nbox)
        _check(self.lib.lbm_totals(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(self.nbox, 4)

    def residual(self, rho_ref, u_ref) -> dict:
        rs, us = self._field_shapes()
        if isinstance(rho_ref, np.ndarray):
            rho_ref = np.ascontiguousarray(rho_ref, dtype=np.float64).reshape(rs)
            u_ref = np.ascontiguousarray(u_ref, dtype=np.float64).reshape(us)
        pr, dev = _ptr_of(rho_ref)
        pu, _ = _ptr_of(u_ref)
        out = np.zeros(4)
        _check(self.lib.lbm_residual(self.h, pr, pu, dev, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return {"u_max": out[0], "u_l2": out[1], "rho_max": out[2], "rho_l2": out[3]}

    def residual_noalloc(self, rho_ref, u_ref, out):
        """lbm_residual_noalloc: all three are contiguous float64 CUDA tensors
        (out holds 4 values); nothing is allocated and nothing synchronises."""
        pr, dr = _ptr_of(rho_ref)
        pu, du = _ptr_of(u_ref)
        po, do = _ptr_of(out)
        if not (dr and du and do) or out.numel() < 4:
            raise TypeError("rho_ref, u_ref and out must be device tensors; out holds 4 values")
        _check(self.lib.lbm_residual_noalloc(self.h, pr, pu, po))
        return out

    def get_state(self) -> np.ndarray:
        n = ctypes.c_size_t()
        _check(self.lib.lbm_checkpoint_bytes(self.h, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(self.lib.lbm_get_state(self.h, ctypes.c_void_p(buf.ctypes.data), n.value))
        return buf

    def set_state(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(self.lib.lbm_set_state(self.h, ctypes.c_void_p(buf.ctypes.data), buf.nbytes))
        return self

    def info(self) -> dict:
        inf = lbm_info()
        _check(self.lib.lbm_get_info(self.h, ctypes.byref(inf)))
        d = {name: getattr(inf, name) for name, _ in lbm_info._fields_}
        d["dims"] = tuple(inf.dims)
        return d

    @property
    def t(self) -> int:
        return int(self.info()["t"])


def copy_probe(nbytes: int, reps: int = 20, stream=None) -> float:
    """Mean milliseconds for one device-to-device copy of `nbytes` with the
    library's plain vectorised copy kernel."""
    torch = _torch()
    lib = load_library()
    nbytes = (int(nbytes) // 16) * 16
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    stream = torch.cuda.current_stream() if stream is None else stream
    ms = ctypes.c_double()
    _check(lib.lbm_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes, int(reps),
                              ctypes.c_void_p(int(stream.cuda_stream)), ctypes.byref(ms)))
    return ms.value
