"""Python front end of the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark may import this module.  The product
package never imports it, and the two share no code or tables; the only thing
both sides consume is the seeded macroscopic input fields (rho, u).

The C file writes out the paper's definitions literally (Hermite tensors by the
recursion eq. recurG, contracted per eq. hermite and eq. hermite-coll) and also
carries the printed closed forms eq. filter-Pi / filter-1st / filter-2nd as a
second mode, so the two can be checked against each other.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

LATTICES = {"D2Q9": 0, "D3Q19": 1, "D3Q39": 2, "D3Q15": 3}
KINDS = {"filtered": 0, "bgk": 1, "none": 2}
MODES = {"literal": 0, "closed": 1}

# Default Hermite truncation order per lattice (reading R1 in the C header).
DEFAULT_K = {"D2Q9": 3, "D3Q15": 3, "D3Q19": 3, "D3Q39": 4}

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ``lbm_oracle.c`` with gcc into ``liblbm_oracle.so`` (IEEE FP64,
    no fast-math, OpenMP)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_lattice.argtypes = [ctypes.c_int, ip, ip, dp, ip, ip, dp]
        lib.oracle_hermite.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_feq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        lib.oracle_fneq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        lib.oracle_fq.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        lib.oracle_collide.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.oracle_sim_create.restype = ctypes.c_void_p
        lib.oracle_sim_create.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                          ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double]
        lib.oracle_sim_destroy.argtypes = [ctypes.c_void_p]
        lib.oracle_sim_init.argtypes = [ctypes.c_void_p, dp, dp]
        lib.oracle_sim_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        lib.oracle_sim_moments.argtypes = [ctypes.c_void_p, dp, dp]
        lib.oracle_sim_totals.argtypes = [ctypes.c_void_p, dp]
        lib.oracle_sim_get.argtypes = [ctypes.c_void_p, dp]
        lib.oracle_sim_set.argtypes = [ctypes.c_void_p, dp]
        lib.oracle_sim_time.argtypes = [ctypes.c_void_p]
        lib.oracle_sim_time.restype = ctypes.c_long
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_get_threads.restype = ctypes.c_int
        _lib = lib
        return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def lattice(name: str) -> dict:
    """Velocity set, weights, T0 and order of isotropy 2N of a lattice."""
    lib = _load()
    D, Q, two_n = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    T0 = ctypes.c_double()
    c = np.zeros((39, 3), dtype=np.int32)
    w = np.zeros(39)
    _check(lib.oracle_lattice(LATTICES[name], ctypes.byref(D), ctypes.byref(Q), ctypes.byref(T0),
                              ctypes.byref(two_n), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              _dp(w)), "lattice")
    q = Q.value
    return {"D": D.value, "Q": q, "T0": T0.value, "two_n": two_n.value,
            "c": c[:q, :D.value].astype(np.int64), "w": w[:q].copy()}


def hermite(name: str, n: int) -> np.ndarray:
    """H^(n)(xi_i) for every velocity i, shape (Q, D, ..., D) with n trailing axes."""
    lat = lattice(name)
    D, Q = lat["D"], lat["Q"]
    out = np.zeros(Q * D ** n)
    _check(_load().oracle_hermite(LATTICES[name], n, _dp(out)), "hermite")
    return out.reshape((Q,) + (D,) * n)


def _vec3(u) -> np.ndarray:
    v = np.zeros(3)
    u = np.asarray(u, dtype=np.float64).ravel()
    v[: u.size] = u
    return v


def _mat3(P) -> np.ndarray:
    m = np.zeros((3, 3))
    P = np.asarray(P, dtype=np.float64)
    m[: P.shape[0], : P.shape[1]] = P
    return np.ascontiguousarray(m)


def feq(name: str, K: int, rho: float, u, mode: str = "literal") -> np.ndarray:
    """Equilibrium truncated at Hermite order K (eq. hermite)."""
    Q = lattice(name)["Q"]
    out = np.zeros(Q)
    _check(_load().oracle_feq(LATTICES[name], K, MODES[mode], float(rho), _dp(_vec3(u)), _dp(out)), "feq")
    return out


def fneq(name: str, K: int, u, Pi, mode: str = "literal") -> np.ndarray:
    """Filtered non-equilibrium part truncated at order K (eq. hermite-coll)."""
    Q = lattice(name)["Q"]
    out = np.zeros(Q)
    _check(_load().oracle_fneq(LATTICES[name], K, MODES[mode], _dp(_vec3(u)), _dp(_mat3(Pi)), _dp(out)),
           "fneq")
    return out


def fq(name: str, K: int, u, Qt) -> np.ndarray:
    """Energy-flux part of eq. pq in Hermite form, truncated at order K (reading
    R4 of the C file): (w_i / 6 T0^{3/2}) sum_{n=3}^{K} H^(n)(xi_i) (V^[n-3] Qt) / (n-3)!.
    Qt is a D x D x D (or 3 x 3 x 3) tensor."""
    Q = lattice(name)["Q"]
    out = np.zeros(Q)
    Qt = np.asarray(Qt, dtype=np.float64)
    q3 = np.zeros((3, 3, 3))
    q3[: Qt.shape[0], : Qt.shape[1], : Qt.shape[2]] = Qt
    _check(_load().oracle_fq(LATTICES[name], K, _dp(_vec3(u)), _dp(np.ascontiguousarray(q3)), _dp(out)), "fq")
    return out


def collide(name: str, f, tau: float, K: int | None = None, Keq: int | None = None,
            kind: str = "filtered", mode: str = "literal", theta: float = 0.0) -> np.ndarray:
    """One collision at one site (eq. post-1 with eq. hermite-coll, plus theta
    times the energy-flux part of eq. pq; or eq. BGK)."""
    K = DEFAULT_K[name] if K is None else K
    Keq = K if Keq is None else Keq
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    _check(_load().oracle_collide(LATTICES[name], KINDS[kind], MODES[mode], Keq, K, float(tau),
                                  float(theta), _dp(f), _dp(out)), "collide")
    return out


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


class Sim:
    """Periodic box evolved by the lattice Boltzmann equation (eq. lbe-reg).
    ``theta`` weights the energy-flux part of eq. pq (filtered kind only).

    ``dims`` is (nx, ny, nz); D2Q9 needs nz == 1.  Fields use the layout
    rho[z, y, x] and u[a, z, y, x].  The stored state is post-collision
    (reading R3)."""

    def __init__(self, name: str, dims, tau: float, K: int | None = None, Keq: int | None = None,
                 kind: str = "filtered", mode: str = "literal", theta: float = 0.0):
        self.lib = _load()
        self.name = name
        self.lat = lattice(name)
        nx, ny, nz = (list(dims) + [1, 1])[:3]
        self.dims = (int(nx), int(ny), int(nz))
        self.K = DEFAULT_K[name] if K is None else K
        self.Keq = self.K if Keq is None else Keq
        self.tau = float(tau)
        self.theta = float(theta)
        self.h = self.lib.oracle_sim_create(LATTICES[name], nx, ny, nz, float(tau), self.Keq, self.K,
                                            KINDS[kind], MODES[mode], self.theta)
        if not self.h:
            raise ValueError("oracle_sim_create rejected its arguments")
        self.nsites = nx * ny * nz

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.oracle_sim_destroy(h)
            self.h = None

    @property
    def shape(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    def init(self, rho, u):
        D = self.lat["D"]
        rho = np.ascontiguousarray(np.broadcast_to(rho, self.shape), dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape((D,) + self.shape)
        _check(self.lib.oracle_sim_init(self.h, _dp(rho), _dp(u)), "init")
        return self

    def step(self, n: int = 1):
        _check(self.lib.oracle_sim_step(self.h, int(n)), "step")
        return self

    @property
    def t(self) -> int:
        return int(self.lib.oracle_sim_time(self.h))

    def moments(self):
        D = self.lat["D"]
        rho = np.zeros(self.shape)
        u = np.zeros((D,) + self.shape)
        _check(self.lib.oracle_sim_moments(self.h, _dp(rho), _dp(u)), "moments")
        return rho, u

    def totals(self) -> np.ndarray:
        out = np.zeros(4)
        _check(self.lib.oracle_sim_totals(self.h, _dp(out)), "totals")
        return out

    def populations(self) -> np.ndarray:
        """f[z, y, x, i] in the oracle's own velocity order."""
        out = np.zeros(self.shape + (self.lat["Q"],))
        _check(self.lib.oracle_sim_get(self.h, _dp(out)), "get")
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.shape + (self.lat["Q"],))
        _check(self.lib.oracle_sim_set(self.h, _dp(f)), "set")
        return self


def lightcone_samples(name: str, rho0, u0, tau: float, steps: int, points, K: int | None = None,
                      mode: str = "closed", **kw):
    """(rho, u) at `points` (a list of (z, y, x)) after `steps` steps of a run
    started from (rho0, u0) on the full periodic box, computed site by site.

    The state at site x after s steps depends only on the initial fields
    within R s sites of x (R the largest velocity component).  A periodic box
    of side 2 R s + 1 centred on x and cut out of the full initial field
    therefore gives the exact value at its centre: the wrap-around of the
    small box reaches only the layers closer than R s to its faces.  Further
    keywords (kind, theta) go to Sim."""
    L = lattice(name)
    D = L["D"]
    R = int(np.abs(L["c"]).max())
    r = R * steps
    nz, ny, nx = np.shape(rho0)
    side = 2 * r + 1
    rho_out, u_out = [], []
    for z, y, x in points:
        ix = (x + np.arange(-r, r + 1)) % nx
        iy = (y + np.arange(-r, r + 1)) % ny
        iz = (z + np.arange(-r, r + 1)) % nz if D == 3 else np.array([0])
        sub_r = rho0[np.ix_(iz, iy, ix)]
        sub_u = u0[(slice(None),) + np.ix_(iz, iy, ix)]
        dims = (side, side, side if D == 3 else 1)
        sim = Sim(name, dims, tau, K=K, mode=mode, **kw).init(sub_r, sub_u).step(steps)
        rr, uu = sim.moments()
        cz = r if D == 3 else 0
        rho_out.append(rr[cz, r, r])
        u_out.append(uu[:, cz, r, r])
    return np.array(rho_out), np.array(u_out).T

