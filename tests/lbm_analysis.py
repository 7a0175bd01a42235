"""Small analysis helpers shared by the tests: Fourier-mode amplitudes, decay
fits, error norms and the independent isotropy / Hermite constructions the
oracle is pinned against.  Nothing here calls the oracle or the GPU library."""
from __future__ import annotations

import itertools
import math

import numpy as np


def mode_amplitude(field: np.ndarray, axis_len: int, axis: int, mode: int = 1) -> complex:
    """Complex amplitude of Fourier mode `mode` along `axis` of `field`, averaged
    over the other axes: (1/N) sum field * exp(-i k x).  Its modulus does not
    change when the pattern is advected, so advection drops out of decay fits."""
    x = np.arange(axis_len)
    shape = [1] * field.ndim
    shape[axis] = axis_len
    ph = np.exp(-2j * np.pi * mode * x / axis_len).reshape(shape)
    return complex(np.mean(field * ph))


def fit_decay(ts, amps, start_frac: float = 0.2) -> float:
    """Least-squares slope gamma of log|amp| = c - gamma t over t >= start_frac * T."""
    ts = np.asarray(ts, dtype=np.float64)
    a = np.log(np.abs(np.asarray(amps)))
    sel = ts >= start_frac * ts.max()
    A = np.vstack([np.ones(sel.sum()), ts[sel]]).T
    coef, *_ = np.linalg.lstsq(A, a[sel], rcond=None)
    return -float(coef[1])


def rel_errors(u_test: np.ndarray, u_ref: np.ndarray, rho_test: np.ndarray, rho_ref: np.ndarray) -> dict:
    """Error norms: max and L2 of u relative to the reference's max / L2 norm,
    and max |delta rho| relative to max |rho_ref|."""
    du = u_test - u_ref
    dr = rho_test - rho_ref
    return {
        "u_max": float(np.abs(du).max() / np.abs(u_ref).max()),
        "u_l2": float(np.sqrt(np.sum(du * du)) / np.sqrt(np.sum(u_ref * u_ref))),
        "rho_max": float(np.abs(dr).max() / np.abs(rho_ref).max()),
        "rho_l2": float(np.sqrt(np.sum(dr * dr)) / np.sqrt(np.sum(rho_ref * rho_ref))),
    }


def kronecker_delta_tensor(D: int, n: int) -> np.ndarray:
    """Delta^n: the sum over all pairings of n indices of products of Kronecker
    deltas (zero for odd n).  Built by brute-force enumeration of pairings."""
    T = np.zeros((D,) * n)
    if n % 2:
        return T
    pairings = list(_pairings(list(range(n))))
    for idx in itertools.product(range(D), repeat=n):
        T[idx] = sum(all(idx[a] == idx[b] for a, b in p) for p in pairings)
    return T


def _pairings(items):
    if not items:
        yield []
        return
    a = items[0]
    for k in range(1, len(items)):
        b = items[k]
        rest = items[1:k] + items[k + 1:]
        for p in _pairings(rest):
            yield [(a, b)] + p


def moment_tensor(c: np.ndarray, w: np.ndarray, n: int) -> np.ndarray:
    """E^(n) = sum_i w_i c_i ... c_i (n times)."""
    D = c.shape[1]
    T = np.zeros((D,) * n)
    for ci, wi in zip(c.astype(np.float64), w):
        t = np.array(wi)
        for _ in range(n):
            t = np.multiply.outer(t, ci)
        T = T + t
    return T


def hermite_explicit(xi: np.ndarray, n: int) -> np.ndarray:
    """Grad's tensor Hermite polynomial from its explicit expansion
    H^(n)_{a1..an} = sum_k (-1)^k sum over sets of k disjoint index pairs
    [prod of deltas over the pairs] [prod of xi over the unpaired indices].
    (Independent of the three-term recursion the oracle uses.)"""
    D = xi.shape[0]
    H = np.zeros((D,) * n)
    idx_all = list(range(n))
    partials = []
    for k in range(0, n // 2 + 1):
        for chosen in itertools.combinations(idx_all, 2 * k):
            for p in _pairings(list(chosen)):
                free = [m for m in idx_all if m not in chosen]
                partials.append((k, p, free))
    for idx in itertools.product(range(D), repeat=n):
        val = 0.0
        for k, p, free in partials:
            if all(idx[a] == idx[b] for a, b in p):
                val += (-1) ** k * math.prod(xi[idx[m]] for m in free)
        H[idx] = val
    return H


def sym_perm_delta(D: int, n: int) -> np.ndarray:
    """The 2n-index tensor sum over permutations s of S_n of
    prod_k delta_{a_k, b_s(k)}: Hermite orthonormality's right-hand side."""
    T = np.zeros((D,) * (2 * n))
    for idx in itertools.product(range(D), repeat=2 * n):
        a, b = idx[:n], idx[n:]
        T[idx] = sum(all(a[k] == b[s[k]] for k in range(n)) for s in itertools.permutations(range(n)))
    return T
