"""Pins of the oracle's energy-flux term (eq. pq with eq. filter-Q, weight theta).

The paper prints the energy-flux part in two places: at zero velocity as the
theta term of eq. filter2, and as the compact relative-velocity form
eq. filter-Q built on the relative energy flux eq. Q_def.  The oracle expands
the compact form in Hermite tensors, truncated at the same order K as
eq. hermite-coll (reading R4 in the oracle's C file).  These tests pin that
expansion against what the paper and the mathematics fix:

  * u = 0: the theta term of eq. filter2, typed again here from the paper;
  * K -> infinity: the compact form eq. filter-Q evaluated directly;
  * Hermite orthogonality: the term adds no mass, momentum or momentum flux
    for K <= 2N - 1, and on D3Q39 (2N = 6) its relative third moment is the
    relative energy flux it was built from;
  * the full collision: equilibrium fixed point, conservation, Pi relaxed as
    without the term, and on D3Q39 the relative non-equilibrium energy flux
    relaxed by (1 - 1/tau) theta;
  * physics: the shear viscosity T0 (tau - 1/2) does not depend on theta.
"""
import itertools
import math

import numpy as np
import pytest

from lbm_analysis import fit_decay, mode_amplitude

LATS = ["D2Q9", "D3Q15", "D3Q19", "D3Q39"]
RNG = np.random.default_rng(20020253)


def _rand_sym3(D, scale=1e-3):
    """A random fully symmetric D x D x D tensor."""
    A = RNG.uniform(-scale, scale, size=(D, D, D))
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    return sum(np.transpose(A, p) for p in perms) / 6.0


def _filter2_theta_term(L, Q):
    """The theta term of eq. filter2 without theta, typed from the paper:
    (w_i / 6 T0^2) [c c c / T0 - 3 c I] (triple contraction) Q."""
    c, w, T0, D = L["c"].astype(float), L["w"], L["T0"], L["D"]
    I = np.eye(D)
    out = np.zeros(L["Q"])
    for i in range(L["Q"]):
        ci = c[i]
        ccc = np.einsum("a,b,g->abg", ci, ci, ci)
        cI = np.einsum("a,bg->abg", ci, I) + np.einsum("b,ag->abg", ci, I) + np.einsum("g,ab->abg", ci, I)
        out[i] = w[i] / (6 * T0 * T0) * np.sum((ccc / T0 - cI) * Q)
    return out


def _rel3(L, f, u):
    """sum_i c'_i c'_i c'_i f_i with c' = c - u."""
    cp = L["c"].astype(float) - u
    return np.einsum("ia,ib,ig,i->abg", cp, cp, cp, f)


@pytest.mark.parametrize("name", LATS)
def test_zero_velocity_is_the_filter2_theta_term(oracle_mod, name):
    L = oracle_mod.lattice(name)
    D = L["D"]
    for K in range(3, L["two_n"]):
        for _ in range(4):
            Q = _rand_sym3(D)
            got = oracle_mod.fq(name, K, np.zeros(D), Q)
            ref = _filter2_theta_term(L, Q)
            assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max(), (K, np.abs(got - ref).max())


@pytest.mark.parametrize("name", LATS)
def test_large_K_reaches_the_compact_filter_Q(oracle_mod, name):
    """The series in K converges to eq. filter-Q (with f^eq / rho, eq. feq_full)."""
    L = oracle_mod.lattice(name)
    c, w, T0, D = L["c"].astype(float), L["w"], L["T0"], L["D"]
    u = np.array([0.02, -0.015, 0.01])[:D]
    Q = _rand_sym3(D)
    cp = c - u
    g = w * np.exp((c * c).sum(1) / (2 * T0)) * np.exp(-(cp * cp).sum(1) / (2 * T0))  # f^eq_full / rho
    I = np.eye(D)
    full = np.zeros(L["Q"])
    for i in range(L["Q"]):
        ccc = np.einsum("a,b,g->abg", cp[i], cp[i], cp[i])
        cI = (np.einsum("a,bg->abg", cp[i], I) + np.einsum("b,ag->abg", cp[i], I)
              + np.einsum("g,ab->abg", cp[i], I))
        full[i] = g[i] / (6 * T0 ** 3) * np.sum((ccc - T0 * cI) * Q)
    got = oracle_mod.fq(name, 10, u, Q)
    assert np.abs(got - full).max() < 1e-12 * np.abs(full).max()
    # the lowest truncation differs at first order in u
    assert np.abs(oracle_mod.fq(name, 3, u, Q) - full).max() > 1e-8


@pytest.mark.parametrize("name", LATS)
def test_low_moments_vanish(oracle_mod, name):
    """For 3 <= K <= 2N - 1 the term carries no mass, momentum or momentum flux
    (Hermite orthogonality: n + 2 <= 2N + 1)."""
    L = oracle_mod.lattice(name)
    c, D = L["c"].astype(float), L["D"]
    for K in range(3, L["two_n"]):
        for _ in range(4):
            u = RNG.uniform(-0.12, 0.12, size=D)
            f = oracle_mod.fq(name, K, u, _rand_sym3(D))
            assert abs(f.sum()) < 1e-18
            assert np.abs(c.T @ f).max() < 1e-18
            assert np.abs(np.einsum("ia,ib,i->ab", c, c, f)).max() < 1e-18


@pytest.mark.parametrize("K", [3, 4])
def test_d3q39_reproduces_the_relative_energy_flux(oracle_mod, K):
    """On D3Q39 (2N = 6) the relative third moment of the term is exactly the
    relative energy flux it was built from, at any u."""
    L = oracle_mod.lattice("D3Q39")
    for _ in range(5):
        u = RNG.uniform(-0.15, 0.15, size=3)
        Q = _rand_sym3(3)
        f = oracle_mod.fq("D3Q39", K, u, Q)
        assert np.abs(_rel3(L, f, u) - Q).max() < 1e-17


def test_d2q9_reproduces_the_mixed_components(oracle_mod):
    """On D2Q9 (2N = 4) at u = 0 the mixed components Q_xxy and Q_xyy are
    reproduced exactly, and Q_xxx, Q_yyy give nothing: on these nodes
    c_a^3 = c_a, so the third moment along one axis is tied to the momentum
    (H^(3)_aaa vanishes).  On the 3-D 2N = 4 lattices the third moment is only a
    lattice projection of Q (D3Q15's corners have c_x^2 = c_y^2 = c_z^2, D3Q19
    has no corner velocities), so exact reproduction is pinned on D2Q9 and
    D3Q39 alone."""
    L = oracle_mod.lattice("D2Q9")
    for _ in range(4):
        Q = _rand_sym3(2)
        M = _rel3(L, oracle_mod.fq("D2Q9", 3, np.zeros(2), Q), np.zeros(2))
        assert abs(M[0, 0, 1] - Q[0, 0, 1]) < 1e-18 and abs(M[0, 1, 1] - Q[0, 1, 1]) < 1e-18
        assert abs(M[0, 0, 0]) < 1e-18 and abs(M[1, 1, 1]) < 1e-18


@pytest.mark.parametrize("name", LATS)
def test_equilibrium_is_still_a_fixed_point(oracle_mod, name):
    L = oracle_mod.lattice(name)
    K = oracle_mod.DEFAULT_K[name]
    f = oracle_mod.feq(name, K, 1.03, RNG.uniform(-0.1, 0.1, size=L["D"]))
    out = oracle_mod.collide(name, f, tau=0.6, K=K, theta=0.7)
    assert np.abs(out - f).max() < 1e-15


@pytest.mark.parametrize("name", LATS)
def test_collision_with_energy_flux_conserves_and_relaxes_pi(oracle_mod, name):
    L = oracle_mod.lattice(name)
    c, D, T0 = L["c"].astype(float), L["D"], L["T0"]
    K = oracle_mod.DEFAULT_K[name]
    tau = 0.7
    f = oracle_mod.feq(name, K, 1.02, RNG.uniform(-0.08, 0.08, size=D)) * (1 + RNG.uniform(-0.02, 0.02, L["Q"]))
    rho, j = f.sum(), c.T @ f
    u = j / rho
    Pi_in = np.einsum("ia,ib,i->ab", c, c, f) - rho * (np.outer(u, u) + T0 * np.eye(D))
    out = oracle_mod.collide(name, f, tau=tau, theta=0.8)
    assert abs(out.sum() - rho) < 1e-15
    assert np.abs(c.T @ out - j).max() < 1e-15
    Pi_out = np.einsum("ia,ib,i->ab", c, c, out) - rho * (np.outer(u, u) + T0 * np.eye(D))
    assert np.abs(Pi_out - (1 - 1 / tau) * Pi_in).max() < 1e-15
    # theta changes the post-collision state
    assert np.abs(out - oracle_mod.collide(name, f, tau=tau)).max() > 1e-7


def test_d3q39_relaxes_the_relative_energy_flux_by_theta(oracle_mod):
    """On D3Q39 at K = 4: sum c'c'c' (f' - f^eq) = (1 - 1/tau) theta Qt, where Qt
    is the relative non-equilibrium energy flux eq. Q_def of the incoming f."""
    L = oracle_mod.lattice("D3Q39")
    K, tau = 4, 0.65
    for theta in [0.0, 0.5, 1.0]:
        f = oracle_mod.feq("D3Q39", K, 0.98, RNG.uniform(-0.1, 0.1, size=3)) * (1 + RNG.uniform(-0.02, 0.02, 39))
        rho = f.sum()
        u = (L["c"].T @ f) / rho
        feq = oracle_mod.feq("D3Q39", K, rho, u)
        Qt = _rel3(L, f - feq, u)
        out = oracle_mod.collide("D3Q39", f, tau=tau, K=K, theta=theta)
        got = _rel3(L, out - feq, u)
        assert np.abs(got - (1 - 1 / tau) * theta * Qt).max() < 1e-15


def test_relative_energy_flux_identity(oracle_mod):
    """Mass and momentum of f - f^eq vanish, so eq. Q_def equals the absolute
    flux eq. coeff-3 minus the symmetrised product of u and Pi (the statement
    after eq. filter-Q)."""
    for name in ["D3Q19", "D3Q39"]:
        L = oracle_mod.lattice(name)
        c = L["c"].astype(float)
        K = oracle_mod.DEFAULT_K[name]
        f = oracle_mod.feq(name, K, 1.01, RNG.uniform(-0.1, 0.1, size=3)) * (1 + RNG.uniform(-0.02, 0.02, L["Q"]))
        rho = f.sum()
        u = c.T @ f / rho
        d = f - oracle_mod.feq(name, K, rho, u)
        Qabs = np.einsum("ia,ib,ig,i->abg", c, c, c, d)
        Pi = np.einsum("ia,ib,i->ab", c, c, d)
        sym = np.einsum("a,bg->abg", u, Pi) + np.einsum("b,ag->abg", u, Pi) + np.einsum("g,ab->abg", u, Pi)
        assert np.abs(_rel3(L, d, u) - (Qabs - sym)).max() < 1e-16


def _shear_rate(oracle_mod, name, n, tau, theta, steps):
    x = np.arange(n)
    u = np.zeros((3, 1, 1, n))
    u[1, 0, 0] = 0.01 * np.sin(2 * np.pi * x / n)
    sim = oracle_mod.Sim(name, (n, 1, 1), tau, theta=theta).init(np.ones((1, 1, n)), u)
    every = steps // 15
    ts, amps = [0], [mode_amplitude(u[1, 0, 0], n, axis=0)]
    for t in range(every, 15 * every + 1, every):
        sim.step(every)
        _, uu = sim.moments()
        ts.append(t)
        amps.append(mode_amplitude(uu[1, 0, 0], n, axis=0))
    return fit_decay(ts, amps)


@pytest.mark.parametrize("name", ["D3Q19", "D3Q39"])
def test_shear_viscosity_does_not_depend_on_theta(oracle_mod, name):
    """The energy-flux term changes no second moment, so the shear viscosity
    T0 (tau - 1/2) is the same for every theta: a shear wave at U = 0 decays at
    nu k^2, and what theta changes in the rate is of higher order in k (the
    relative change falls 4x when k halves; it is about 1e-3 at k = 2 pi / 32)."""
    tau = 0.8
    T0 = oracle_mod.lattice(name)["T0"]
    d = {}
    for n in [32, 64]:
        steps = int(1500 * (n / 64) ** 2)
        g0 = _shear_rate(oracle_mod, name, n, tau, 0.0, steps)
        g1 = _shear_rate(oracle_mod, name, n, tau, 1.0, steps)
        k = 2 * math.pi / n
        assert abs(g1 / (T0 * (tau - 0.5) * k * k) - 1) < 6e-3
        d[n] = g1 / g0 - 1
    assert 3.8 < d[32] / d[64] < 4.2, d


def test_d3q19_stability_bound_of_the_energy_flux_term(oracle_mod):
    """On D3Q19 the third-order Hermite tensors are not orthogonal under the
    lattice weights (the (3,3) pair fails), so the term maps the mixed
    components (Q_xxy, Q_yzz) through a matrix with eigenvalues 1/2 and 3/2
    (the lattice's sixth moments), and the post-collision energy flux of that
    mode is (1 - 1/tau) theta 3/2 times the incoming one.  The run is therefore
    stable only while |1 - 1/tau| theta 3/2 < 1: at tau = 0.55, theta = 0.5
    stays bounded and theta = 1 grows without bound."""
    L = oracle_mod.lattice("D3Q19")
    c = L["c"].astype(float)
    M = np.zeros((2, 2))
    for j, a in enumerate([(0, 0, 1), (1, 2, 2)]):  # Q_xxy, Q_yzz
        Q = np.zeros((3, 3, 3))
        for p in itertools.permutations(a):
            Q[p] = 1.0
        f = oracle_mod.fq("D3Q19", 3, np.zeros(3), Q)
        T = np.einsum("ia,ib,ig,i->abg", c, c, c, f)
        M[0, j], M[1, j] = T[0, 0, 1], T[1, 2, 2]
    assert np.allclose(sorted(np.linalg.eigvalsh(M)), [0.5, 1.5], atol=1e-14)
    n, tau = 64, 0.55
    x = np.arange(n)
    u = np.zeros((3, 1, 1, n))
    u[1, 0, 0] = 0.01 * np.sin(2 * np.pi * x / n)
    amp = {}
    for theta in [0.5, 1.0]:
        sim = oracle_mod.Sim("D3Q19", (n, 1, 1), tau, theta=theta, mode="closed").init(np.ones((1, 1, n)), u)
        with np.errstate(all="ignore"):
            sim.step(200)
            _, uu = sim.moments()
        amp[theta] = float(np.abs(uu[1]).max())
    assert amp[0.5] < 0.01
    assert not (amp[1.0] < 1.0)  # grown past any physical value (or overflowed)
