// Per-site filtered, Galilean-invariant collision, in registers.
//
// The step at one site (eq. lbe-reg with eq. post-1):
//     f'_i = f^eq_i + (1 - 1/tau) fhat^neq_i
// with the equilibrium truncated at Hermite order K (eq. hermite),
//     f^eq_i = w_i rho sum_{n<=K} H^(n)(xi_i) . V^[n] / n!,
// and the filtered non-equilibrium part written in the frame of the local
// velocity and truncated at the same order (eq. hermite-coll),
//     fhat_i = (w_i / 2 T0) sum_{n=2..K} H^(n)(xi_i) : V^[n-2] Pi / (n-2)!.
// Pi is the non-equilibrium momentum flux (eq. coeff-2, equal to eq. Pi_def).
//
// Closed form used here.  With a = c_i.u / T0, v = u.u / T0 and the scalar
// Hermite polynomials h_0 = 1, h_1 = a, h_{n+1} = a h_n - n v h_{n-1}
// (H^(n)(xi).V^[n] = h_n), the equilibrium is w_i rho P_K(a) with
// P_m = sum_{n<=m} h_n / n!.  Contracting eq. hermite-coll the same way (the
// generating function of the H^(n) is exp(xi.t - t.t/2); two derivatives in t
// contracted with Pi and evaluated along t = sV give the series term by term):
//     fhat_i = (w_i / 2 T0) [A_i P_{K-2} - B_i P_{K-3} + C P_{K-4}],
//     A_i = c_i.Pi.c_i / T0 - tr Pi,   B_i = 2 c_i.Pi.u / T0,   C = u.Pi.u / T0,
// with P_m = 0 for m < 0.  K = 2 gives eq. filter-Pi, K = 3 eq. filter-1st and
// K = 4 eq. filter-2nd exactly.
//
// Stored variable.  The state holds G_i = S (f_i - w_i): the deviation from
// the rest weights in units of the lattice's weight quantum 1/S, so that the
// weights enter only as the exact integers W_i = S w_i.  Then
//     rho = 1 + sum G / S,   rho u = sum c G / S,   sum c c f = T0 I + sum c c G / S,
// and because the truncated equilibrium has exact moments up to second order
// (K <= 2N-1),
//     Pi  = sum c c G / S - (rho - 1) T0 I - rho u u,
//     G'_i = W_i [(rho - 1) P_K + (P_K - 1)] + W_i (1 - 1/tau) / (2 T0) N_i,
// N_i the bracket of fhat_i above.  Every quantity is of the size of the
// perturbation, not of w_i, and no rounded weight biases the sums.
//
// Finite-precision conservation.  Collision conserves mass and momentum
// exactly (eq. conserv) only in exact arithmetic.  With PROJ (single
// precision) the post-collision G' is projected back onto the pre-collision
// rho and rho u:
//     G'_i += W_i [dm + c_i . dj / T0],  dm = (S(rho-1) - sum G') / S,
//                                        dj = (S rho u - sum c G') / S.
// The correction is of rounding size and vanishes in exact arithmetic.  All
// arithmetic is in the compute type R (float for every storage type except
// double); no wider type is used inside the step.
#pragma once

#include "lattice.hpp"

namespace lbm {

// a b + c rounded once, in the compute type R.
template <class R>
__device__ __forceinline__ R fused(R a, R b, R c)
{
    if constexpr (std::is_same<R, float>::value) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// Sparse dot products with compile-time integer coefficients: zero terms are
// dropped and the sum starts from -0.0, which IEEE addition leaves unchanged,
// so no "0 + x" or "0 * x" survives into the instruction stream.
template <int X, int Y, int Z, class R>
__device__ __forceinline__ R cdot(R ax, R ay, R az)
{
    R acc = R(-0.0);
    if constexpr (X != 0) acc += R(X) * ax;
    if constexpr (Y != 0) acc += R(Y) * ay;
    if constexpr (Z != 0) acc += R(Z) * az;
    return acc;
}

// c.q.c for a symmetric q given by its six components
template <int X, int Y, int Z, class R>
__device__ __forceinline__ R cquad(R qxx, R qyy, R qzz, R qxy, R qxz, R qyz)
{
    R acc = R(-0.0);
    if constexpr (X != 0) acc += R(X * X) * qxx;
    if constexpr (Y != 0) acc += R(Y * Y) * qyy;
    if constexpr (Z != 0) acc += R(Z * Z) * qzz;
    if constexpr (X * Y != 0) acc += R(2 * X * Y) * qxy;
    if constexpr (X * Z != 0) acc += R(2 * X * Z) * qxz;
    if constexpr (Y * Z != 0) acc += R(2 * Y * Z) * qyz;
    return acc;
}

// Collision kinds.  kFiltered is the operator above.  kBGK is eq. BGK with the
// same truncated equilibrium: G' = G^eq + (1 - 1/tau)(G - G^eq).  kFilteredQ
// adds theta times the energy-flux part of eq. pq: the compact form
// eq. filter-Q (with f^eq / rho, so that it is the theta term of eq. filter2
// at u = 0) expanded in Hermite tensors and truncated at the same K.  Three
// t-derivatives of the generating function, contracted with the relative
// energy flux Qt (eq. Q_def) and evaluated along t = V, give
//     fhat^q_i = (w_i / 6 T0^3) [d0 P_{K-3} + d1 P_{K-4} + d2 P_{K-5}],
//     d0 = Qt.ccc - 3 T0 c.qt,  d1 = -3 c.(Qt.u).c + 3 T0 u.qt,  d2 = 3 c.(Qt:uu),
// with qt_c = sum_a Qt_aac (the next term, -Qt:uuu P_{K-6}, needs K >= 6).
// Because f - f^eq carries no mass or momentum,
//     Qt = sum c c c (f - f^eq) - (u Pi + Pi u + the third permutation).
// (The kind codes, CollisionKind, are in lattice.hpp.)

// Third moment accumulators, stored by the number of x, y and z indices.
template <class R>
struct Sym3 {
    R xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz;
};

// acc += v * c c c for a compile-time c, component by component
template <int X, int Y, int Z, class R>
__device__ __forceinline__ void add_ccc(Sym3<R>& t, R v)
{
    if constexpr (X * X * X != 0) t.xxx += R(X * X * X) * v;
    if constexpr (X * X * Y != 0) t.xxy += R(X * X * Y) * v;
    if constexpr (X * X * Z != 0) t.xxz += R(X * X * Z) * v;
    if constexpr (X * Y * Y != 0) t.xyy += R(X * Y * Y) * v;
    if constexpr (X * Y * Z != 0) t.xyz += R(X * Y * Z) * v;
    if constexpr (X * Z * Z != 0) t.xzz += R(X * Z * Z) * v;
    if constexpr (Y * Y * Y != 0) t.yyy += R(Y * Y * Y) * v;
    if constexpr (Y * Y * Z != 0) t.yyz += R(Y * Y * Z) * v;
    if constexpr (Y * Z * Z != 0) t.yzz += R(Y * Z * Z) * v;
    if constexpr (Z * Z * Z != 0) t.zzz += R(Z * Z * Z) * v;
}

// t : c c c (full contraction with a symmetric tensor) for a compile-time c
template <int X, int Y, int Z, class R>
__device__ __forceinline__ R ccc_dot(const Sym3<R>& t)
{
    R acc = R(-0.0);
    if constexpr (X * X * X != 0) acc += R(X * X * X) * t.xxx;
    if constexpr (X * X * Y != 0) acc += R(3 * X * X * Y) * t.xxy;
    if constexpr (X * X * Z != 0) acc += R(3 * X * X * Z) * t.xxz;
    if constexpr (X * Y * Y != 0) acc += R(3 * X * Y * Y) * t.xyy;
    if constexpr (X * Y * Z != 0) acc += R(6 * X * Y * Z) * t.xyz;
    if constexpr (X * Z * Z != 0) acc += R(3 * X * Z * Z) * t.xzz;
    if constexpr (Y * Y * Y != 0) acc += R(Y * Y * Y) * t.yyy;
    if constexpr (Y * Y * Z != 0) acc += R(3 * Y * Y * Z) * t.yyz;
    if constexpr (Y * Z * Z != 0) acc += R(3 * Y * Z * Z) * t.yzz;
    if constexpr (Z * Z * Z != 0) acc += R(Z * Z * Z) * t.zzz;
    return acc;
}

template <class L, int K, int KIND, bool PROJ, class R>
__device__ __forceinline__ void collide_site(R (&G)[L::Q], R omega, R theta)
{
    static_assert(K >= 2 && K <= L::K_MAX, "Hermite order outside 2..2N-1");
    static_assert(KIND == kFiltered || KIND == kBGK || (KIND == kFilteredQ && K >= 3), "collision kind");
    constexpr int NP = (L::Q - 1) / 2;  // opposite pairs (2p+1, 2p+2)
    constexpr bool D3 = (L::D == 3);
    constexpr R IT0 = R(L::INV_T0);
    constexpr R T0 = R(L::T0);
    constexpr R SR = R(L::S);
    constexpr R IS = R(1.0 / L::S);
    constexpr R NZ = R(-0.0);

    // zeroth, first and second moments (eq. mme, eq. Mflux), scaled by S,
    // from pair sums s = G_+ + G_- and differences d = G_+ - G_-
    R sd = G[0], jx = NZ, jy = NZ, jz = NZ;
    R sxx = NZ, syy = NZ, szz = NZ, sxy = NZ, sxz = NZ, syz = NZ;
    unroll<NP>([&](auto P) {
        constexpr int i = 2 * decltype(P)::value + 1;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const R sp = G[i] + G[i + 1];
        const R dp = G[i] - G[i + 1];
        sd += sp;
        if constexpr (cx != 0) jx += R(cx) * dp;
        if constexpr (cy != 0) jy += R(cy) * dp;
        if constexpr (cz != 0) jz += R(cz) * dp;
        if constexpr (cx != 0) sxx += R(cx * cx) * sp;
        if constexpr (cy != 0) syy += R(cy * cy) * sp;
        if constexpr (cz != 0) szz += R(cz * cz) * sp;
        if constexpr (cx * cy != 0) sxy += R(cx * cy) * sp;
        if constexpr (cx * cz != 0) sxz += R(cx * cz) * sp;
        if constexpr (cy * cz != 0) syz += R(cy * cz) * sp;
    });

    // In single precision 1 / (S rho) is the hardware reciprocal (about one
    // unit in the last place) and sd / S a product with the rounded 1 / S:
    // an IEEE division is some ten instructions, and these single-precision
    // steps are bound by instruction issue at 16-bit storage.
    R drho, inv_rho_s;  // rho - 1 and 1 / (S rho)
    if constexpr (std::is_same<R, float>::value) {
        drho = sd * IS;
        inv_rho_s = __builtin_amdgcn_rcpf(SR + sd);
    } else {
        drho = sd / SR;
        inv_rho_s = R(1) / (SR + sd);
    }
    const R rho = R(1) + drho;
    const R ux = jx * inv_rho_s, uy = jy * inv_rho_s;
    const R uz = D3 ? jz * inv_rho_s : R(0);

    // non-equilibrium momentum flux Pi = sum c c G / S - (rho-1) T0 I - rho u u,
    // kept as q = Pi / T0
    const R dT = drho * T0;
    const R qxx = (sxx * IS - dT - rho * ux * ux) * IT0;
    const R qyy = (syy * IS - dT - rho * uy * uy) * IT0;
    const R qxy = (sxy * IS - rho * ux * uy) * IT0;
    R qzz = R(0), qxz = R(0), qyz = R(0);
    if constexpr (D3) {
        qzz = (szz * IS - dT - rho * uz * uz) * IT0;
        qxz = (sxz * IS - rho * ux * uz) * IT0;
        qyz = (syz * IS - rho * uy * uz) * IT0;
    }

    // site constants: a_i = c_i.uq, A_i = c_i.q.c_i - tr Pi, B_i = c_i.bq,
    // C = u.Pi.u / T0, v = u.u / T0
    const R uqx = ux * IT0, uqy = uy * IT0;
    const R uqz = D3 ? uz * IT0 : R(0);
    R v = ux * uqx + uy * uqy;
    R trP = (qxx + qyy) * T0;
    R bqx = qxx * ux + qxy * uy, bqy = qxy * ux + qyy * uy, bqz = R(0);
    if constexpr (D3) {
        v += uz * uqz;
        trP = (qxx + qyy + qzz) * T0;
        bqx += qxz * uz;
        bqy += qyz * uz;
        bqz = qxz * ux + qyz * uy + qzz * uz;
    }
    bqx *= R(2);
    bqy *= R(2);
    bqz *= R(2);
    const R Cs = D3 ? R(0.5) * (ux * bqx + uy * bqy + uz * bqz) : R(0.5) * (ux * bqx + uy * bqy);
    const R om2 = omega * R(0.5) * IT0;

    // Per pair: a, h_n and the even / odd parts of P_m = sum_{n<=m} h_n/n!.
    // Pe_0 = Pe_1 = 1, Pe_2 = Pe_3 = 1 + h2/2, Pe_4 = Pe_5 = Pe_2 + h4/24;
    // Po_1 = Po_2 = a, Po_3 = Po_4 = a + h3/6, Po_5 = Po_3 + h5/120.
    // Ee = Pe_K - 1 and Po = Po_K.
    auto eq_parts = [&](R a, R& Ee, R& Po) {
        const R h2 = a * a - v;
        Ee = R(0.5) * h2;
        if constexpr (K == 2) {
            Po = a;
        } else {
            const R h3 = a * (h2 - R(2) * v);
            Po = a + R(1.0 / 6.0) * h3;
            if constexpr (K >= 4) {
                const R h4 = a * h3 - R(3) * v * h2;
                Ee = Ee + R(1.0 / 24.0) * h4;
                if constexpr (K == 5) {
                    const R h5 = a * h4 - R(4) * v * h3;
                    Po = Po + R(1.0 / 120.0) * h5;
                }
            }
        }
    };

    // Energy flux (kFilteredQ): Qt scaled by omega theta / (6 T0^3), the
    // factor of fhat^q in stored units.
    Sym3<R> Qs{};
    R qsx = R(0), qsy = R(0), qsz = R(0);            // qt_c
    R rxx = R(0), ryy = R(0), rzz = R(0), rxy = R(0), rxz = R(0), ryz = R(0);  // Qt.u
    R rsx = R(0), rsy = R(0), rsz = R(0);            // Qt:uu
    R d1u = R(0);                                     // 3 T0 u.qt
    if constexpr (KIND == kFilteredQ) {
        // S sum c c c (G - G^eq): only the odd part G_+ - G_- of each pair counts
        Sym3<R> t{NZ, NZ, NZ, NZ, NZ, NZ, NZ, NZ, NZ, NZ};
        unroll<NP>([&](auto P) {
            constexpr int i = 2 * decltype(P)::value + 1;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            R Ee, Po;
            eq_parts(cdot<cx, cy, cz>(uqx, uqy, uqz), Ee, Po);
            const R dneq = (G[i] - G[i + 1]) - R(2 * L::W[i]) * rho * Po;
            add_ccc<cx, cy, cz>(t, dneq);
        });
        const R cq = omega * theta * R(1.0 / (6.0 * L::T0 * L::T0 * L::T0));
        const R cs = cq * IS;
        const R Pxx = qxx * T0, Pyy = qyy * T0, Pxy = qxy * T0;
        const R Pzz = qzz * T0, Pxz = qxz * T0, Pyz = qyz * T0;
        Qs.xxx = t.xxx * cs - cq * (R(3) * ux * Pxx);
        Qs.xxy = t.xxy * cs - cq * (R(2) * ux * Pxy + uy * Pxx);
        Qs.xyy = t.xyy * cs - cq * (R(2) * uy * Pxy + ux * Pyy);
        Qs.yyy = t.yyy * cs - cq * (R(3) * uy * Pyy);
        if constexpr (D3) {
            Qs.xxz = t.xxz * cs - cq * (R(2) * ux * Pxz + uz * Pxx);
            Qs.xyz = t.xyz * cs - cq * (ux * Pyz + uy * Pxz + uz * Pxy);
            Qs.xzz = t.xzz * cs - cq * (R(2) * uz * Pxz + ux * Pzz);
            Qs.yyz = t.yyz * cs - cq * (R(2) * uy * Pyz + uz * Pyy);
            Qs.yzz = t.yzz * cs - cq * (R(2) * uz * Pyz + uy * Pzz);
            Qs.zzz = t.zzz * cs - cq * (R(3) * uz * Pzz);
        }
        qsx = Qs.xxx + Qs.xyy + Qs.xzz;
        qsy = Qs.xxy + Qs.yyy + Qs.yzz;
        qsz = Qs.xxz + Qs.yyz + Qs.zzz;
        if constexpr (K >= 4) {
            rxx = Qs.xxx * ux + Qs.xxy * uy + Qs.xxz * uz;
            ryy = Qs.xyy * ux + Qs.yyy * uy + Qs.yyz * uz;
            rzz = Qs.xzz * ux + Qs.yzz * uy + Qs.zzz * uz;
            rxy = Qs.xxy * ux + Qs.xyy * uy + Qs.xyz * uz;
            rxz = Qs.xxz * ux + Qs.xyz * uy + Qs.xzz * uz;
            ryz = Qs.xyz * ux + Qs.yyz * uy + Qs.yzz * uz;
            d1u = R(3) * T0 * (qsx * ux + qsy * uy + qsz * uz);
        }
        if constexpr (K >= 5) {
            rsx = rxx * ux + rxy * uy + rxz * uz;
            rsy = rxy * ux + ryy * uy + ryz * uz;
            rsz = rxz * ux + ryz * uy + rzz * uz;
        }
    }

    // Each pair shares a, h_n and A; a, B and the odd h_n change sign under
    // c -> -c.  With Pe / Po the even / odd parts of P_m,
    //   N_even = A Pe_{K-2} - B Po_{K-3} + C Pe_{K-4},
    //   N_odd  = A Po_{K-2} - B Pe_{K-3} + C Po_{K-4},
    //   G_+- = W [(rho-1) + rho (Pe_K - 1) + om2 N_even] +- W [rho Po_K + om2 N_odd].
    {
        // rest particle: a = 0, B = 0, A = -tr Pi, h2 = -v, h3 = 0, h4 = 3 v^2
        const R A0 = -trP;
        const R Ee2 = R(-0.5) * v;
        R Ee = Ee2;
        if constexpr (K >= 4) Ee = Ee2 + R(0.125) * v * v;
        R Xe;
        if constexpr (KIND == kBGK) {
            const R geq = R(L::W[0]) * (drho + rho * Ee);
            Xe = geq + omega * (G[0] - geq);
        } else {
            if constexpr (K <= 3) {
                Xe = drho + rho * Ee + om2 * A0;
            } else {
                Xe = drho + rho * Ee + om2 * (A0 + A0 * Ee2 + Cs);
            }
            if constexpr (KIND == kFilteredQ && K >= 4) Xe += d1u;
            Xe = R(L::W[0]) * Xe;
        }
        G[0] = Xe;
    }
    unroll<NP>([&](auto P) {
        constexpr int i = 2 * decltype(P)::value + 1;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        constexpr R Wi = R(L::W[i]);
        const R a = cdot<cx, cy, cz>(uqx, uqy, uqz);
        if constexpr (KIND == kBGK) {
            R Ee, Po;
            eq_parts(a, Ee, Po);
            const R Xe = drho + rho * Ee;
            const R Xo = rho * Po;
            const R gp = Wi * (Xe + Xo);
            const R gm = Wi * (Xe - Xo);
            G[i] = gp + omega * (G[i] - gp);
            G[i + 1] = gm + omega * (G[i + 1] - gm);
        } else {
            const R A = cquad<cx, cy, cz>(qxx, qyy, qzz, qxy, qxz, qyz) - trP;
            const R h2 = a * a - v;
            const R Ee2 = R(0.5) * h2;
            R Xe, Xo;
            if constexpr (K == 2) {
                Xe = drho + rho * Ee2 + om2 * A;
                Xo = rho * a;
            } else {
                const R B = cdot<cx, cy, cz>(bqx, bqy, bqz);
                const R h3 = a * (h2 - R(2) * v);
                const R Po3 = a + R(1.0 / 6.0) * h3;
                if constexpr (K == 3) {
                    Xe = drho + rho * Ee2 + om2 * A;
                    Xo = rho * Po3 + om2 * (A * a - B);
                } else {
                    const R h4 = a * h3 - R(3) * v * h2;
                    const R Ee4 = Ee2 + R(1.0 / 24.0) * h4;
                    const R Ne = A + A * Ee2 - B * a + Cs;
                    Xe = drho + rho * Ee4 + om2 * Ne;
                    if constexpr (K == 4) {
                        Xo = rho * Po3 + om2 * (A * a - B);
                    } else {
                        const R h5 = a * h4 - R(4) * v * h3;
                        const R Po5 = Po3 + R(1.0 / 120.0) * h5;
                        Xo = rho * Po5 + om2 * (A * Po3 - B - B * Ee2 + Cs * a);
                    }
                }
                if constexpr (KIND == kFilteredQ) {
                    // d0 (odd), d1 (even), d2 (odd) of the energy-flux part
                    const R d0 = ccc_dot<cx, cy, cz>(Qs) - R(3) * T0 * cdot<cx, cy, cz>(qsx, qsy, qsz);
                    if constexpr (K == 3) {
                        Xo += d0;
                    } else {
                        const R d1 = d1u - R(3) * cquad<cx, cy, cz>(rxx, ryy, rzz, rxy, rxz, ryz);
                        Xe += d0 * a + d1;
                        if constexpr (K == 4) {
                            Xo += d0;
                        } else {
                            const R d2 = R(3) * cdot<cx, cy, cz>(rsx, rsy, rsz);
                            Xo += d0 * (R(1) + Ee2) + d1 * a + d2;
                        }
                    }
                }
            }
            // W (Xe +- Xo) as W Xe +- W Xo: one product and two fused
            // multiply-adds instead of two sums and two products
            const R WXo = Wi * Xo;
            G[i] = fused(Wi, Xe, WXo);
            G[i + 1] = fused(Wi, Xe, -WXo);
        }
    });

    if constexpr (PROJ) {
        R m0 = G[0], mx = NZ, my = NZ, mz = NZ;
        unroll<NP>([&](auto P) {
            constexpr int i = 2 * decltype(P)::value + 1;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            const R dp = G[i] - G[i + 1];
            m0 += G[i] + G[i + 1];
            if constexpr (cx != 0) mx += R(cx) * dp;
            if constexpr (cy != 0) my += R(cy) * dp;
            if constexpr (cz != 0) mz += R(cz) * dp;
        });
        const R dm = (sd - m0) * IS;
        const R dx = (jx - mx) * (IS * IT0);
        const R dy = (jy - my) * (IS * IT0);
        const R dz = D3 ? (jz - mz) * (IS * IT0) : R(0);
        G[0] += R(L::W[0]) * dm;
        unroll<NP>([&](auto P) {
            constexpr int i = 2 * decltype(P)::value + 1;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            constexpr R Wi = R(L::W[i]);
            const R cd = cdot<cx, cy, cz>(dx, dy, dz);
            G[i] += Wi * (dm + cd);
            G[i + 1] += Wi * (dm - cd);
        });
    }
}

// Equilibrium in stored units, G_i = S (f^eq_i - w_i) (eq. hermite truncated at K).
template <class L, int K, class R>
__device__ __forceinline__ void equilibrium_scaled(R drho, R ux, R uy, R uz, R (&G)[L::Q])
{
    constexpr R IT0 = R(L::INV_T0);
    const R v = (ux * ux + uy * uy + uz * uz) * IT0;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        constexpr R Wi = R(L::W[i]);
        const R a = (R(cx) * ux + R(cy) * uy + R(cz) * uz) * IT0;
        R hm1 = R(1), h = a, E = a;
        R fact = R(1);
        for (int n = 1; n < K; ++n) {
            const R hn = a * h - R(n) * v * hm1;
            hm1 = h;
            h = hn;
            fact *= R(n + 1);
            E += h / fact;
        }
        G[i] = Wi * (drho * (R(1) + E) + E);
    });
}

}  // namespace lbm
