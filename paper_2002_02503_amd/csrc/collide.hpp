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

template <class L, int K, bool PROJ, class R>
__device__ __forceinline__ void collide_site(R (&G)[L::Q], R omega)
{
    static_assert(K >= 2 && K <= L::K_MAX, "Hermite order outside 2..2N-1");
    constexpr R IT0 = R(L::INV_T0);
    constexpr R T0 = R(L::T0);
    constexpr R SR = R(L::S);
    constexpr R IS = R(1.0 / L::S);

    // zeroth, first and second moments (eq. mme, eq. Mflux), scaled by S
    R sd = R(0), jx = R(0), jy = R(0), jz = R(0);
    R sxx = R(0), syy = R(0), szz = R(0), sxy = R(0), sxz = R(0), syz = R(0);
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const R gi = G[i];
        sd += gi;
        if constexpr (cx != 0) jx += R(cx) * gi;
        if constexpr (cy != 0) jy += R(cy) * gi;
        if constexpr (cz != 0) jz += R(cz) * gi;
        if constexpr (cx != 0) sxx += R(cx * cx) * gi;
        if constexpr (cy != 0) syy += R(cy * cy) * gi;
        if constexpr (cz != 0) szz += R(cz * cz) * gi;
        if constexpr (cx * cy != 0) sxy += R(cx * cy) * gi;
        if constexpr (cx * cz != 0) sxz += R(cx * cz) * gi;
        if constexpr (cy * cz != 0) syz += R(cy * cz) * gi;
    });

    const R drho = sd / SR;
    const R rho = R(1) + drho;
    const R rho_s = SR + sd;  // S rho
    const R ux = jx / rho_s, uy = jy / rho_s, uz = jz / rho_s;

    // non-equilibrium momentum flux Pi = sum c c G / S - (rho-1) T0 I - rho u u
    const R dT = drho * T0;
    const R pxx = sxx * IS - dT - rho * ux * ux;
    const R pyy = syy * IS - dT - rho * uy * uy;
    const R pzz = (L::D == 3) ? szz * IS - dT - rho * uz * uz : R(0);
    const R pxy = sxy * IS - rho * ux * uy;
    const R pxz = (L::D == 3) ? sxz * IS - rho * ux * uz : R(0);
    const R pyz = (L::D == 3) ? syz * IS - rho * uy * uz : R(0);
    const R trP = pxx + pyy + pzz;
    const R pux = pxx * ux + pxy * uy + pxz * uz;
    const R puy = pxy * ux + pyy * uy + pyz * uz;
    const R puz = pxz * ux + pyz * uy + pzz * uz;
    const R Cs = (ux * pux + uy * puy + uz * puz) * IT0;
    const R v = (ux * ux + uy * uy + uz * uz) * IT0;
    const R om2 = omega * R(0.5) * IT0;

    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        constexpr R Wi = R(L::W[i]);
        const R a = (R(cx) * ux + R(cy) * uy + R(cz) * uz) * IT0;
        // scalar Hermite polynomials and their partial sums
        const R h1 = a;
        const R h2 = a * a - v;
        R h3 = R(0), h4 = R(0), h5 = R(0);
        if constexpr (K >= 3) h3 = a * h2 - R(2) * v * h1;
        if constexpr (K >= 4) h4 = a * h3 - R(3) * v * h2;
        if constexpr (K >= 5) h5 = a * h4 - R(4) * v * h3;
        // E_m = P_m - 1
        const R E1 = h1;
        const R E2 = E1 + h2 * R(0.5);
        const R E3 = E2 + h3 * R(1.0 / 6.0);
        const R E4 = E3 + h4 * R(1.0 / 24.0);
        const R E5 = E4 + h5 * R(1.0 / 120.0);
        R EK;
        if constexpr (K == 2) EK = E2;
        else if constexpr (K == 3) EK = E3;
        else if constexpr (K == 4) EK = E4;
        else EK = E5;
        // A_i = c.Pi.c / T0 - tr Pi,  B_i = 2 c.Pi.u / T0
        const R cPc = R(cx * cx) * pxx + R(cy * cy) * pyy + R(cz * cz) * pzz +
                      R(2 * cx * cy) * pxy + R(2 * cx * cz) * pxz + R(2 * cy * cz) * pyz;
        const R Ai = cPc * IT0 - trP;
        const R Bi = R(2) * (R(cx) * pux + R(cy) * puy + R(cz) * puz) * IT0;
        R N;
        if constexpr (K == 2) N = Ai;
        else if constexpr (K == 3) N = Ai * (R(1) + E1) - Bi;
        else if constexpr (K == 4) N = Ai * (R(1) + E2) - Bi * (R(1) + E1) + Cs;
        else N = Ai * (R(1) + E3) - Bi * (R(1) + E2) + Cs * (R(1) + E1);
        G[i] = Wi * (drho * (R(1) + EK) + EK) + Wi * om2 * N;
    });

    if constexpr (PROJ) {
        R m0 = R(0), mx = R(0), my = R(0), mz = R(0);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            const R gi = G[i];
            m0 += gi;
            if constexpr (cx != 0) mx += R(cx) * gi;
            if constexpr (cy != 0) my += R(cy) * gi;
            if constexpr (cz != 0) mz += R(cz) * gi;
        });
        const R dm = (sd - m0) * IS;
        const R dx = (jx - mx) * (IS * IT0);
        const R dy = (jy - my) * (IS * IT0);
        const R dz = (jz - mz) * (IS * IT0);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            constexpr R Wi = R(L::W[i]);
            G[i] += Wi * (dm + R(cx) * dx + R(cy) * dy + R(cz) * dz);
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
