// Lattice descriptors for the GPU path: velocity sets c_i, weights w_i and the
// lattice temperature T0 of D2Q9, D3Q15, D3Q19 and D3Q39.
//
// A lattice is "2N-th order isotropic" when sum_i w_i c_i...c_i (n times)
// equals T0^(n/2) times the n-th order Kronecker-delta tensor for even
// n <= 2N and vanishes for odd n (eq. iso, section "Basic Filtered Collision
// Formulation").  D2Q9, D3Q15 and D3Q19 have 2N = 4 with T0 = 1/3; D3Q39 has
// 2N = 6 with T0 = 2/3 (its six shell weights are the unique positive
// solution of eq. iso through sixth order).
//
// Weight quantum.  Every weight is an integer multiple of 1/S (S = 36 for
// D2Q9 and D3Q19, 72 for D3Q15, 6480 for D3Q39), so W_i = S w_i are small
// integers, exact in
// any floating-point type.  The kernels keep the populations in these units
// (see collide.hpp): no rounded weight ever enters the arithmetic.
//
// Velocity order.  The rest velocity comes first; every other velocity is
// followed by its opposite (c_{2k} = -c_{2k-1}), so kernels can treat the
// (Q-1)/2 pairs together.
//
// Every table is a compile-time constant.  Kernels index them only with
// compile-time indices (through `unroll`), so each c_i component and weight is
// folded into the instruction stream: zero components disappear and +/-1
// multiplications become adds.
#pragma once

#include <cstdint>
#include <type_traits>
#include <utility>

#if defined(__HIP__)
#include <hip/hip_runtime.h>
#else
#define __host__
#define __device__
#define __forceinline__ inline
#endif

namespace lbm {

enum LatticeId : int { kD2Q9 = 0, kD3Q19 = 1, kD3Q39 = 2, kD3Q15 = 3 };

// Collision operators of the step (collide.hpp): the filtered operator, BGK
// with the same truncated equilibrium, and the filtered operator with the
// energy-flux term of weight theta.
enum CollisionKind : int { kFiltered = 0, kBGK = 1, kFilteredQ = 2 };

struct D2Q9 {
    static constexpr int id = kD2Q9;
    static constexpr int D = 2, Q = 9, TWO_N = 4, K_DEFAULT = 3, K_MAX = 3;
    static constexpr int R = 1;  // largest |c_i component|
    static constexpr double T0 = 1.0 / 3.0, INV_T0 = 3.0;
    static constexpr int S = 36;
    static constexpr int W[Q] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    static constexpr int8_t c[Q][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    static constexpr double w[Q] = {
        4.0 / 9.0,
        1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

struct D3Q15 {
    static constexpr int id = kD3Q15;
    static constexpr int D = 3, Q = 15, TWO_N = 4, K_DEFAULT = 3, K_MAX = 3;
    static constexpr int R = 1;
    static constexpr double T0 = 1.0 / 3.0, INV_T0 = 3.0;
    static constexpr int S = 72;
    static constexpr int W[Q] = {16, 8, 8, 8, 8, 8, 8, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int8_t c[Q][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
        {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
    static constexpr double w[Q] = {
        2.0 / 9.0,
        1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
        1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0,
        1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0};
};

struct D3Q19 {
    static constexpr int id = kD3Q19;
    static constexpr int D = 3, Q = 19, TWO_N = 4, K_DEFAULT = 3, K_MAX = 3;
    static constexpr int R = 1;
    static constexpr double T0 = 1.0 / 3.0, INV_T0 = 3.0;
    static constexpr int S = 36;
    static constexpr int W[Q] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int8_t c[Q][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr double w[Q] = {
        1.0 / 3.0,
        1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

struct D3Q39 {
    static constexpr int id = kD3Q39;
    static constexpr int D = 3, Q = 39, TWO_N = 6, K_DEFAULT = 4, K_MAX = 5;
    static constexpr int R = 3;
    static constexpr double T0 = 2.0 / 3.0, INV_T0 = 1.5;
    static constexpr int S = 6480;
    static constexpr int W[Q] = {540, 540, 540, 540, 540, 540, 540,
                                 240, 240, 240, 240, 240, 240, 240, 240,
                                 96, 96, 96, 96, 96, 96,
                                 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15,
                                 4, 4, 4, 4, 4, 4};
    static constexpr int8_t c[Q][3] = {
        {0, 0, 0},
        // |c| = 1, axis
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        // (+-1, +-1, +-1)
        {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
        {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1},
        // (+-2, 0, 0) and permutations
        {2, 0, 0}, {-2, 0, 0}, {0, 2, 0}, {0, -2, 0}, {0, 0, 2}, {0, 0, -2},
        // (+-2, +-2, 0) and permutations
        {2, 2, 0}, {-2, -2, 0}, {2, -2, 0}, {-2, 2, 0},
        {2, 0, 2}, {-2, 0, -2}, {2, 0, -2}, {-2, 0, 2},
        {0, 2, 2}, {0, -2, -2}, {0, 2, -2}, {0, -2, 2},
        // (+-3, 0, 0) and permutations
        {3, 0, 0}, {-3, 0, 0}, {0, 3, 0}, {0, -3, 0}, {0, 0, 3}, {0, 0, -3}};
    static constexpr double w[Q] = {
        1.0 / 12.0,
        1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0,
        1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0,
        1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0,
        2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0,
        1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
        1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
        1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
        1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0};
};

// W_i = S w_i exactly, and the W_i add up to S.
template <class L>
constexpr bool integer_weights_consistent()
{
    int sum = 0;
    for (int i = 0; i < L::Q; ++i) {
        const double d = L::S * L::w[i] - L::W[i];
        if (d > 1e-12 || d < -1e-12) return false;
        sum += L::W[i];
    }
    return sum == L::S;
}
// Rest velocity first, then opposite pairs with equal weights.
template <class L>
constexpr bool opposite_pairs()
{
    if (L::c[0][0] != 0 || L::c[0][1] != 0 || L::c[0][2] != 0 || (L::Q % 2) != 1) return false;
    for (int k = 1; k < L::Q; k += 2)
        for (int a = 0; a < 3; ++a)
            if (L::c[k + 1][a] != -L::c[k][a] || L::W[k + 1] != L::W[k]) return false;
    return true;
}
static_assert(opposite_pairs<D2Q9>() && opposite_pairs<D3Q15>() && opposite_pairs<D3Q19>() &&
                  opposite_pairs<D3Q39>(),
              "pair order");

static_assert(integer_weights_consistent<D2Q9>(), "D2Q9 weight quantum");
static_assert(integer_weights_consistent<D3Q15>(), "D3Q15 weight quantum");
static_assert(integer_weights_consistent<D3Q19>(), "D3Q19 weight quantum");
static_assert(integer_weights_consistent<D3Q39>(), "D3Q39 weight quantum");

// Index of the velocity opposite to c_i (rest first, then pairs (2k-1, 2k)).
constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Twisted layouts of the in-place "twist" step (step.hpp, k_step_tw): the
// populations of site x are kept at the cells x + b_i, b_i the positive part
// of c_i, component by component.  Population i of site x is in tile row m(i)
// at even times and in tile row m(opp(i)) at odd times.
template <class L>
constexpr int twist_offset(int i, int a)
{
    return L::c[i][a] > 0 ? L::c[i][a] : 0;
}

// Memory order of the populations inside a row tile: sorted by (c_z, c_y, c_x),
// so the populations a step pulls from one neighbouring row tile are adjacent
// rows of that tile.  mem_row(i) is the tile row of population i, mem_pop(m)
// the population stored in tile row m.
template <class L>
constexpr int mem_row(int i)
{
    int rank = 0;
    const int R = L::R, W = 2 * L::R + 1;
    const int ki = ((L::c[i][2] + R) * W + (L::c[i][1] + R)) * W + (L::c[i][0] + R);
    for (int j = 0; j < L::Q; ++j) {
        const int kj = ((L::c[j][2] + R) * W + (L::c[j][1] + R)) * W + (L::c[j][0] + R);
        if (kj < ki) ++rank;
    }
    return rank;
}

template <class L>
constexpr int mem_pop(int m)
{
    for (int i = 0; i < L::Q; ++i)
        if (mem_row<L>(i) == m) return i;
    return -1;
}

template <class L>
constexpr bool mem_order_is_permutation()
{
    for (int m = 0; m < L::Q; ++m)
        if (mem_pop<L>(m) < 0 || mem_row<L>(mem_pop<L>(m)) != m) return false;
    return true;
}
static_assert(mem_order_is_permutation<D2Q9>() && mem_order_is_permutation<D3Q15>() &&
                  mem_order_is_permutation<D3Q19>() && mem_order_is_permutation<D3Q39>(),
              "tile row order");

// Calls f(std::integral_constant<int, i>{}) for i = 0 .. N-1, fully unrolled.
template <class F, int... I>
__host__ __device__ __forceinline__ void unroll_impl(F&& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}

template <int N, class F>
__host__ __device__ __forceinline__ void unroll(F&& f)
{
    unroll_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace lbm
