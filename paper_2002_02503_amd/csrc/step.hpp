// The fused pull-stream + collide step on a single box: one site per thread
// (k_step, k_step_pair, and the in-place forms k_step_ip and k_step_tw) or V
// sites per lane (k_step_vec), templated on lattice, storage type, Hermite
// order and collision kind.  Included by the per-lattice
// translation units, which instantiate the launchers for one lattice.
#pragma once

#include "device.hpp"
#include "step_launch.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Fused step, single box, one site per thread.  The grid is (x-blocks, ny,
// nz): a block covers blockDim.x sites of one x-row, so y, z and the source
// row of every population are block-uniform; only the x wrap is per lane.
// Every access is a uniform 64-bit pointer (row tile + population row) plus a
// 32-bit lane offset.
// ---------------------------------------------------------------------------

template <class L, class S, int K, int KIND>
__global__ __launch_bounds__(256) void k_step(const S* __restrict__ src, S* __restrict__ dst, StepGeom geo,
                                              typename Store<S>::R omega, typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const int x = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (x >= geo.nx) return;
    const long long tile = (long long)L::Q * geo.nx;  // elements per row tile

    int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * RR; ++k) {
        xw[k] = wrap_coord(x + k - RR, geo.nx);
        yw[k] = wrap_coord(y + k - RR, geo.ny);
        zw[k] = wrap_coord(z + k - RR, geo.nz);
    }

    R g[L::Q];
    unroll<L::Q>([&](auto M) {  // in tile-row order
        constexpr int m = decltype(M)::value;
        constexpr int i = mem_pop<L>(m);
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const int row = zw[RR - cz] * geo.ny + yw[RR - cy];
        const S* p = src + row * tile + (long long)m * geo.nx;
        g[i] = load_population<ST, cx>(at32(p, unsigned(xw[RR - cx])));
    });

    collide_site<L, K, KIND, PROJ, R>(g, omega, theta);

    S* q = dst + (long long)(z * geo.ny + y) * tile;
    unroll<L::Q>([&](auto M) {
        constexpr int m = decltype(M)::value;
        constexpr int i = mem_pop<L>(m);  // a constant expression: the array index must fold
        ST::put_nt(at32(q + (long long)m * geo.nx, unsigned(x)), g[i]);
    });
}

// ---------------------------------------------------------------------------
// Fused step, single box, two sites per thread: the sites at x of the rows
// y0 = 2 blockIdx.y and y0 + 1 (ny even).  Both sites' populations are loaded
// before the first site collides, so while one site computes, the other's
// loads are in flight; the in-order memory counter lets the second site's
// loads complete while the first site's stores are still outstanding.  The
// per-site arithmetic is that of k_step (the same bits).
// ---------------------------------------------------------------------------

template <class L, class S, int K, int KIND>
__global__ __launch_bounds__(256) void k_step_pair(const S* __restrict__ src, S* __restrict__ dst, StepGeom geo,
                                                   typename Store<S>::R omega, typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    const int y0 = 2 * int(blockIdx.y);
    const int z = blockIdx.z;
    const int x = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (x >= geo.nx) return;
    const long long tile = (long long)L::Q * geo.nx;

    // yw[k] = y0 + k - RR for k = 0 .. 2 RR + 1 (both rows' neighbourhoods)
    int xw[2 * RR + 1], yw[2 * RR + 2], zw[2 * RR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * RR; ++k) {
        xw[k] = wrap_coord(x + k - RR, geo.nx);
        zw[k] = wrap_coord(z + k - RR, geo.nz);
    }
#pragma unroll
    for (int k = 0; k <= 2 * RR + 1; ++k) yw[k] = wrap_coord(y0 + k - RR, geo.ny);

    R g[2][L::Q];
    unroll<2>([&](auto Sj) {
        constexpr int sj = decltype(Sj)::value;
        unroll<L::Q>([&](auto M) {  // in tile-row order
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            const int row = zw[RR - cz] * geo.ny + yw[sj + RR - cy];
            const S* p = src + row * tile + (long long)m * geo.nx;
            g[sj][i] = load_population<ST, cx>(at32(p, unsigned(xw[RR - cx])));
        });
    });
    unroll<2>([&](auto Sj) {
        constexpr int sj = decltype(Sj)::value;
        collide_site<L, K, KIND, PROJ, R>(g[sj], omega, theta);
        S* q = dst + (long long)(z * geo.ny + y0 + sj) * tile;
        unroll<L::Q>([&](auto M) {
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);
            ST::put_nt(at32(q + (long long)m * geo.nx, unsigned(x)), g[sj][i]);
        });
    });
}

// ---------------------------------------------------------------------------
// Fused step, single box, in place: one buffer, two alternating forms.
// The state is in one of two layouts:
//   natural: tile row m(i) of site x holds the post-collision population i of
//            site x (the layout every other kernel reads and writes);
//   swapped: the post-collision population i of site x sits at site x + c_i,
//            in tile row m(opp(i)).
// From natural, site x reads population i from site x - c_i, tile row m(i)
// (the pull of k_step), collides, and writes its result for direction
// opp(i) back to that same element, which leaves the state swapped.  From
// swapped, site x finds population i in its own tile row m(opp(i)) and writes
// population j to its own tile row m(j), which leaves it natural.  Each
// element is read and then written by one thread only, so no second buffer is
// needed and there is no race; two steps stream every population exactly as
// two pull steps do, and the per-site arithmetic is that of k_step (the same
// bits).  A row's reads and writes touch the same lines, which the memory
// system serves faster than the two separate buffers of k_step.
// ---------------------------------------------------------------------------

template <class L, class S, int K, int KIND, bool FROM_NATURAL>
__global__ __launch_bounds__(256) void k_step_ip(S* __restrict__ buf, StepGeom geo, typename Store<S>::R omega,
                                                 typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const int x = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (x >= geo.nx) return;
    const long long tile = (long long)L::Q * geo.nx;

    R g[L::Q];
    if constexpr (FROM_NATURAL) {
        int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
        for (int k = 0; k <= 2 * RR; ++k) {
            xw[k] = wrap_coord(x + k - RR, geo.nx);
            yw[k] = wrap_coord(y + k - RR, geo.ny);
            zw[k] = wrap_coord(z + k - RR, geo.nz);
        }
        // element of population i at site x - c_i: uniform row pointer, lane offset
        auto elem = [&](auto M) -> S* {
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            const int row = zw[RR - cz] * geo.ny + yw[RR - cy];
            return at32(buf + row * tile + (long long)m * geo.nx, unsigned(xw[RR - cx]));
        };
        unroll<L::Q>([&](auto M) {  // in tile-row order
            constexpr int i = mem_pop<L>(decltype(M)::value);
            g[i] = load_population<ST, L::c[i][0]>(elem(M));
        });
        collide_site<L, K, KIND, PROJ, R>(g, omega, theta);
        unroll<L::Q>([&](auto M) {
            constexpr int i = mem_pop<L>(decltype(M)::value);
            constexpr int io = opp(i);
            const R v = g[io];
            if constexpr (L::c[i][0] == 0) ST::put_nt(elem(M), v);
            else ST::put(elem(M), v);
        });
    } else {
        S* q = buf + (long long)(z * geo.ny + y) * tile;
        unroll<L::Q>([&](auto M) {
            constexpr int m = decltype(M)::value;
            constexpr int i = opp(mem_pop<L>(m));
            g[i] = ST::get_nt(at32(q + (long long)m * geo.nx, unsigned(x)));
        });
        collide_site<L, K, KIND, PROJ, R>(g, omega, theta);
        unroll<L::Q>([&](auto M) {
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);
            ST::put_nt(at32(q + (long long)m * geo.nx, unsigned(x)), g[i]);
        });
    }
}

// ---------------------------------------------------------------------------
// Fused step, single box, in place with the twisted layouts ("esoteric twist").
// The populations of site x are kept at the cells x + b_i, b_i the positive
// part of c_i component by component (lattice.hpp, twist_offset); population
// i is in tile row m(i) at even times and m(opp(i)) at odd times.  Site x
// finds its incoming population i (f'_i of site x - c_i) at the cell
// x - c_i + b_i = x + b_opp(i): tile row m(i) at an even time, m(opp(i)) at
// an odd one.  After the collision it writes its population opp(i) back into
// that same element, which is where that population belongs at the next
// time.  So every step reads and writes each element once, by one thread,
// and every step of both parities touches only the cells x + b: for D3Q19
// four row tiles (own, +y, +z, +y+z) and x offsets 0 and +1, for D3Q39 nine
// row tiles and x offsets 0..3.  The per-site arithmetic is that of k_step
// (the same bits).
// ---------------------------------------------------------------------------

template <class L, class S, int K, int KIND, bool EVEN>
__global__ __launch_bounds__(256) void k_step_tw(S* __restrict__ buf, StepGeom geo, typename Store<S>::R omega,
                                                 typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const int x = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (x >= geo.nx) return;
    const long long tile = (long long)L::Q * geo.nx;

    int xw[RR + 1], yw[RR + 1], zw[RR + 1];
#pragma unroll
    for (int k = 0; k <= RR; ++k) {
        xw[k] = wrap_coord(x + k, geo.nx);
        yw[k] = wrap_coord(y + k, geo.ny);
        zw[k] = wrap_coord(z + k, geo.nz);
    }
    // tile row m holds, for this site, population pop_in_row(m) at the cell
    // x + b_opp(pop_in_row(m))
    auto elem = [&](auto M) -> S* {
        constexpr int m = decltype(M)::value;
        constexpr int i = EVEN ? mem_pop<L>(m) : opp(mem_pop<L>(m));
        constexpr int io = opp(i);
        const int row = zw[twist_offset<L>(io, 2)] * geo.ny + yw[twist_offset<L>(io, 1)];
        return at32(buf + row * tile + (long long)m * geo.nx, unsigned(xw[twist_offset<L>(io, 0)]));
    };
    R g[L::Q];
    unroll<L::Q>([&](auto M) {  // in tile-row order
        constexpr int i = EVEN ? mem_pop<L>(decltype(M)::value) : opp(mem_pop<L>(decltype(M)::value));
        // elements at the site's own x belong to this wavefront alone
        if constexpr (twist_offset<L>(opp(i), 0) == 0) g[i] = ST::get_nt(elem(M));
        else g[i] = ST::get(elem(M));
    });
    collide_site<L, K, KIND, PROJ, R>(g, omega, theta);
    unroll<L::Q>([&](auto M) {
        constexpr int i = EVEN ? mem_pop<L>(decltype(M)::value) : opp(mem_pop<L>(decltype(M)::value));
        constexpr int io = opp(i);
        const R v = g[io];
        if constexpr (twist_offset<L>(io, 0) == 0) ST::put_nt(elem(M), v);
        else ST::put(elem(M), v);
    });
}

template <class L, class S, int K, int KIND>
__global__ __launch_bounds__(256) void k_step_vec(const S* __restrict__ src, S* __restrict__ dst, VecGeom geo,
                                                  typename Store<S>::R omega, typename Store<S>::R theta)
{
    using R = typename Store<S>::R;
    constexpr int V = vec_sites<S>();
    using IO = VecIO<S, V>;
    using VT = typename IO::VT;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;
    static_assert(RR < V, "a shifted population must come from at most one neighbouring lane");

    const int lane = int(threadIdx.x) & 63;
    const int wave = int(blockIdx.x) * (int(blockDim.x) >> 6) + (int(threadIdx.x) >> 6);
    const int lpr = geo.lanes_per_row;
    const int r = lane / lpr;          // row within the wave
    const int li = lane - r * lpr;     // lane within the row
    const int row = wave * geo.rows_per_wave + r;
    // Lanes past the last row of the wave, or past the last row of the box,
    // leave now; every lane that stays only reads lanes of its own row.
    if (r >= geo.rows_per_wave || row >= geo.nrows) return;
    const int prev = r * lpr + (li == 0 ? lpr - 1 : li - 1);
    const int next = r * lpr + (li == lpr - 1 ? 0 : li + 1);
    const int y = row % geo.ny;
    const int z = row / geo.ny;
    const long long tile = (long long)L::Q * geo.nx;
    int yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * RR; ++k) {
        yw[k] = wrap_coord(y + k - RR, geo.ny);
        zw[k] = wrap_coord(z + k - RR, geo.nz);
    }

    R g[V][L::Q];
    unroll<L::Q>([&](auto M) {  // in tile-row order
        constexpr int m = decltype(M)::value;
        constexpr int i = mem_pop<L>(m);
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const long long srow = zw[RR - cz] * geo.ny + yw[RR - cy];
        const S* p = src + srow * tile + (long long)m * geo.nx;
        R own[V];
        // every lane reads its own aligned V-site chunk: no line is shared
        IO::unpack(__builtin_nontemporal_load(reinterpret_cast<const VT*>(p + (long long)li * V)), own);
        // site j pulls from x_j - c_x: element j - c_x of this lane when it is
        // in [0, V), otherwise the wrapped element of the neighbouring lane
        unroll<V>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr int e = j - cx;
            if constexpr (e >= 0 && e < V) {
                g[j][i] = own[e];
            } else if constexpr (e < 0) {
                g[j][i] = __shfl(own[e + V], prev, 64);
            } else {
                g[j][i] = __shfl(own[e - V], next, 64);
            }
        });
    });

    unroll<V>([&](auto J) {
        constexpr int j = decltype(J)::value;
        collide_site<L, K, KIND, PROJ, R>(g[j], omega, theta);
    });

    S* q = dst + (long long)row * tile + (long long)li * V;
    unroll<L::Q>([&](auto M) {
        constexpr int m = decltype(M)::value;
        constexpr int i = mem_pop<L>(m);
        R v[V];
        unroll<V>([&](auto J) {
            constexpr int j = decltype(J)::value;
            v[j] = g[j][i];
        });
        __builtin_nontemporal_store(IO::pack(v), reinterpret_cast<VT*>(q + (long long)m * geo.nx));
    });
}

template <class L, class S>
hipError_t launch_step_l(int K, int kind, const void* src, void* dst, const StepGeom& geo, double omega,
                         double theta, int block, bool pair, hipStream_t s)
{
    return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        constexpr int KD = decltype(Kind)::value;
        if (pair) {
            if (geo.ny % 2 != 0) return hipErrorInvalidValue;
            k_step_pair<L, S, KK, KD>
                <<<dim3(unsigned(geo.xblocks), unsigned(geo.ny / 2), unsigned(geo.nz)), block, 0, s>>>(
                    static_cast<const S*>(src), static_cast<S*>(dst), geo, R(omega), R(theta));
        } else {
            k_step<L, S, KK, KD><<<dim3(unsigned(geo.xblocks), unsigned(geo.ny), unsigned(geo.nz)), block, 0, s>>>(
                static_cast<const S*>(src), static_cast<S*>(dst), geo, R(omega), R(theta));
        }
        return hipGetLastError();
    });
}

template <class L, class S>
hipError_t launch_step_ip_l(int K, int kind, void* buf, bool from_natural, const StepGeom& geo, double omega,
                            double theta, int block, hipStream_t s)
{
    return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        constexpr int KD = decltype(Kind)::value;
        const dim3 grid(unsigned(geo.xblocks), unsigned(geo.ny), unsigned(geo.nz));
        if (from_natural)
            k_step_ip<L, S, KK, KD, true><<<grid, block, 0, s>>>(static_cast<S*>(buf), geo, R(omega), R(theta));
        else
            k_step_ip<L, S, KK, KD, false><<<grid, block, 0, s>>>(static_cast<S*>(buf), geo, R(omega), R(theta));
        return hipGetLastError();
    });
}

template <class L, class S>
hipError_t launch_step_tw_l(int K, int kind, void* buf, bool even, const StepGeom& geo, double omega, double theta,
                            int block, hipStream_t s)
{
    return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        constexpr int KD = decltype(Kind)::value;
        const dim3 grid(unsigned(geo.xblocks), unsigned(geo.ny), unsigned(geo.nz));
        if (even)
            k_step_tw<L, S, KK, KD, true><<<grid, block, 0, s>>>(static_cast<S*>(buf), geo, R(omega), R(theta));
        else
            k_step_tw<L, S, KK, KD, false><<<grid, block, 0, s>>>(static_cast<S*>(buf), geo, R(omega), R(theta));
        return hipGetLastError();
    });
}

template <class L, class S>
int vec_sites_l()
{
    return (L::R < vec_sites<S>()) ? vec_sites<S>() : 0;
}

template <class L, class S>
hipError_t launch_step_vec_l(int K, int kind, const void* src, void* dst, const VecGeom& geo, double omega,
                             double theta, hipStream_t s)
{
    if constexpr (L::R < vec_sites<S>()) {
        return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
            using R = typename Store<S>::R;
            constexpr int KK = decltype(Kc)::value;
            constexpr int KD = decltype(Kind)::value;
            const long long waves = (geo.nrows + geo.rows_per_wave - 1) / geo.rows_per_wave;
            const long long nblocks = (waves + 3) / 4;
            k_step_vec<L, S, KK, KD><<<dim3((unsigned)nblocks), 256, 0, s>>>(
                static_cast<const S*>(src), static_cast<S*>(dst), geo, R(omega), R(theta));
            return hipGetLastError();
        });
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace lbm
