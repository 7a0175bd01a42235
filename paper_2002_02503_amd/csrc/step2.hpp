// Two fused time steps per launch on a single box (temporal blocking of the
// pull step), for 3-D lattices whose velocity components are at most 1 in
// magnitude (D3Q15, D3Q19).  Included by the per-pair translation units,
// which instantiate launch_step2_l for one (lattice, storage type).
#pragma once

#include "device.hpp"
#include "step_launch.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// A block owns a column of TX x TY sites of the (x, y) plane over a range of
// z-planes and walks it upwards in z.  At each plane p it
//   1. takes the step t -> t + 1 at the (TX + 2) x (TY + 2) sites of the
//      column and its one-site ring, one site per thread, pulling from HBM,
//      and writes every result into an LDS plane in the storage type (so a
//      read gives back exactly what a store to HBM and a reload would);
//   2. takes the step t + 1 -> t + 2 at the TX x TY column sites of plane
//      p - 1.  Its pulls from plane p - 1 + c_z come from the LDS plane just
//      written (c_z = -1) or from registers holding LDS values read one plane
//      (c_z = 0) or two planes (c_z = +1) earlier; thread j owns the column
//      site (j % TX, j / TX) for the whole walk, so step 2 runs on
//      TX TY / 64 whole waves.
// The state at t + 1 never reaches HBM: one launch reads and writes the state
// once per two steps.  The price is the ring, computed in step 1 only, which
// adds (TX + 2)(TY + 2) / (TX TY) - 1 of one step's arithmetic, and two extra
// step-1 planes per column segment.  Each site's arithmetic is k_step's on
// the same values, so the launch gives the bits of two k_step launches.
// The LDS planes are double-buffered: a wave that has finished step 2 at
// plane p - 1 (reading plane p's buffer) goes on to fill the other buffer with
// plane p + 1 while slower waves still read, so one barrier per plane
// suffices (the barrier after plane p + 1's writes comes after every read of
// plane p - 1's buffer, which plane p + 2 refills).
// The loads of plane p + 1 are issued before plane p's collisions, so they
// are in flight during both steps.
// Blocks are dealt to the eight XCDs in turn; with the grid a multiple of 8
// the block -> column order puts consecutive columns (which share ring rows)
// on one XCD and its L2 (measured on D3Q19 256^3 FP32: 2% faster than the
// plain order with 64 x 8 tiles, 12% with 32 x 16 ones).
// ---------------------------------------------------------------------------

template <class S>
constexpr int step2_threads()
{
    return (kTwoStepTileX + 2) * (two_step_tile_y(sizeof(S)) + 2);
}

template <class L, class S, int K, int KIND>
__global__ __launch_bounds__(step2_threads<S>(), 2) void k_step2(const S* __restrict__ src, S* __restrict__ dst,
                                                                 Step2Geom geo, typename Store<S>::R omega,
                                                                 typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int Q = L::Q;
    constexpr int TX = kTwoStepTileX, TY = two_step_tile_y(sizeof(S));
    constexpr int WX = TX + 2, NT = WX * (TY + 2);
    static_assert(L::D == 3 && L::R == 1, "a one-site ring in x, y and z");
    static_assert((TX * TY) % 64 == 0, "step 2 on whole waves");
    // How an element's address is formed.  SCALAR_BASE: a uniform row pointer
    // (z-plane, tile row m; scalar registers) plus the lane's 32-bit offset in
    // the plane, so no 64-bit vector address is held.  Otherwise the lane's
    // 64-bit address, formed at each access.  Measured on D3Q19 256^3 (A/B on
    // one GPU): the first form is 1.1-1.3% faster in FP64 and the second
    // 1.6-2.2% faster in FP32 (and for D3Q15).  The energy-flux kind takes the
    // first: its 20-60 fewer registers per lane keep it from spilling (330
    // against 400 us per FP32 step).
    constexpr bool SCALAR_BASE = sizeof(S) == 8 || KIND == kFilteredQ;
    __shared__ S lplane[2][Q][NT];

    const int tid = threadIdx.x;
    const int hx = tid % WX, hy = tid / WX;  // step-1 site in the ring-extended column
    const bool owner = tid < TX * TY;
    const int ox = tid % TX, oy = tid / TX;  // step-2 site (owners)
    const int oh = (oy + 1) * WX + ox + 1;   // the same, ring-extended
    const unsigned row_bytes = unsigned(geo.nx) * unsigned(sizeof(S));
    const unsigned tile_bytes = unsigned(Q) * row_bytes;  // one x-row's tile
    const long long plane_bytes = (long long)tile_bytes * geo.ny;

    const unsigned nb = gridDim.x;
    const long long lb =
        geo.xcd_order ? (long long)(blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : (long long)blockIdx.x;
    long long w = lb * geo.per;
    const long long wend = (w + geo.per < geo.total) ? w + geo.per : geo.total;
    while (w < wend) {  // one column segment per pass; uniform over the block
        const long long col = w / geo.nz;
        const long long seg_end = (wend < (col + 1) * geo.nz) ? wend : (col + 1) * geo.nz;
        const int za = int(w - col * geo.nz);
        const int zb = za + int(seg_end - w);
        w = seg_end;
        const int x0 = int(col % geo.ncx) * TX, y0 = int(col / geo.ncx) * TY;
        const int x = wrap_coord(x0 + hx - 1, geo.nx), y = wrap_coord(y0 + hy - 1, geo.ny);
        // Byte offsets inside a z-plane of the step-1 site's x- and
        // y-neighbours, fixed for the whole column.
        unsigned xoff[3], yoff[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xoff[k] = unsigned(wrap_coord(x + k - 1, geo.nx)) * unsigned(sizeof(S));
            yoff[k] = unsigned(wrap_coord(y + k - 1, geo.ny)) * tile_bytes;
        }
        const unsigned own = unsigned(y0 + oy) * tile_bytes + unsigned(x0 + ox) * unsigned(sizeof(S));

        // step-1 inputs of plane p (p in [-2, nz + 1])
        auto pull = [&](int p, R(&g)[Q]) {
            const char* base[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                base[k] = reinterpret_cast<const char*>(src) + (long long)wrap_coord(p + k - 1, geo.nz) * plane_bytes;
            unroll<Q>([&](auto M) {  // in tile-row order
                constexpr int m = decltype(M)::value;
                constexpr int i = mem_pop<L>(m);
                constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
                const char* p8;
                if constexpr (SCALAR_BASE)
                    p8 = (base[1 - cz] + (long long)m * row_bytes) + (yoff[1 - cy] + xoff[1 - cx]);
                else
                    p8 = base[1 - cz] + (yoff[1 - cy] + unsigned(m) * row_bytes + xoff[1 - cx]);
                g[i] = load_population<ST, cx>(reinterpret_cast<const S*>(p8));
            });
        };

        // held LDS values: read from the first plane on, used from the third
        // (k >= 2); zeroed so that no read is of an indeterminate value
        R next[Q], hold0[Q] = {}, hold1a[Q] = {}, hold1b[Q] = {};
        const int planes = zb - za + 2;  // step-1 planes za - 1 .. zb
        pull(za - 1, next);
        for (int k = 0; k < planes; ++k) {
            const int p = za - 1 + k;
            R g[Q];
            unroll<Q>([&](auto I) { g[decltype(I)::value] = next[decltype(I)::value]; });
            if (k + 1 < planes) pull(p + 1, next);
            collide_site<L, K, KIND, PROJ, R>(g, omega, theta);
            S(&buf)[Q][NT] = lplane[k & 1];
            unroll<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                ST::put(&buf[i][tid], g[i]);
            });
            __syncthreads();
            if (owner) {
                R h[Q];
                unroll<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
                    const R v = ST::get(&buf[i][oh - cx - cy * WX]);
                    if constexpr (cz == -1) {
                        h[i] = v;
                    } else if constexpr (cz == 0) {
                        h[i] = hold0[i];
                        hold0[i] = v;
                    } else {
                        h[i] = hold1b[i];
                        hold1b[i] = hold1a[i];
                        hold1a[i] = v;
                    }
                });
                if (k >= 2) {  // plane p - 1 has all its inputs
                    collide_site<L, K, KIND, PROJ, R>(h, omega, theta);
                    char* out = reinterpret_cast<char*>(dst) + (long long)wrap_coord(p - 1, geo.nz) * plane_bytes;
                    unroll<Q>([&](auto M) {
                        constexpr int m = decltype(M)::value;
                        constexpr int i = mem_pop<L>(m);
                        char* p8;
                        if constexpr (SCALAR_BASE)
                            p8 = (out + (long long)m * row_bytes) + own;
                        else
                            p8 = out + (own + unsigned(m) * row_bytes);
                        ST::put_nt(reinterpret_cast<S*>(p8), h[i]);
                    });
                }
            }
        }
        __syncthreads();  // the next segment's first plane refills buffer 0
    }
}

template <class L, class S>
hipError_t launch_step2_l(int K, int kind, const void* src, void* dst, const Step2Geom& geo, double omega,
                          double theta, int grid, hipStream_t s)
{
    if constexpr (L::D == 3 && L::R == 1) {
        return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
            using R = typename Store<S>::R;
            constexpr int KK = decltype(Kc)::value;
            constexpr int KD = decltype(Kind)::value;
            k_step2<L, S, KK, KD><<<dim3(unsigned(grid)), step2_threads<S>(), 0, s>>>(
                static_cast<const S*>(src), static_cast<S*>(dst), geo, R(omega), R(theta));
            return hipGetLastError();
        });
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace lbm
