// The fused pull-stream + collide step on a batch of boxes, templated on
// lattice, storage type, Hermite order and collision kind.  Included by the
// per-lattice translation units.
#pragma once

#include "device.hpp"
#include "step_launch.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Fused step, batch of boxes.  A tile is one wavefront's work: whole x-rows of
// one z-plane of one box (rows * nx <= 64), or a 64-site piece of one row when
// nx exceeds 64.  The box and z are uniform over the wave, so each wave reads
// its tile descriptor with one scalar load, and each lane finds its row with
// one exact reciprocal multiply.  Every row tile (all populations of one
// x-row) is written by one wave: measured, tiles that split rows between
// waves (flat 64-site runs, or rows spread over the waves of a block) leave
// partly written cache lines in every population row and run at half the
// bandwidth.  A block of W waves takes W consecutive tiles; a fixed grid walks
// the tile table (grid-stride).  One launch advances every box by one step,
// each with its own tau.  Offsets inside a box fit 32 bits (checked on the
// host).
// ---------------------------------------------------------------------------

template <class L, class S, int K, int KIND>
__global__ __launch_bounds__(256) void k_step_batch(const S* __restrict__ src, S* __restrict__ dst,
                                                    const TileDesc* __restrict__ tiles, int ntiles,
                                                    typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    const int waves = int(blockDim.x) >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);  // uniform: scalar descriptor loads
    const int tid = int(threadIdx.x) & 63;
    for (int t = int(blockIdx.x) * waves + wave; t < ntiles; t += int(gridDim.x) * waves) {
        const TileDesc b = tiles[t];
        int r, x;
        if (b.nx <= 64) {
            // (tid + 1/2) / nx is at least 1/(2 nx) away from an integer, far
            // more than the float rounding of the product: the floor is exact
            r = int((float(tid) + 0.5f) * b.inv_nx);
            x = tid - r * b.nx;
        } else {
            r = 0;
            x = b.x0 + tid;
        }
        if (r >= b.rows || x >= b.nx) continue;
        const int y = b.y0 + r;
        const int z = b.z;
        const S* sb = src + (long long)L::Q * b.offset;
        S* db = dst + (long long)L::Q * b.offset;

        int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
        for (int k = 0; k <= 2 * RR; ++k) {
            xw[k] = wrap_coord(x + k - RR, b.nx);
            yw[k] = wrap_coord(y + k - RR, b.ny);
            zw[k] = wrap_coord(z + k - RR, b.nz);
        }
        // element offset of a row tile = plane part (uniform) + row part (per lane)
        const int tq = L::Q * b.nx;
        int zo[2 * RR + 1], yo[2 * RR + 1];
#pragma unroll
        for (int k = 0; k <= 2 * RR; ++k) {
            zo[k] = zw[k] * (b.ny * tq);
            yo[k] = yw[k] * tq;
        }
        R g[L::Q];
        unroll<L::Q>([&](auto M) {  // in tile-row order
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            const int off = zo[RR - cz] + m * b.nx + (yo[RR - cy] + xw[RR - cx]);
            g[i] = load_population<ST, cx>(at32(sb, unsigned(off)));
        });

        collide_site<L, K, KIND, PROJ, R>(g, R(b.omega), theta);

        const int out_off = (z * b.ny + y) * tq + x;
        unroll<L::Q>([&](auto M) {
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);  // a constant expression: the array index must fold
            ST::put_nt(at32(db, unsigned(out_off + m * b.nx)), g[i]);
        });
    }
}

template <class L, class S>
hipError_t launch_step_batch_l(int K, int kind, const void* src, void* dst, const TileDesc* tiles, int ntiles,
                               double theta, int block, int grid, hipStream_t s)
{
    return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        constexpr int KD = decltype(Kind)::value;
        const int waves = block / 64;
        const int need = (ntiles + waves - 1) / waves;  // blocks that give every tile its own wave
        const int g = (grid > 0 && grid < need) ? grid : need;
        k_step_batch<L, S, KK, KD><<<g, block, 0, s>>>(static_cast<const S*>(src), static_cast<S*>(dst), tiles,
                                                       ntiles, R(theta));
        return hipGetLastError();
    });
}

}  // namespace lbm
