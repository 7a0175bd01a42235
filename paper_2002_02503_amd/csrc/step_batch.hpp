// The fused pull-stream + collide step on a batch of boxes, templated on
// lattice, storage type, Hermite order and collision kind.  Included by the
// per-lattice translation units.
#pragma once

#include "device.hpp"
#include "step_launch.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Fused step, batch of boxes, blocked layout (BoxDesc, w = 64).  A tile is one
// block: 64 consecutive sites of a box in x-fastest order, whatever its row
// length, so every lane of a wave has a site (but in the box's last block).
// The wave writes each population of its block as one aligned run of 64
// values.  A population shifted by c is read, for the sites away from the
// periodic seams, as one run of 64 consecutive values in the box's site order,
// shifted by c_x + nx (c_y + ny c_z) and so spread over at most two blocks;
// the neighbouring tiles read the rest of those lines at about the same time.
// (Measured against tiles of whole x-rows in row tiles, where a short row
// leaves partly used lines in every population row and idle lanes: 60% -> 75%
// of the HBM peak on 256 boxes of sides 16..64.)  The box and its geometry are
// uniform over the wave, so each wave reads its tile descriptor with one
// scalar load.  A block of W waves takes W consecutive tiles; a fixed grid
// walks the tile table (grid-stride).  One launch advances every box by one
// step, each with its own tau.  Offsets inside a box fit 32 bits (checked on
// the host).
//
// ALIGNED_ROWS (every box has nx a multiple of 64): a population with c_x = 0
// is then read in whole blocks, by this wave alone, and is loaded
// non-temporally like the own-site population; otherwise only the rest
// population c = 0 is.
// ---------------------------------------------------------------------------

template <class L, class S, int K, int KIND, bool ALIGNED_ROWS>
__global__ __launch_bounds__(256) void k_step_batch(const S* __restrict__ src, S* __restrict__ dst,
                                                    const TileDesc* __restrict__ tiles, int ntiles,
                                                    typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;
    constexpr int Q = L::Q;

    const int waves = int(blockDim.x) >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);  // uniform: scalar descriptor loads
    const int lane = int(threadIdx.x) & 63;
    for (int t = int(blockIdx.x) * waves + wave; t < ntiles; t += int(gridDim.x) * waves) {
        const TileDesc b = tiles[t];
        if (lane >= b.count) continue;
        // The lane's site l = blk * 64 + lane, from the block's first site on.
        // xx < nx + 64 and yy < ny + 64, so (xx + 1/2) / nx is at least
        // 1/(2 nx) away from an integer while the float rounding of the
        // product is below (xx + 1/2) 2^-23 < 1/(2 nx) for xx < 2^22 (ny and
        // nz are at most 65535): the floor is the exact quotient.
        const int xx = b.x0 + lane;
        const int dy = int((float(xx) + 0.5f) * b.inv_nx);
        const int x = xx - dy * b.nx;
        const int yy = b.y0 + dy;
        const int dz = int((float(yy) + 0.5f) * b.inv_ny);
        const int y = yy - dz * b.ny;
        const int z = b.z0 + dz;

        int xw[2 * RR + 1], yo[2 * RR + 1], zo[2 * RR + 1];
#pragma unroll
        for (int k = 0; k <= 2 * RR; ++k) {
            xw[k] = wrap_coord(x + k - RR, b.nx);
            yo[k] = wrap_coord(y + k - RR, b.ny) * b.nx;
            zo[k] = wrap_coord(z + k - RR, b.nz) * (b.ny * b.nx);
        }
        const S* sb = src + b.mem;
        R g[Q];
        unroll<Q>([&](auto M) {  // in tile-row order
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);  // a constant expression: the array index must fold
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            constexpr bool nt = (cx == 0 && cy == 0 && cz == 0) || (ALIGNED_ROWS && cx == 0);
            const int l = zo[RR - cz] + yo[RR - cy] + xw[RR - cx];  // source site
            // element (l / 64) Q 64 + m 64 + l % 64, with the constant m 64
            // left for the instruction's offset field
            const unsigned e = unsigned(l) + (unsigned(l) >> 6) * unsigned(64 * (Q - 1));
            const S* p = at32(sb, e) + m * 64;
            if constexpr (nt) g[i] = ST::get_nt(p);
            else g[i] = ST::get(p);
        });

        collide_site<L, K, KIND, PROJ, R>(g, R(b.omega), theta);

        S* db = dst + b.mem;
        const unsigned out = unsigned(b.blk * Q * 64 + lane);
        unroll<Q>([&](auto M) {
            constexpr int m = decltype(M)::value;
            constexpr int i = mem_pop<L>(m);
            ST::put_nt(at32(db, out + unsigned(m * 64)), g[i]);
        });
    }
}

template <class L, class S>
hipError_t launch_step_batch_l(int K, int kind, const void* src, void* dst, const TileDesc* tiles, int ntiles,
                               double theta, int block, int grid, bool aligned_rows, hipStream_t s)
{
    return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        constexpr int KD = decltype(Kind)::value;
        const int waves = block / 64;
        const int need = (ntiles + waves - 1) / waves;  // blocks that give every tile its own wave
        const int g = (grid > 0 && grid < need) ? grid : need;
        if (aligned_rows)
            k_step_batch<L, S, KK, KD, true><<<g, block, 0, s>>>(static_cast<const S*>(src), static_cast<S*>(dst),
                                                                 tiles, ntiles, R(theta));
        else
            k_step_batch<L, S, KK, KD, false><<<g, block, 0, s>>>(static_cast<const S*>(src), static_cast<S*>(dst),
                                                                  tiles, ntiles, R(theta));
        return hipGetLastError();
    });
}

}  // namespace lbm
