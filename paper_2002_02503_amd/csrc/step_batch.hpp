// The fused pull-stream + collide step on a batch of boxes, templated on
// lattice, storage type, Hermite order and collision kind.  Included by the
// per-lattice translation units.
#pragma once

#include <algorithm>

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

// STAGED: a tile of whole rows (nx <= 64) is written through LDS.  Its row
// tiles form one contiguous run of rows * Q * nx elements; each lane puts its
// site's populations into the wave's slice of LDS at their offsets in that
// run, and the wave then stores the run with every lane active, 64
// consecutive elements per instruction.  Rows of a length that does not fill
// whole cache lines are otherwise written as partial lines, population row by
// population row.
template <class L, class S, int K, int KIND, bool STAGED>
__global__ __launch_bounds__(256) void k_step_batch(const S* __restrict__ src, S* __restrict__ dst,
                                                    const TileDesc* __restrict__ tiles, int ntiles,
                                                    typename Store<S>::R theta)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;
    extern __shared__ unsigned char stage_bytes[];

    const int waves = int(blockDim.x) >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);  // uniform: scalar descriptor loads
    const int tid = int(threadIdx.x) & 63;
    S* stage = reinterpret_cast<S*>(stage_bytes) + wave * (L::Q * 64);
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
        const bool active = (r < b.rows) && (x < b.nx);
        const bool staged = STAGED && (b.nx <= 64);  // uniform over the wave
        const int tq = L::Q * b.nx;
        S* db = dst + (long long)L::Q * b.offset;
        if (active) {
            const int y = b.y0 + r;
            const int z = b.z;
            const S* sb = src + (long long)L::Q * b.offset;

            int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
            for (int k = 0; k <= 2 * RR; ++k) {
                xw[k] = wrap_coord(x + k - RR, b.nx);
                yw[k] = wrap_coord(y + k - RR, b.ny);
                zw[k] = wrap_coord(z + k - RR, b.nz);
            }
            // element offset of a row tile = plane part (uniform) + row part (per lane)
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

            if (staged) {
                const int loc = r * tq + x;  // offset in the tile's run
                unroll<L::Q>([&](auto M) {
                    constexpr int m = decltype(M)::value;
                    constexpr int i = mem_pop<L>(m);
                    ST::put(stage + loc + m * b.nx, g[i]);
                });
            } else {
                const int out_off = (z * b.ny + y) * tq + x;
                unroll<L::Q>([&](auto M) {
                    constexpr int m = decltype(M)::value;
                    constexpr int i = mem_pop<L>(m);  // a constant expression: the array index must fold
                    ST::put_nt(at32(db, unsigned(out_off + m * b.nx)), g[i]);
                });
            }
        }
        if constexpr (STAGED) {
            if (staged) {
                // the wave's own LDS slice: order the lanes' writes before the reads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int n = b.rows * tq;
                const int base = (b.z * b.ny + b.y0) * tq;
                // the stored bits, moved as integers of the storage width
                using W = std::conditional_t<sizeof(S) == 8, unsigned long long,
                                             std::conditional_t<sizeof(S) == 4, unsigned, unsigned short>>;
                const W* from = reinterpret_cast<const W*>(stage);
                W* to = reinterpret_cast<W*>(at32(db, unsigned(base)));
                for (int k = tid; k < n; k += 64) __builtin_nontemporal_store(from[k], to + k);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
}

template <class L, class S>
hipError_t launch_step_batch_l(int K, int kind, const void* src, void* dst, const TileDesc* tiles, int ntiles,
                               double theta, int block, int grid, bool staged, hipStream_t s)
{
    return dispatch_pair<L, S>(K, kind, [&](auto, auto*, auto Kc, auto Kind) -> hipError_t {
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        constexpr int KD = decltype(Kind)::value;
        // staged: each wave holds Q * 64 values in LDS; at most 64 KiB per
        // block (fewer waves per block for D3Q39 in FP64)
        constexpr int kStageWave = L::Q * 64 * int(sizeof(S));
        const int waves = staged ? std::min(block / 64, 65536 / kStageWave) : block / 64;
        const int need = (ntiles + waves - 1) / waves;  // blocks that give every tile its own wave
        const int g = (grid > 0 && grid < need) ? grid : need;
        if (staged) {
            k_step_batch<L, S, KK, KD, true><<<g, waves * 64, size_t(waves) * kStageWave, s>>>(
                static_cast<const S*>(src), static_cast<S*>(dst), tiles, ntiles, R(theta));
        } else {
            k_step_batch<L, S, KK, KD, false><<<g, block, 0, s>>>(static_cast<const S*>(src), static_cast<S*>(dst),
                                                                  tiles, ntiles, R(theta));
        }
        return hipGetLastError();
    });
}

}  // namespace lbm
