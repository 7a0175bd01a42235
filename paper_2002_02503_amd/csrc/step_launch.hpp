// Launchers of the fused step kernels for one (lattice, storage type).  Each
// pair's instances are compiled in translation units of their own, which the
// build writes (two lines each: include step.hpp or step_batch.hpp, then
// LBM_DECLARE_*_INSTANCES for the pair); the runtime-lattice entry points in
// internal.hpp forward to these.
#pragma once

#include "internal.hpp"
#include "lattice.hpp"

namespace lbm {

struct bf16_t;

// Single box, one site per thread: grid (xblocks, ny, nz) of `block` threads;
// pair: two sites per thread in rows 2j and 2j + 1 (ny even), grid
// (xblocks, ny / 2, nz).
template <class L, class S>
hipError_t launch_step_l(int K, int kind, const void* src, void* dst, const StepGeom& geo, double omega,
                         double theta, int block, bool pair, hipStream_t s);

// Single box, in place: from the natural layout to the swapped one
// (from_natural) or back (see k_step_ip).
template <class L, class S>
hipError_t launch_step_ip_l(int K, int kind, void* buf, bool from_natural, const StepGeom& geo, double omega,
                            double theta, int block, hipStream_t s);

// Single box, in place on the twisted layouts: from an even time (even) or
// an odd one (see k_step_tw).
template <class L, class S>
hipError_t launch_step_tw_l(int K, int kind, void* buf, bool even, const StepGeom& geo, double omega, double theta,
                            int block, hipStream_t s);

// Single box, two steps per launch (3-D lattices with a one-site ring only).
template <class L, class S>
hipError_t launch_step2_l(int K, int kind, const void* src, void* dst, const Step2Geom& geo, double omega,
                          double theta, int grid, hipStream_t s);

// Sites per lane of the row-wave form (0: none for this pair).
template <class L, class S>
int vec_sites_l();

// Single box, row-wave form.
template <class L, class S>
hipError_t launch_step_vec_l(int K, int kind, const void* src, void* dst, const VecGeom& geo, double omega,
                             double theta, hipStream_t s);

// Batch of boxes in the blocked layout: one wave per tile; a fixed grid
// walks the tile table.
template <class L, class S>
hipError_t launch_step_batch_l(int K, int kind, const void* src, void* dst, const TileDesc* tiles, int ntiles,
                               double theta, int block, int grid, bool aligned_rows, hipStream_t s);

#define LBM_DECLARE_STEP_INSTANCES(EXT, L, S)                                                                    \
    EXT template hipError_t launch_step_l<L, S>(int, int, const void*, void*, const StepGeom&, double, double,  \
                                                int, bool, hipStream_t);                                       \
    EXT template hipError_t launch_step_ip_l<L, S>(int, int, void*, bool, const StepGeom&, double, double, int, \
                                                   hipStream_t);                                               \
    EXT template hipError_t launch_step_tw_l<L, S>(int, int, void*, bool, const StepGeom&, double, double, int, \
                                                   hipStream_t);                                               \
    EXT template int vec_sites_l<L, S>();                                                                      \
    EXT template hipError_t launch_step_vec_l<L, S>(int, int, const void*, void*, const VecGeom&, double,      \
                                                    double, hipStream_t);

#define LBM_DECLARE_STEP2_INSTANCES(EXT, L, S)                                                                 \
    EXT template hipError_t launch_step2_l<L, S>(int, int, const void*, void*, const Step2Geom&, double, double, \
                                                 int, hipStream_t);

#define LBM_DECLARE_BATCH_INSTANCES(EXT, L, S)                                                                 \
    EXT template hipError_t launch_step_batch_l<L, S>(int, int, const void*, void*, const TileDesc*, int,    \
                                                      double, int, int, bool, hipStream_t);

#define LBM_EXTERN_PAIR(L, S)                  \
    LBM_DECLARE_STEP_INSTANCES(extern, L, S)   \
    LBM_DECLARE_BATCH_INSTANCES(extern, L, S)

#define LBM_EXTERN_LATTICE(L)       \
    LBM_EXTERN_PAIR(L, double)      \
    LBM_EXTERN_PAIR(L, float)       \
    LBM_EXTERN_PAIR(L, _Float16)    \
    LBM_EXTERN_PAIR(L, bf16_t)

#define LBM_EXTERN_STEP2(L)                            \
    LBM_DECLARE_STEP2_INSTANCES(extern, L, double)     \
    LBM_DECLARE_STEP2_INSTANCES(extern, L, float)      \
    LBM_DECLARE_STEP2_INSTANCES(extern, L, _Float16)   \
    LBM_DECLARE_STEP2_INSTANCES(extern, L, bf16_t)

LBM_EXTERN_LATTICE(D2Q9)
LBM_EXTERN_LATTICE(D3Q15)
LBM_EXTERN_LATTICE(D3Q19)
LBM_EXTERN_LATTICE(D3Q39)
LBM_EXTERN_STEP2(D3Q15)
LBM_EXTERN_STEP2(D3Q19)

}  // namespace lbm
