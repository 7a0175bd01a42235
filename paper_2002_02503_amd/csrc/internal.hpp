// Library-internal declarations shared by the C-ABI implementation and the
// kernel launchers (the host-only ones are in host.hpp).
//
// Population layout ("blocked structure of arrays", BoxDesc).  The local
// sites of a box, x fastest, are cut into blocks of w consecutive sites; a
// block holds Q runs of w values, population i in run m(i), with the runs
// ordered by (c_z, c_y, c_x) (lattice.hpp, mem_row).  A single box has w = nx:
// each x-row is one block ("row tile"), every population row is contiguous in
// x, a step writes each tile as one contiguous run of Q * nx elements, and
// the populations it pulls from one neighbouring tile are adjacent rows.  The
// boxes of a batch have w = 64, one wavefront's sites, whatever their row
// length.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "host.hpp"

namespace lbm {

// Single box, one site per thread: grid (xblocks, ny, nz).
struct StepGeom {
    int nx, ny, nz;
    int xblocks;          // blocks per x-row
};

// Single box, two-step kernel (step2.hpp): the (x, y) plane is cut into
// columns of the output tile, ncx of them along x; column-plane
// w = column * nz + z, and block b takes the `per` consecutive column-planes
// from (b or its XCD-ordered index) * per on, `total` of them in all.
struct Step2Geom {
    int nx, ny, nz;
    int ncx;
    long long total;
    long long per;
    int xcd_order;        // 1: consecutive columns on one XCD (grid a multiple of 8)
};

// Single box, row-wave form: each lane owns V consecutive sites of an x-row,
// a row takes lanes_per_row = nx / V lanes and a 64-lane wavefront holds
// rows_per_wave = 64 / lanes_per_row rows.
struct VecGeom {
    int nx, ny, nz;
    int lanes_per_row;
    int rows_per_wave;
    int nrows;            // ny * nz
};

// A tile of the batched step, one wavefront's work: block `blk` of box `box`,
// that is its local sites blk * 64 .. blk * 64 + count - 1 (x fastest, then
// y, then z), the first of which is (x0, y0, z0).  The tile carries its box's
// geometry, population offset and relaxation factor, so a wave starts after
// one 64-byte scalar load.
struct alignas(64) TileDesc {
    int nx, ny, nz;
    int x0, y0, z0;
    int blk, count;
    long long mem;        // element offset of the box's populations
    double omega;         // 1 - 1/tau of the box
    int box;
    float inv_nx, inv_ny; // 1 / nx, 1 / ny, for the lane -> (x, y, z) split
};
static_assert(sizeof(TileDesc) == 64, "tile descriptor is one scalar load");

// Population layout of a box: its local sites l = (z * ny + y) * nx + x are
// cut into blocks of w consecutive sites, and block l / w holds Q runs of w
// values, population i of site l at element
//   mem + (l / w) * Q * w + m(i) * w + l % w      (m: tile row, lattice.hpp).
// A single box has w = nx (a block is an x-row: the row-tiled layout); the
// boxes of a batch have w = 64, each padded to a whole number of blocks.
struct BoxDesc {
    int nx, ny, nz;
    int w;                // sites per block
    long long offset;     // O_b: global index of the box's first site (fields)
    long long mem;        // element offset of the box's populations
    double omega;         // 1 - 1/tau
};

// A run of `count` consecutive global sites of one box (never two boxes),
// the unit of the set-up, moment and reduction kernels.
struct ChunkDesc {
    long long start;
    int count;
    int box;
};

// Kernel launchers (kernels.hip).  All return hipSuccess or the first error.
// layout: kNatural, or kTwistEven for a single box stepped by k_step_tw.
hipError_t launch_init(int lat, int dtype, int K, int layout, const double* rho, const double* u, void* dst,
                       const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites,
                       hipStream_t s);
// The fused step.  kind: collision kind (collide.hpp: 0 filtered, 1 BGK,
// 2 filtered with the energy-flux term of weight theta).
// pair: two sites per thread (rows 2j, 2j + 1; ny even).
hipError_t launch_step(int lat, int dtype, int K, int kind, const void* src, void* dst, const StepGeom& geo,
                       double omega, double theta, int block, bool pair, hipStream_t s);
// The in-place step on one buffer: from the natural layout to the swapped one
// (from_natural) or back (step.hpp, k_step_ip).
hipError_t launch_step_ip(int lat, int dtype, int K, int kind, void* buf, bool from_natural, const StepGeom& geo,
                          double omega, double theta, int block, hipStream_t s);
// The in-place step on the twisted layouts, from an even time (even) or an
// odd one (step.hpp, k_step_tw).
hipError_t launch_step_tw(int lat, int dtype, int K, int kind, void* buf, bool even, const StepGeom& geo,
                          double omega, double theta, int block, hipStream_t s);
// Two steps in one launch (step2.hpp, k_step2), from src to dst, on `grid`
// blocks; D3Q15 and D3Q19 only (two_step_fits), else hipErrorInvalidValue.
hipError_t launch_step2(int lat, int dtype, int K, int kind, const void* src, void* dst, const Step2Geom& geo,
                        double omega, double theta, int grid, hipStream_t s);
// A single box's state from `layout` to the natural layout (to_natural) or
// back, into another buffer (bit-exact permutation).
hipError_t launch_relayout(int lat, int dtype, int layout, bool to_natural, const void* src, void* dst,
                           const StepGeom& geo, int block, hipStream_t s);
// Sites per lane of the row-wave kernel for (lattice, dtype), 0 if that pair
// has no row-wave form (a velocity component as large as V).
int vec_sites_per_lane(int lat, int dtype);
hipError_t launch_step_vec(int lat, int dtype, int K, int kind, const void* src, void* dst, const VecGeom& geo,
                           double omega, double theta, hipStream_t s);
// Batch of boxes in the blocked layout.  aligned_rows: every box has nx a
// multiple of 64, so populations with c_x = 0 are read in whole blocks.
hipError_t launch_step_batch(int lat, int dtype, int K, int kind, const void* src, void* dst, const TileDesc* tiles,
                             int ntiles, double theta, int block, int grid, bool aligned_rows, hipStream_t s);
// Readers of the stored state, in any StateLayout (the in-place layouts for
// a single box only).
hipError_t launch_moments(int lat, int dtype, const void* src, int layout, double* rho, double* u,
                          const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites, hipStream_t s);
hipError_t launch_totals(int lat, int dtype, const void* src, int layout, const ChunkDesc* chunks, int nchunks,
                         const int* box_chunk_begin, int nbox, const BoxDesc* boxes, double* partial, double* out,
                         hipStream_t s);
// Error residuals: partial holds 4 doubles per chunk; out gets {max |du|,
// sum du^2, max |drho|, sum drho^2}, or the square roots of the two sums when
// sqrt_l2.
hipError_t launch_residual(int lat, int dtype, const void* src, int layout, const double* rho_ref,
                           const double* u_ref, const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes,
                           long long nsites, double* partial, double* out, bool sqrt_l2, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace lbm
