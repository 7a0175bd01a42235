// Library-internal declarations shared by the C-ABI implementation and the
// kernel launchers.
//
// Population layout ("row-tiled structure of arrays").  Box b starts at site
// offset O_b of the concatenated site space and holds nx * ny * nz sites.
// Its populations occupy elements [Q O_b, Q (O_b + n_b)) of a buffer; inside
// the box, x-row r = z * ny + y is one tile of Q * nx elements in which
// population i of site x sits at r Q nx + m(i) nx + x, with the tile rows
// m ordered by (c_z, c_y, c_x) (lattice.hpp, mem_row).  A row tile is thus a
// small structure of arrays: every population row is contiguous in x, a step
// writes each tile as one contiguous run of Q * nx elements, and the
// populations it pulls from one neighbouring tile are adjacent rows.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace lbm {

// Single box, one site per thread: grid (xblocks, ny, nz).
struct StepGeom {
    int nx, ny, nz;
    int xblocks;          // blocks per x-row
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

// A tile of the batched step, one wavefront's work: in box `box`, plane z,
// the x-rows y0 .. y0 + rows - 1 (rows * nx <= 64), or, when nx exceeds 64,
// the 64 sites of row y0 from x0 on.  The tile carries its box's geometry, first
// site and relaxation factor, so a block starts after one 64-byte scalar load.
struct alignas(64) TileDesc {
    int z, y0, rows, x0;
    int nx, ny, nz;
    float inv_nx;         // 1 / nx, for the lane -> (row, x) split of a tile
    long long offset;     // the box's first global site
    double omega;         // 1 - 1/tau of the box
    int box;
};
static_assert(sizeof(TileDesc) == 64, "tile descriptor is one scalar load");

struct BoxDesc {
    int nx, ny, nz;
    long long offset;     // O_b: global index of the box's first site
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
hipError_t launch_init(int lat, int dtype, int K, const double* rho, const double* u, void* dst,
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
// Swapped layout -> natural layout into another buffer (bit-exact permutation).
hipError_t launch_unswap(int lat, int dtype, const void* src, void* dst, const StepGeom& geo, int block,
                         hipStream_t s);
// Sites per lane of the row-wave kernel for (lattice, dtype), 0 if that pair
// has no row-wave form (a velocity component as large as V).
int vec_sites_per_lane(int lat, int dtype);
hipError_t launch_step_vec(int lat, int dtype, int K, int kind, const void* src, void* dst, const VecGeom& geo,
                           double omega, double theta, hipStream_t s);
// staged: whole-row tiles written through LDS as one contiguous run.
hipError_t launch_step_batch(int lat, int dtype, int K, int kind, const void* src, void* dst, const TileDesc* tiles,
                             int ntiles, double theta, int block, int grid, bool staged, hipStream_t s);
// Readers of the stored state.  swapped: the state is in the swapped layout
// the in-place step leaves after an odd number of steps (single box).
hipError_t launch_moments(int lat, int dtype, const void* src, bool swapped, double* rho, double* u,
                          const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites, hipStream_t s);
hipError_t launch_totals(int lat, int dtype, const void* src, bool swapped, const ChunkDesc* chunks, int nchunks,
                         const int* box_chunk_begin, int nbox, const BoxDesc* boxes, double* partial, double* out,
                         hipStream_t s);
hipError_t launch_residual(int lat, int dtype, const void* src, bool swapped, const double* rho_ref,
                           const double* u_ref, const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes,
                           long long nsites, double* partial, double* out, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Host copy of a lattice's tables (from the compile-time descriptors).
struct LatticeInfo {
    int D, Q, two_n, k_default, k_max, R;
    double T0;
    std::vector<int> c;     // Q * 3
    std::vector<double> w;  // Q
    std::vector<int> mrow;  // Q: tile row m(i) of population i
};
bool lattice_info(int lat, LatticeInfo* out);

size_t storage_bytes(int dtype);

}  // namespace lbm
