// Library-internal declarations shared by the C-ABI implementation and the
// kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

namespace lbm {

// Geometry of a single box for the row-blocked step kernel.
struct StepGeom {
    int nx, ny, nz;
    int xblocks;          // blocks per x row
    long long plane;      // elements per population plane
};

// A tile of the batched step: `count` consecutive sites of one box, starting
// at local site index `start` (count <= threads per block).
struct TileDesc {
    int box;
    int start;
};

struct BoxDesc {
    int nx, ny, nz, pad;
    long long offset;     // global index of the box's first site
    double omega;         // 1 - 1/tau
};

// A reduction chunk: `count` consecutive global sites belonging to one box.
struct ChunkDesc {
    long long start;
    int count;
    int box;
};

// Kernel launchers (kernels.hip).  All return hipSuccess or the first error.
hipError_t launch_init(int lat, int dtype, int K, const double* rho, const double* u, void* dst,
                       long long nsites, long long plane, hipStream_t s);
hipError_t launch_step(int lat, int dtype, int K, const void* src, void* dst, const StepGeom& geo,
                       double omega, int block, hipStream_t s);
hipError_t launch_step_batch(int lat, int dtype, int K, const void* src, void* dst, const TileDesc* tiles,
                             int ntiles, const BoxDesc* boxes, long long plane, int block, int grid,
                             hipStream_t s);
hipError_t launch_moments(int lat, int dtype, const void* src, double* rho, double* u, long long nsites,
                          long long plane, hipStream_t s);
hipError_t launch_totals(int lat, int dtype, const void* src, const ChunkDesc* chunks, int nchunks,
                         const int* box_chunk_begin, int nbox, long long plane, double* partial,
                         double* out, hipStream_t s);
hipError_t launch_residual(int lat, int dtype, const void* src, const double* rho_ref, const double* u_ref,
                           const ChunkDesc* chunks, int nchunks, long long nsites, long long plane,
                           double* partial, double* out, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Host copy of a lattice's tables (from the compile-time descriptors).
struct LatticeInfo {
    int D, Q, two_n, k_default, k_max, R;
    double T0;
    std::vector<int> c;     // Q * 3
    std::vector<double> w;  // Q
};
bool lattice_info(int lat, LatticeInfo* out);

size_t storage_bytes(int dtype);

}  // namespace lbm
