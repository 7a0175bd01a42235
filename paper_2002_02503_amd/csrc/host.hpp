// Host-only parts of the library, free of any HIP call or type: lattice
// tables, argument checks, the checkpoint header, rearrangement of a state
// between its layouts, and the tune cache.  Used by the C-ABI implementation
// (api.hip); plain C++, so it also builds with the host compiler alone (the
// sanitizer test builds it with AddressSanitizer and UBSan on the CPU).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace lbm {

// Where a single box's populations are, as the step kernels leave them.
//   kNatural:   population i of site x in its own row tile, tile row m(i)
//               (every batch, and the two-buffer single-box steps);
//   kSwapped:   at site x + c_i, tile row m(opp(i)) (k_step_ip after an odd
//               number of its steps);
//   kTwistEven: at site x + b_i, b_i the positive part of c_i, tile row m(i)
//               (k_step_tw after an even number of its steps);
//   kTwistOdd:  at site x + b_i, tile row m(opp(i)) (k_step_tw, odd).
enum StateLayout : int { kNatural = 0, kSwapped = 1, kTwistEven = 2, kTwistOdd = 3 };

// Host copy of a lattice's tables (from the compile-time descriptors).
struct LatticeInfo {
    int D, Q, two_n, k_default, k_max, R;
    double T0;
    std::vector<int> c;     // Q * 3
    std::vector<double> w;  // Q
    std::vector<int> mrow;  // Q: tile row m(i) of population i
};
bool lattice_info(int lat, LatticeInfo* out);

// Bytes per stored population of a dtype code (8, 4, 2, 2), 0 if unknown.
size_t storage_bytes(int dtype);

// Limits of the addressing, checked before anything else happens.
constexpr int64_t kMaxSites = int64_t(1) << 36;  // total sites: keeps chunk and tile counts in int
constexpr int kBlockSites = 64;                  // sites per block of a batched box's layout (one wave)

// Output tile of the two-step kernel (step2.hpp): kTwoStepTileX x
// two_step_tile_y(elem) sites of a z-plane per block, which also computes the
// one-site ring around them in its first step.  8-byte storage takes half the
// rows, so that the kernel's two LDS planes (2 Q (TX + 2)(TY + 2) values)
// stay within a compute unit's 160 KiB.  (Measured on D3Q19 256^3: 64 x 8
// tiles ran 8.5% faster than 32 x 16 in FP32, and 64 x 4 9% faster than 32 x 8
// in FP64: the ring costs more arithmetic, but each population row's ring
// cache lines are shared by twice as many sites.)
constexpr int kTwoStepTileX = 64;
constexpr int two_step_tile_y(size_t elem) { return elem == 8 ? 4 : 8; }

// Whether the two-step kernel applies to a single nx x ny x nz box: a 3-D
// lattice whose velocity components are at most 1 in magnitude (a one-site
// ring), nx and ny multiples of the tile, and one z-plane of populations
// (Q nx ny values) below 2 GiB, since offsets inside a plane are formed in
// 32 bits.
bool two_step_fits(const LatticeInfo& L, int dtype, int64_t nx, int64_t ny, int64_t nz);

// The argument checks of lbm_create / lbm_create_batch for nbox boxes
// (dims: nbox * 3, tau: nbox).  True when every box is valid; otherwise false
// with the reason in *why.
bool check_boxes(const LatticeInfo& L, int dtype, int nbox, const int64_t* dims, const double* tau, std::string* why);

// FNV-1a hash of the box dimensions (checkpoint header, tune-cache key).
uint64_t geometry_hash(const std::vector<int64_t>& dims);

// The 64-byte header in front of a checkpoint's raw populations.
constexpr uint64_t kCkptMagic = 0x314b4350434d424cULL;  // "LBMCPCK1"
struct CkptHeader {
    uint64_t magic;
    int32_t lattice, dtype, K, nbox;
    int64_t nsites, t;
    uint64_t geometry_hash;
    uint64_t payload_bytes;
    uint64_t reserved;  // keeps the header 64 bytes, so the payload is 64-byte aligned
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header layout");

// Check a checkpoint of `bytes` bytes at `buf` against the header a handle
// would write (`expect`, t ignored).  True when it matches; otherwise false
// with the reason in *why.  Reads at most sizeof(CkptHeader) bytes of buf.
bool check_checkpoint(const void* buf, size_t bytes, const CkptHeader& expect, std::string* why);

// Rearrange a single box's state (row tiles, nx * ny * nz sites, elem bytes
// per value) between `layout` and the natural layout: to_natural reads src in
// `layout` and writes dst natural; otherwise the reverse.  src and dst hold
// Q * nx * ny * nz values each and do not overlap.
void relayout_host(const LatticeInfo& L, int64_t nx, int64_t ny, int64_t nz, size_t elem, int layout,
                   bool to_natural, const char* src, char* dst);

// Tune cache: a text file of lines "<key> | <kernel> <block> <grid>".
struct LaunchChoice {
    int kernel, block, grid;
};
// The last entry for `key` in the file at `path` (NULL or "" : none).
bool tune_cache_lookup(const char* path, const std::string& key, LaunchChoice* out);
void tune_cache_store(const char* path, const std::string& key, const LaunchChoice& c);

}  // namespace lbm
