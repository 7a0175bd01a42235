// C-ABI implementation of liblbm.so (declared in include/lbm.h).
//
// Host-side responsibilities: argument validation before any device work,
// ownership of device allocations, the two-buffer (read A / write B) step
// sequence, capture of step sequences into HIP graphs, reduction tables,
// checkpoint format and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <utility>
#include <string>
#include <vector>

#include "internal.hpp"
#include "lattice.hpp"
#include "lbm.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

lbm_status fail_hip(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory) return fail(LBM_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                              \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return fail_hip(e_, what); \
    } while (0)

constexpr int kChunkSites = 4096;   // sites per reduction chunk
constexpr int kDefaultGraphChunk = 32;
constexpr int kTuneRounds = 3;

// Scratch of the allocation-free residual (lbm_residual_noalloc): the
// per-chunk partial sums of the residual kernels, 4 doubles per reduction
// chunk.  Every GPU the library runs on holds its own copy of this array for
// the life of the process.  In host code `scratch` is only a stand-in for the
// symbol: its device address on the current GPU comes from
// hipGetSymbolAddress (scratch_address), and only that address is handed to
// kernels.
constexpr size_t kScratchBytes = size_t(2) << 20;
constexpr int kScratchChunks = int(kScratchBytes / (4 * sizeof(double)));
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

struct lbm_ctx {
    int lattice = 0, dtype = 0, K = 0;
    int collision = LBM_COLLISION_FILTERED;
    double theta = 0.0;             // weight of the energy-flux term
    LatticeInfo lat;
    int nbox = 0;
    std::vector<int64_t> dims;      // nbox * 3
    std::vector<double> tau;        // nbox
    std::vector<int64_t> offset;    // nbox: first global site (field index)
    std::vector<int64_t> mem;       // nbox: element offset of the populations
    int64_t nsites = 0;
    int64_t nstored = 0;            // stored sites, with the blocked layout's padding
    bool aligned_rows = false;      // batch: every box has nx % 64 == 0
    size_t elem = 0;                // bytes per stored population
    size_t state_bytes = 0;
    void* buf[2] = {nullptr, nullptr};
    bool owns_buf = false;
    bool bound = false;
    int cur = 0;
    int64_t t = 0;
    bool initialized = false;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int device = 0;
    int cus = 1;                    // compute units of the device
    int block = 0;                  // 0 = automatic
    int grid = 0;                   // batched: 0 = one block per tile
    int kernel = LBM_KERNEL_AUTO;   // single box: scalar or row-wave step
    int graph_chunk = kDefaultGraphChunk;
    // batched step tables
    TileDesc* d_tiles = nullptr;
    int ntiles = 0;
    BoxDesc* d_boxes = nullptr;
    // reductions
    ChunkDesc* d_chunks = nullptr;
    int nchunks = 0;
    int* d_box_chunk_begin = nullptr;
    double* d_partial = nullptr;
    double* d_out = nullptr;
    // captured step graphs, one per starting buffer
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gexec_steps[2] = {0, 0};
};

namespace {

bool is_single(const lbm_ctx* h) { return h->nbox == 1; }

// Sites per lane when the row-wave step applies to this box (0 otherwise):
// whole x-rows of nx = lanes_per_row * V sites with at most 64 lanes per row.
int row_wave_sites(const lbm_ctx* h)
{
    if (!is_single(h)) return 0;
    const int V = vec_sites_per_lane(h->lattice, h->dtype);
    const int64_t nx = h->dims[0];
    if (V == 0 || nx % V != 0 || nx / V > 64) return 0;
    return V;
}

// Collision kind of the step kernels (lattice.hpp, CollisionKind).
int step_kind(const lbm_ctx* h)
{
    if (h->collision == LBM_COLLISION_BGK) return kBGK;
    return h->theta != 0.0 ? kFilteredQ : kFiltered;
}

int effective_kernel(const lbm_ctx* h)
{
    if (!is_single(h)) return LBM_KERNEL_SCALAR;
    if (h->kernel == LBM_KERNEL_AUTO) return LBM_KERNEL_SCALAR;  // measured faster unless tuned otherwise
    return h->kernel;
}

int effective_block(const lbm_ctx* h)
{
    if (h->block > 0) return h->block;
    if (!is_single(h)) return 256;
    const int64_t nx = h->dims[0];
    int64_t b = ((nx + 63) / 64) * 64;
    if (b > 256) b = 256;
    return int(b);
}

uint64_t geometry_hash(const lbm_ctx* h) { return lbm::geometry_hash(h->dims); }

lbm_status check_handle(lbm_t h)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    return LBM_OK;
}

void drop_graphs(lbm_ctx* h)
{
    for (int p = 0; p < 2; ++p) {
        if (h->gexec[p]) (void)hipGraphExecDestroy(h->gexec[p]);
        h->gexec[p] = nullptr;
        h->gexec_steps[p] = 0;
    }
}

void free_all(lbm_ctx* h)
{
    drop_graphs(h);
    if (h->owns_buf) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
    }
    h->buf[0] = h->buf[1] = nullptr;
    (void)hipFree(h->d_tiles);
    (void)hipFree(h->d_boxes);
    (void)hipFree(h->d_chunks);
    (void)hipFree(h->d_box_chunk_begin);
    (void)hipFree(h->d_partial);
    (void)hipFree(h->d_out);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    h->cap_stream = nullptr;
}

lbm_status device_check(int* dev)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1) return fail(LBM_ENODEV, "no usable GPU (%s)", hipGetErrorString(e));
    HIP_TRY(hipGetDevice(dev), "hipGetDevice");
    return LBM_OK;
}

// Device address of `scratch` on GPU `dev`, which must be the current device.
// Resolved once per device (at lbm_create) and kept; later calls only read
// the table.
lbm_status scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

// Wave tiles of the batched step (step_batch.hpp): one per 64-site block of
// each box.  The table does not depend on the block size.
lbm_status build_tiles(lbm_ctx* h)
{
    if (is_single(h)) return LBM_OK;
    if (h->d_tiles) return LBM_OK;
    std::vector<TileDesc> tiles;
    for (int b = 0; b < h->nbox; ++b) {
        const int64_t nx = h->dims[3 * b], ny = h->dims[3 * b + 1], nz = h->dims[3 * b + 2];
        const int64_t n = nx * ny * nz;
        TileDesc t{};
        t.nx = int(nx);
        t.ny = int(ny);
        t.nz = int(nz);
        t.mem = h->mem[b];
        t.omega = 1.0 - 1.0 / h->tau[b];
        t.box = b;
        t.inv_nx = float(1.0 / double(nx));
        t.inv_ny = float(1.0 / double(ny));
        for (int64_t l0 = 0; l0 < n; l0 += kBlockSites) {
            t.x0 = int(l0 % nx);
            t.y0 = int((l0 / nx) % ny);
            t.z0 = int(l0 / (nx * ny));
            t.blk = int(l0 / kBlockSites);
            t.count = int(std::min<int64_t>(kBlockSites, n - l0));
            tiles.push_back(t);
        }
    }
    HIP_TRY(hipMalloc(&h->d_tiles, tiles.size() * sizeof(TileDesc)), "hipMalloc(tiles)");
    HIP_TRY(hipMemcpy(h->d_tiles, tiles.data(), tiles.size() * sizeof(TileDesc), hipMemcpyHostToDevice),
            "copy tiles");
    h->ntiles = int(tiles.size());
    drop_graphs(h);
    return LBM_OK;
}

lbm_status create_common(lbm_t* out, int32_t lattice, int32_t nbox, const int64_t* dims, const double* tau,
                         int32_t dtype)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    LatticeInfo L;
    if (!lattice_info(lattice, &L)) return fail(LBM_EINVAL, "unknown lattice %d", lattice);
    if (storage_bytes(dtype) == 0) return fail(LBM_EINVAL, "unknown dtype %d", dtype);
    if (nbox < 1) return fail(LBM_EINVAL, "nbox must be >= 1");
    if (!dims || !tau) return fail(LBM_EINVAL, "dims or tau is NULL");
    // every argument is checked here, on the host, before any device call
    std::string why;
    if (!check_boxes(L, dtype, nbox, dims, tau, &why)) return fail(LBM_EINVAL, "%s", why.c_str());
    int dev = 0;
    lbm_status st = device_check(&dev);
    if (st != LBM_OK) return st;
    double* scratch_ptr = nullptr;
    if ((st = scratch_address(dev, &scratch_ptr)) != LBM_OK) return st;

    lbm_ctx* h = new lbm_ctx();
    // an exception (host allocation) past this point frees the handle
    // before the entry point's guard turns it into an error code
    try {
        h->lattice = lattice;
        h->dtype = dtype;
        h->lat = L;
        h->K = L.k_default;
        h->nbox = nbox;
        h->dims.assign(dims, dims + 3 * nbox);
        h->tau.assign(tau, tau + nbox);
        h->offset.resize(nbox);
        h->mem.resize(nbox);
        h->device = dev;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            h->cus = cus;
        // A single box is stored in row tiles (blocks of w = nx sites); the boxes
        // of a batch in blocks of 64 sites, each box padded to whole blocks.
        int64_t off = 0, stored = 0;
        bool aligned = true;
        for (int b = 0; b < nbox; ++b) {
            const int64_t n = dims[3 * b] * dims[3 * b + 1] * dims[3 * b + 2];
            h->offset[b] = off;
            h->mem[b] = stored * L.Q;
            off += n;
            stored += (nbox == 1) ? n : (n + kBlockSites - 1) / kBlockSites * kBlockSites;
            aligned = aligned && dims[3 * b] % kBlockSites == 0;
        }
        h->nsites = off;
        h->nstored = stored;
        h->aligned_rows = aligned;
        h->elem = storage_bytes(dtype);
        // Q * nstored elements, allocation rounded to 256 bytes
        h->state_bytes = ((size_t(h->nstored) * size_t(L.Q) * h->elem + 255) / 256) * 256;

        auto cleanup = [&](lbm_status s) {
            free_all(h);
            delete h;
            return s;
        };
        hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return cleanup(fail_hip(e, "hipStreamCreate"));

        // reduction chunks (never straddle two boxes)
        std::vector<ChunkDesc> chunks;
        std::vector<int> begin;
        for (int b = 0; b < nbox; ++b) {
            begin.push_back(int(chunks.size()));
            const int64_t n = dims[3 * b] * dims[3 * b + 1] * dims[3 * b + 2];
            for (int64_t s = 0; s < n; s += kChunkSites) {
                const int64_t cnt = (n - s < kChunkSites) ? (n - s) : kChunkSites;
                chunks.push_back({h->offset[b] + s, int(cnt), b});
            }
        }
        begin.push_back(int(chunks.size()));
        h->nchunks = int(chunks.size());
        if ((e = hipMalloc(&h->d_chunks, chunks.size() * sizeof(ChunkDesc))) != hipSuccess ||
            (e = hipMalloc(&h->d_box_chunk_begin, begin.size() * sizeof(int))) != hipSuccess ||
            (e = hipMalloc(&h->d_partial, chunks.size() * 4 * sizeof(double))) != hipSuccess ||
            (e = hipMalloc(&h->d_out, size_t(nbox) * 4 * sizeof(double))) != hipSuccess)
            return cleanup(fail_hip(e, "hipMalloc(reduction tables)"));
        if ((e = hipMemcpy(h->d_chunks, chunks.data(), chunks.size() * sizeof(ChunkDesc), hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(h->d_box_chunk_begin, begin.data(), begin.size() * sizeof(int), hipMemcpyHostToDevice)) !=
                hipSuccess)
            return cleanup(fail_hip(e, "copy reduction tables"));

        {
            std::vector<BoxDesc> boxes(nbox);
            for (int b = 0; b < nbox; ++b) {
                boxes[b].nx = int(dims[3 * b]);
                boxes[b].ny = int(dims[3 * b + 1]);
                boxes[b].nz = int(dims[3 * b + 2]);
                boxes[b].w = (nbox == 1) ? boxes[b].nx : kBlockSites;
                boxes[b].offset = h->offset[b];
                boxes[b].mem = h->mem[b];
                boxes[b].omega = 1.0 - 1.0 / tau[b];
            }
            if ((e = hipMalloc(&h->d_boxes, boxes.size() * sizeof(BoxDesc))) != hipSuccess)
                return cleanup(fail_hip(e, "hipMalloc(boxes)"));
            if ((e = hipMemcpy(h->d_boxes, boxes.data(), boxes.size() * sizeof(BoxDesc), hipMemcpyHostToDevice)) !=
                hipSuccess)
                return cleanup(fail_hip(e, "copy boxes"));
        }
        *out = h;
        return LBM_OK;
    } catch (...) {
        free_all(h);
        delete h;
        throw;
    }
}

lbm_status alloc_buffer(lbm_ctx* h, int k)
{
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, h->state_bytes);
    if (e != hipSuccess) return fail_hip(e, "hipMalloc(population buffer)");
    h->buf[k] = p;
    h->owns_buf = true;
    return LBM_OK;
}

// The population buffers, unless the caller bound its own.  The in-place step
// needs only buf[0]; buf[1] then comes later, if ever (ensure_second).
lbm_status ensure_buffers(lbm_ctx* h)
{
    if (!h->buf[0])
        if (lbm_status st = alloc_buffer(h, 0)) return st;
    const bool one = is_single(h) && (h->kernel == LBM_KERNEL_IN_PLACE || h->kernel == LBM_KERNEL_TWIST);
    if (!h->buf[1] && !one)
        if (lbm_status st = alloc_buffer(h, 1)) return st;
    return LBM_OK;
}

lbm_status ensure_second(lbm_ctx* h)
{
    if (h->buf[1]) return LBM_OK;
    return alloc_buffer(h, 1);
}

bool in_place(const lbm_ctx* h) { return is_single(h) && effective_kernel(h) == LBM_KERNEL_IN_PLACE; }
bool twisted(const lbm_ctx* h) { return is_single(h) && effective_kernel(h) == LBM_KERNEL_TWIST; }
// The step works inside one buffer (either in-place form).
bool one_buffer(const lbm_ctx* h) { return in_place(h) || twisted(h); }

// The two-step kernel applies to this box (host.hpp, two_step_fits) / is the
// one in use.
bool two_step_ok(const lbm_ctx* h)
{
    return is_single(h) && two_step_fits(h->lat, h->dtype, h->dims[0], h->dims[1], h->dims[2]);
}
bool two_step(const lbm_ctx* h) { return is_single(h) && effective_kernel(h) == LBM_KERNEL_TWO_STEP; }

// Blocks of the two-step kernel: the chosen grid, else one per compute unit
// (its LDS planes leave room for one block per CU; measured fastest).
int two_step_grid(const lbm_ctx* h) { return h->grid > 0 ? h->grid : h->cus; }

// Layout of the current state (StateLayout): the in-place forms alternate
// two layouts, h->cur being the parity of the steps they took.
int state_layout(const lbm_ctx* h)
{
    if (in_place(h)) return h->cur == 1 ? kSwapped : kNatural;
    if (twisted(h)) return h->cur == 1 ? kTwistOdd : kTwistEven;
    return kNatural;
}

// The padding sites of a batch's blocked layout are never read or written by
// the step; zero them in both buffers (before lbm_init or lbm_set_state writes
// the state), so that checkpoints are deterministic.  Not part of any
// captured graph.
lbm_status clear_padding(lbm_ctx* h)
{
    if (h->nstored == h->nsites) return LBM_OK;
    for (int k = 0; k < 2; ++k)
        if (h->buf[k]) HIP_TRY(hipMemsetAsync(h->buf[k], 0, h->state_bytes, h->stream), "clear the state buffers");
    return LBM_OK;
}

StepGeom single_geom(const lbm_ctx* h, int block)
{
    StepGeom geo;
    geo.nx = int(h->dims[0]);
    geo.ny = int(h->dims[1]);
    geo.nz = int(h->dims[2]);
    geo.xblocks = (geo.nx + block - 1) / block;
    return geo;
}

// One step on stream s.  Two-buffer kernels step from buf[parity] into
// buf[parity ^ 1].  The in-place kernel steps buf[0] from the natural layout
// (parity 0) to the swapped one, or back (parity 1); the twist kernel steps
// buf[0] from the twisted layout of an even time (parity 0) or an odd one.
// Either way the next step has parity ^ 1, which h->cur tracks.
hipError_t launch_one(lbm_ctx* h, int parity, hipStream_t s)
{
    const int block = effective_block(h);
    if (in_place(h))
        return launch_step_ip(h->lattice, h->dtype, h->K, step_kind(h), h->buf[0], parity == 0, single_geom(h, block),
                              1.0 - 1.0 / h->tau[0], h->theta, block, s);
    if (twisted(h))
        return launch_step_tw(h->lattice, h->dtype, h->K, step_kind(h), h->buf[0], parity == 0, single_geom(h, block),
                              1.0 - 1.0 / h->tau[0], h->theta, block, s);
    const void* src = h->buf[parity];
    void* dst = h->buf[parity ^ 1];
    if (is_single(h) && effective_kernel(h) == LBM_KERNEL_ROW_WAVE) {
        VecGeom geo;
        const int V = row_wave_sites(h);
        geo.nx = int(h->dims[0]);
        geo.ny = int(h->dims[1]);
        geo.nz = int(h->dims[2]);
        geo.lanes_per_row = geo.nx / V;
        geo.rows_per_wave = 64 / geo.lanes_per_row;
        geo.nrows = geo.ny * geo.nz;
        return launch_step_vec(h->lattice, h->dtype, h->K, step_kind(h), src, dst, geo, 1.0 - 1.0 / h->tau[0],
                               h->theta, s);
    }
    if (is_single(h))
        return launch_step(h->lattice, h->dtype, h->K, step_kind(h), src, dst, single_geom(h, block),
                           1.0 - 1.0 / h->tau[0], h->theta, block, effective_kernel(h) == LBM_KERNEL_TWO_ROW, s);
    return launch_step_batch(h->lattice, h->dtype, h->K, step_kind(h), src, dst, h->d_tiles, h->ntiles, h->theta,
                             block, h->grid, h->aligned_rows, s);
}

// Two steps in one launch (step2.hpp), from buf[parity] into buf[parity ^ 1]:
// like launch_one for the buffers, two steps for the time.
hipError_t launch_two(lbm_ctx* h, int parity, hipStream_t s)
{
    Step2Geom geo;
    geo.nx = int(h->dims[0]);
    geo.ny = int(h->dims[1]);
    geo.nz = int(h->dims[2]);
    geo.ncx = int(h->dims[0] / kTwoStepTileX);
    const long long ncy = h->dims[1] / two_step_tile_y(h->elem);
    geo.total = (long long)geo.ncx * ncy * geo.nz;
    const int grid = two_step_grid(h);
    geo.per = (geo.total + grid - 1) / grid;
    geo.xcd_order = (grid % 8 == 0) ? 1 : 0;
    return launch_step2(h->lattice, h->dtype, h->K, step_kind(h), h->buf[parity], h->buf[parity ^ 1], geo,
                        1.0 - 1.0 / h->tau[0], h->theta, grid, s);
}

// Steps the next launch takes when `left` remain: two for the two-step kernel
// (an odd last step goes to the one-site step), else one.
int steps_in_launch(const lbm_ctx* h, int64_t left) { return (two_step(h) && left >= 2) ? 2 : 1; }

hipError_t launch_steps(lbm_ctx* h, int parity, int k, hipStream_t s)
{
    return k == 2 ? launch_two(h, parity, s) : launch_one(h, parity, s);
}

// Launches that take n steps; each flips the buffer parity.
int64_t launches_for(const lbm_ctx* h, int64_t n) { return two_step(h) ? n / 2 + n % 2 : n; }

// Where the current state is, and in which layout (StateLayout).
void state_view(const lbm_ctx* h, const void** state, int* layout)
{
    *layout = state_layout(h);
    *state = one_buffer(h) ? h->buf[0] : h->buf[h->cur];
}

// Bring the state into buf[0] in the natural layout (cur = 0), before the
// kernel choice changes on an initialised handle: rearrange an in-place
// layout into the other buffer, or take the two-buffer state from buf[1],
// then swap the two buffer pointers.  Every kernel but the twist step can
// start from there (enter_kernel_layout prepares that one).
lbm_status canonicalize(lbm_ctx* h)
{
    if (!h->initialized) return LBM_OK;
    const int layout = state_layout(h);
    if (layout == kNatural && (one_buffer(h) || h->cur == 0)) return LBM_OK;
    if (layout != kNatural) {
        if (lbm_status st = ensure_second(h)) return st;
        const int block = effective_block(h);
        hipError_t e = launch_relayout(h->lattice, h->dtype, layout, true, h->buf[0], h->buf[1],
                                       single_geom(h, block), block, h->stream);
        if (e != hipSuccess) return fail_hip(e, "relayout kernel");
    }
    std::swap(h->buf[0], h->buf[1]);
    h->cur = 0;
    // the natural state at cur = 0 is the scalar step's starting point, not
    // the twist step's; callers choose the next kernel right after
    if (twisted(h)) h->kernel = LBM_KERNEL_SCALAR;
    drop_graphs(h);
    return LBM_OK;
}

// After a kernel change on an initialised handle (state natural in buf[0],
// cur = 0): put the state into the layout the new kernel starts from.  Only
// the twist kernel needs it (its even-time layout).
lbm_status enter_kernel_layout(lbm_ctx* h)
{
    if (!h->initialized || !twisted(h)) return LBM_OK;
    if (lbm_status st = ensure_second(h)) return st;
    const int block = effective_block(h);
    hipError_t e = launch_relayout(h->lattice, h->dtype, kTwistEven, false, h->buf[0], h->buf[1],
                                   single_geom(h, block), block, h->stream);
    if (e != hipSuccess) return fail_hip(e, "relayout kernel");
    std::swap(h->buf[0], h->buf[1]);
    h->cur = 0;
    drop_graphs(h);
    return LBM_OK;
}

// Host copy of a single box's state between an in-place layout and the
// natural one (host.hpp, relayout_host).
void relayout_host(const lbm_ctx* h, int layout, bool to_natural, const char* src, char* dst)
{
    lbm::relayout_host(h->lat, h->dims[0], h->dims[1], h->dims[2], h->elem, layout, to_natural, src, dst);
}

lbm_status build_graph(lbm_ctx* h, int parity)
{
    const int n = h->graph_chunk;
    if (h->gexec[parity] && h->gexec_steps[parity] == n) return LBM_OK;
    if (h->gexec[parity]) {
        (void)hipGraphExecDestroy(h->gexec[parity]);
        h->gexec[parity] = nullptr;
    }
    lbm_status st = build_tiles(h);
    if (st != LBM_OK) return st;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    int p = parity;
    for (int left = n; left > 0 && le == hipSuccess; p ^= 1) {
        const int k = steps_in_launch(h, left);
        le = launch_steps(h, p, k, h->cap_stream);
        left -= k;
    }
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(h->cap_stream, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail_hip(le, "kernel launch during graph capture");
    }
    if (ee != hipSuccess) return fail_hip(ee, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail_hip(ie, "hipGraphInstantiate");
    h->gexec[parity] = exec;
    h->gexec_steps[parity] = n;
    return LBM_OK;
}

lbm_status stage_in(const double* src, size_t count, int on_device, hipStream_t s, double** out, bool* temp)
{
    if (on_device) {
        *out = const_cast<double*>(src);
        *temp = false;
        return LBM_OK;
    }
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, count * sizeof(double)), "hipMalloc(staging)");
    hipError_t e = hipMemcpyAsync(d, src, count * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail_hip(e, "copy to device");
    }
    *out = d;
    *temp = true;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_create(lbm_t* out, int32_t lattice, const int64_t dims[3], double tau, int32_t dtype)
{
    try {
        return create_common(out, lattice, 1, dims, &tau, dtype);
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_create: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_create: unexpected host exception");
    }
}

lbm_status lbm_create_batch(lbm_t* out, int32_t lattice, int32_t nbox, const int64_t* dims, const double* tau,
                            int32_t dtype)
{
    try {
        return create_common(out, lattice, nbox, dims, tau, dtype);
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_create_batch: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_create_batch: unexpected host exception");
    }
}

lbm_status lbm_set_hermite_order(lbm_t h, int32_t K)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (K < 2 || K > h->lat.k_max)
            return fail(LBM_EINVAL, "Hermite order K = %d outside [2, 2N-1 = %d]", K, h->lat.k_max);
        if (K < 3 && h->theta != 0.0)
            return fail(LBM_EINVAL, "the energy-flux term (theta != 0) needs K >= 3");
        if (h->initialized) return fail(LBM_ESTATE, "set the Hermite order before lbm_init");
        h->K = K;
        drop_graphs(h);
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_set_hermite_order: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_set_hermite_order: unexpected host exception");
    }
}

lbm_status lbm_set_collision(lbm_t h, int32_t collision, double theta)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (collision != LBM_COLLISION_FILTERED && collision != LBM_COLLISION_BGK)
            return fail(LBM_EINVAL, "unknown collision operator %d", collision);
        if (!std::isfinite(theta)) return fail(LBM_EINVAL, "theta must be finite");
        if (theta != 0.0 && collision != LBM_COLLISION_FILTERED)
            return fail(LBM_EINVAL, "the energy-flux term (theta != 0) belongs to the filtered operator");
        if (theta != 0.0 && h->K < 3) return fail(LBM_EINVAL, "the energy-flux term (theta != 0) needs K >= 3");
        if (h->initialized) return fail(LBM_ESTATE, "set the collision operator before lbm_init");
        h->collision = collision;
        h->theta = theta;
        drop_graphs(h);
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_set_collision: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_set_collision: unexpected host exception");
    }
}

lbm_status lbm_set_stream(lbm_t h, void* hip_stream)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        h->stream = static_cast<hipStream_t>(hip_stream);
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_set_stream: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_set_stream: unexpected host exception");
    }
}

lbm_status lbm_state_bytes(lbm_t h, size_t* bytes_each)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!bytes_each) return fail(LBM_EINVAL, "bytes_each is NULL");
        *bytes_each = h->state_bytes;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_state_bytes: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_state_bytes: unexpected host exception");
    }
}

lbm_status lbm_bind_state(lbm_t h, void* buf_a, void* buf_b, size_t bytes_each)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!buf_a || !buf_b || buf_a == buf_b) return fail(LBM_EINVAL, "need two distinct non-NULL buffers");
        if (bytes_each < h->state_bytes)
            return fail(LBM_EINVAL, "buffers hold %zu bytes, need %zu", bytes_each, h->state_bytes);
        if ((reinterpret_cast<uintptr_t>(buf_a) | reinterpret_cast<uintptr_t>(buf_b)) & 255u)
            return fail(LBM_EINVAL, "buffers must be 256-byte aligned");
        if (h->initialized || h->buf[0]) return fail(LBM_ESTATE, "bind buffers before lbm_init / lbm_set_state");
        h->buf[0] = buf_a;
        h->buf[1] = buf_b;
        h->owns_buf = false;
        h->bound = true;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_bind_state: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_bind_state: unexpected host exception");
    }
}

lbm_status lbm_set_graph_chunk(lbm_t h, int32_t steps)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (steps < 1 || steps > 4096) return fail(LBM_EINVAL, "graph chunk must be in [1, 4096]");
        h->graph_chunk = steps;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_set_graph_chunk: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_set_graph_chunk: unexpected host exception");
    }
}

lbm_status lbm_set_launch(lbm_t h, int32_t block, int32_t grid)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!(block == 0 || block == 64 || block == 128 || block == 256))
            return fail(LBM_EINVAL, "block must be 0, 64, 128 or 256");
        if (grid < 0) return fail(LBM_EINVAL, "grid must be >= 0");
        if (h->initialized) return fail(LBM_ESTATE, "set the launch shape before lbm_init");
        h->block = block;
        h->grid = grid;
        drop_graphs(h);
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_set_launch: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_set_launch: unexpected host exception");
    }
}

lbm_status lbm_set_kernel(lbm_t h, int32_t kernel)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (kernel != LBM_KERNEL_AUTO && kernel != LBM_KERNEL_SCALAR && kernel != LBM_KERNEL_ROW_WAVE &&
            kernel != LBM_KERNEL_IN_PLACE && kernel != LBM_KERNEL_TWO_ROW && kernel != LBM_KERNEL_TWIST &&
            kernel != LBM_KERNEL_TWO_STEP)
            return fail(LBM_EINVAL, "unknown kernel variant %d", kernel);
        if (kernel == LBM_KERNEL_TWO_STEP && !two_step_ok(h))
            return fail(LBM_EINVAL,
                        "the two-step kernel needs a single D3Q15 or D3Q19 box with nx a multiple of %d, ny a "
                        "multiple of %d and one z-plane of populations below 2 GiB",
                        kTwoStepTileX, two_step_tile_y(h->elem));
        if ((kernel == LBM_KERNEL_IN_PLACE || kernel == LBM_KERNEL_TWIST) && !is_single(h))
            return fail(LBM_EINVAL, "the in-place steps are for a single box; batches use the tiled batched kernel");
        if (kernel == LBM_KERNEL_TWO_ROW && (!is_single(h) || h->dims[1] % 2 != 0))
            return fail(LBM_EINVAL, "the two-row step needs a single box with ny even");
        if (kernel == LBM_KERNEL_ROW_WAVE && !row_wave_sites(h))
            return fail(LBM_EINVAL, "the row-wave step needs a single box with nx a multiple of the sites per lane "
                                    "and at most 64 lanes per row");
        // on an initialised handle the state first goes to the natural layout in
        // buf[0], where every kernel can start
        if (lbm_status st = canonicalize(h)) return st;
        h->kernel = kernel;
        drop_graphs(h);
        return enter_kernel_layout(h);
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_set_kernel: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_set_kernel: unexpected host exception");
    }
}

lbm_status lbm_init(lbm_t h, const double* rho, const double* u, int32_t on_device)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!rho || !u) return fail(LBM_EINVAL, "rho or u is NULL");
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        if (lbm_status st = ensure_buffers(h)) return st;
        if (lbm_status st = build_tiles(h)) return st;
        if (lbm_status st = clear_padding(h)) return st;
        const size_t n = size_t(h->nsites);
        double *drho = nullptr, *du = nullptr;
        bool t1 = false, t2 = false;
        if (lbm_status st = stage_in(rho, n, on_device, h->stream, &drho, &t1)) return st;
        if (lbm_status st = stage_in(u, n * h->lat.D, on_device, h->stream, &du, &t2)) {
            if (t1) (void)hipFree(drho);
            return st;
        }
        hipError_t e = launch_init(h->lattice, h->dtype, h->K, twisted(h) ? kTwistEven : kNatural, drho, du, h->buf[0],
                                   h->d_chunks, h->nchunks, h->d_boxes,
                                   h->nsites, h->stream);
        hipError_t e2 = hipStreamSynchronize(h->stream);
        if (t1) (void)hipFree(drho);
        if (t2) (void)hipFree(du);
        if (e != hipSuccess) return fail_hip(e, "init kernel");
        if (e2 != hipSuccess) return fail_hip(e2, "init synchronize");
        h->cur = 0;
        h->t = 0;
        h->initialized = true;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_init: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_init: unexpected host exception");
    }
}

lbm_status lbm_prepare(lbm_t h)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_prepare before lbm_init");
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        if (!one_buffer(h))
            if (lbm_status st = ensure_second(h)) return st;
        for (int p = 0; p < 2; ++p)
            if (lbm_status st = build_graph(h, p)) return st;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_prepare: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_prepare: unexpected host exception");
    }
}

lbm_status lbm_step(lbm_t h, int64_t n)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_step before lbm_init");
        if (n == 0) return LBM_OK;
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        if (!one_buffer(h))
            if (lbm_status st = ensure_second(h)) return st;
        if (lbm_status st = build_tiles(h)) return st;
        const int G = h->graph_chunk;
        int64_t left = n;
        if (G > 1) {
            while (left >= G) {
                if (lbm_status st = build_graph(h, h->cur)) return st;
                HIP_TRY(hipGraphLaunch(h->gexec[h->cur], h->stream), "hipGraphLaunch");
                h->cur ^= int(launches_for(h, G) & 1);
                h->t += G;
                left -= G;
            }
        }
        while (left > 0) {
            const int k = steps_in_launch(h, left);
            hipError_t e = launch_steps(h, h->cur, k, h->stream);
            if (e != hipSuccess) return fail_hip(e, "step kernel launch");
            h->cur ^= 1;
            h->t += k;
            left -= k;
        }
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_step: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_step: unexpected host exception");
    }
}

}  // extern "C"

namespace {


std::string tune_key(const lbm_ctx* h)
{
    char buf[256];
    snprintf(buf, sizeof(buf), "lattice=%d dtype=%d K=%d kind=%d nbox=%d nsites=%lld geometry=%016llx",
             h->lattice, h->dtype, h->K, step_kind(h), h->nbox, (long long)h->nsites,
             (unsigned long long)geometry_hash(h));
    return buf;
}

// Switch the launch; the state is first brought into the natural layout in
// buf[0], the one place every kernel can start from.
lbm_status apply_choice(lbm_ctx* h, const LaunchChoice& c)
{
    if (lbm_status st = canonicalize(h)) return st;
    h->kernel = c.kernel;
    h->block = c.block;
    h->grid = c.grid;
    drop_graphs(h);
    return enter_kernel_layout(h);
}

}  // namespace

extern "C" {

lbm_status lbm_tune(lbm_t h, int32_t steps, const char* cache_path)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_tune needs an initialised state");
        if (!cache_path) cache_path = std::getenv("LBM_TUNE_CACHE");
        const std::string key = tune_key(h);
        LaunchChoice best;
        if (tune_cache_lookup(cache_path, key, &best)) {
            // the cache is a text file: take only values this library can launch
            if (best.kernel < LBM_KERNEL_AUTO || best.kernel > LBM_KERNEL_TWO_STEP) best.kernel = LBM_KERNEL_SCALAR;
            if (best.kernel == LBM_KERNEL_TWO_STEP && !two_step_ok(h)) best.kernel = LBM_KERNEL_SCALAR;
            if (!(best.block == 0 || (best.block >= 64 && best.block <= 256 && best.block % 64 == 0))) best.block = 0;
            if (best.grid < 0) best.grid = 0;
            if (best.kernel == LBM_KERNEL_ROW_WAVE && !row_wave_sites(h)) best.kernel = LBM_KERNEL_SCALAR;
            if ((best.kernel == LBM_KERNEL_IN_PLACE || best.kernel == LBM_KERNEL_TWIST) && !is_single(h))
                best.kernel = LBM_KERNEL_SCALAR;
            if (best.kernel == LBM_KERNEL_TWO_ROW && (!is_single(h) || h->dims[1] % 2 != 0))
                best.kernel = LBM_KERNEL_SCALAR;
            return apply_choice(h, best);
        }
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");

        std::vector<LaunchChoice> cand;
        if (is_single(h)) {
            for (int b : {64, 128, 256}) cand.push_back({LBM_KERNEL_SCALAR, b, 0});
            cand.push_back({LBM_KERNEL_IN_PLACE, 256, 0});
            cand.push_back({LBM_KERNEL_TWIST, 256, 0});
            // a block of one whole x-row (nx rounded up to 64 lanes) when that
            // is none of the above: the x-shifted lines then stay within one
            // workgroup (one L2) instead of being fetched by neighbouring ones
            const int64_t row = ((h->dims[0] + 63) / 64) * 64;
            if (row < 256 && row != 64 && row != 128) {
                cand.push_back({LBM_KERNEL_SCALAR, int(row), 0});
                cand.push_back({LBM_KERNEL_IN_PLACE, int(row), 0});
                cand.push_back({LBM_KERNEL_TWIST, int(row), 0});
            }
            if (h->dims[1] % 2 == 0) cand.push_back({LBM_KERNEL_TWO_ROW, 256, 0});
            if (row_wave_sites(h)) cand.push_back({LBM_KERNEL_ROW_WAVE, 0, 0});
            // the two-step kernel at one and two blocks per compute unit
            if (two_step_ok(h)) {
                cand.push_back({LBM_KERNEL_TWO_STEP, 0, 0});
                cand.push_back({LBM_KERNEL_TWO_STEP, 0, 2 * h->cus});
            }
        } else {
            for (int b : {64, 128, 256})
                for (int g : {0, 1024, 2048, 4096}) cand.push_back({LBM_KERNEL_SCALAR, b, g});
        }

        // tuning steps the state: keep a copy and restore it afterwards; the
        // candidates switch kernels, so start from the natural layout in buf[0]
        const LaunchChoice old = {h->kernel, h->block, h->grid};
        if (lbm_status st = canonicalize(h)) return st;
        const int cur0 = h->cur;
        const int64_t t0 = h->t;
        void* saved = nullptr;
        if (hipError_t me = hipMalloc(&saved, h->state_bytes)) {
            lbm_status fst = fail_hip(me, "hipMalloc(tuning copy)");
            (void)apply_choice(h, old);
            return fst;
        }
        // candidates are timed on direct launches: a graph built inside the
        // timed window would charge its capture to one candidate
        const int chunk0 = h->graph_chunk;
        h->graph_chunk = 1;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipMemcpyAsync(saved, h->buf[cur0], h->state_bytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        lbm_status st = (e == hipSuccess) ? LBM_OK : fail_hip(e, "tuning set-up");
        // Every candidate is timed in kTuneRounds interleaved rounds and keeps its
        // fastest round, so a slow window of the device (clock ramp, a neighbour's
        // traffic) does not decide the choice.
        std::vector<float> cand_ms(cand.size(), 0.f);
        for (int round = 0; round < kTuneRounds && st == LBM_OK; ++round) {
            for (size_t k = 0; k < cand.size() && st == LBM_OK; ++k) {
                if ((st = apply_choice(h, cand[k])) != LBM_OK) break;
                if ((st = lbm_step(h, 2)) != LBM_OK) break;
                if ((e = hipEventRecord(e0, h->stream)) != hipSuccess) { st = fail_hip(e, "hipEventRecord"); break; }
                if ((st = lbm_step(h, steps)) != LBM_OK) break;
                if ((e = hipEventRecord(e1, h->stream)) != hipSuccess) { st = fail_hip(e, "hipEventRecord"); break; }
                if ((e = hipEventSynchronize(e1)) != hipSuccess) { st = fail_hip(e, "hipEventSynchronize"); break; }
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { st = fail_hip(e, "hipEventElapsedTime"); break; }
                if (round == 0 || ms < cand_ms[k]) cand_ms[k] = ms;
            }
        }
        float best_ms = 0.f;
        for (size_t k = 0; k < cand.size(); ++k)
            if (k == 0 || cand_ms[k] < best_ms) {
                best_ms = cand_ms[k];
                best = cand[k];
            }
        // restore the state whatever happened
        hipError_t re = hipMemcpyAsync(h->buf[cur0], saved, h->state_bytes, hipMemcpyDeviceToDevice, h->stream);
        if (re == hipSuccess) re = hipStreamSynchronize(h->stream);
        (void)hipFree(saved);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        // buf[0] holds the saved natural state again, which is the state of
        // the scalar step at cur = 0 (the twist step's even layout is not)
        h->kernel = LBM_KERNEL_SCALAR;
        h->cur = cur0;
        h->t = t0;
        h->graph_chunk = chunk0;
        if (st != LBM_OK) {
            (void)apply_choice(h, old);
            return st;
        }
        if (re != hipSuccess) return fail_hip(re, "restoring the state after tuning");
        if (lbm_status ast = apply_choice(h, best)) return ast;
        tune_cache_store(cache_path, key, best);
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_tune: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_tune: unexpected host exception");
    }
}

lbm_status lbm_moments(lbm_t h, double* rho, double* u, int32_t on_device)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!rho || !u) return fail(LBM_EINVAL, "rho or u is NULL");
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_moments before lbm_init");
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        const size_t n = size_t(h->nsites);
        const int D = h->lat.D;
        double *drho = rho, *du = u;
        if (!on_device) {
            HIP_TRY(hipMalloc(&drho, n * (1 + D) * sizeof(double)), "hipMalloc(moments)");
            du = drho + n;
        }
        const void* state = nullptr;
        int layout = kNatural;
        state_view(h, &state, &layout);
        hipError_t e = launch_moments(h->lattice, h->dtype, state, layout, drho, du, h->d_chunks, h->nchunks,
                                      h->d_boxes, h->nsites, h->stream);
        if (e == hipSuccess && !on_device) {
            e = hipMemcpyAsync(rho, drho, n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(u, du, n * D * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        }
        hipError_t e2 = hipStreamSynchronize(h->stream);
        if (!on_device) (void)hipFree(drho);
        if (e != hipSuccess) return fail_hip(e, "moments");
        if (e2 != hipSuccess) return fail_hip(e2, "moments synchronize");
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_moments: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_moments: unexpected host exception");
    }
}

lbm_status lbm_totals(lbm_t h, double* out)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!out) return fail(LBM_EINVAL, "out is NULL");
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_totals before lbm_init");
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        const void* state = nullptr;
        int layout = kNatural;
        state_view(h, &state, &layout);
        hipError_t e = launch_totals(h->lattice, h->dtype, state, layout, h->d_chunks, h->nchunks,
                                     h->d_box_chunk_begin, h->nbox, h->d_boxes, h->d_partial, h->d_out, h->stream);
        if (e != hipSuccess) return fail_hip(e, "totals kernels");
        HIP_TRY(hipMemcpyAsync(out, h->d_out, size_t(h->nbox) * 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                "copy totals");
        HIP_TRY(hipStreamSynchronize(h->stream), "totals synchronize");
        for (int b = 0; b < h->nbox; ++b) {
            bool ok = out[4 * b] > 0.0;
            for (int k = 0; k < 4; ++k) ok = ok && std::isfinite(out[4 * b + k]);
            if (!ok) return fail(LBM_ENUMERIC, "box %d: non-finite totals or non-positive mass", b);
        }
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_totals: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_totals: unexpected host exception");
    }
}

lbm_status lbm_residual(lbm_t h, const double* rho_ref, const double* u_ref, int32_t on_device, double out[4])
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!rho_ref || !u_ref || !out) return fail(LBM_EINVAL, "NULL argument");
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_residual before lbm_init");
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        const size_t n = size_t(h->nsites);
        double *dr = nullptr, *du = nullptr;
        bool t1 = false, t2 = false;
        if (lbm_status st = stage_in(rho_ref, n, on_device, h->stream, &dr, &t1)) return st;
        if (lbm_status st = stage_in(u_ref, n * h->lat.D, on_device, h->stream, &du, &t2)) {
            if (t1) (void)hipFree(dr);
            return st;
        }
        const void* state = nullptr;
        int layout = kNatural;
        state_view(h, &state, &layout);
        hipError_t e = launch_residual(h->lattice, h->dtype, state, layout, dr, du, h->d_chunks, h->nchunks,
                                       h->d_boxes, h->nsites, h->d_partial, h->d_out, false, h->stream);
        double tmp[4] = {0, 0, 0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(tmp, h->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        hipError_t e2 = hipStreamSynchronize(h->stream);
        if (t1) (void)hipFree(dr);
        if (t2) (void)hipFree(du);
        if (e != hipSuccess) return fail_hip(e, "residual kernels");
        if (e2 != hipSuccess) return fail_hip(e2, "residual synchronize");
        out[0] = tmp[0];
        out[1] = std::sqrt(tmp[1]);
        out[2] = tmp[2];
        out[3] = std::sqrt(tmp[3]);
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_residual: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_residual: unexpected host exception");
    }
}

lbm_status lbm_residual_noalloc(lbm_t h, const double* rho_ref, const double* u_ref, double* out)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!rho_ref || !u_ref || !out) return fail(LBM_EINVAL, "NULL argument");
        if (h->nchunks > kScratchChunks)
            return fail(LBM_EINVAL,
                        "lbm_residual_noalloc: %lld sites need %d reduction chunks; the scratch holds %d (%d sites "
                        "per chunk, %zu bytes); use lbm_residual",
                        (long long)h->nsites, h->nchunks, kScratchChunks, kChunkSites, kScratchBytes);
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_residual_noalloc before lbm_init");
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        double* partial = nullptr;
        if (lbm_status st = scratch_address(h->device, &partial)) return st;
        const void* state = nullptr;
        int layout = kNatural;
        state_view(h, &state, &layout);
        // every partial slot the final kernel reads is written first by this
        // call, so nothing needs clearing
        hipError_t e = launch_residual(h->lattice, h->dtype, state, layout, rho_ref, u_ref, h->d_chunks, h->nchunks,
                                       h->d_boxes, h->nsites, partial, out, true, h->stream);
        if (e != hipSuccess) return fail_hip(e, "residual kernels");
        return LBM_OK;
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_residual_noalloc: unexpected host exception");
    }
}

lbm_status lbm_checkpoint_bytes(lbm_t h, size_t* bytes)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
        *bytes = sizeof(CkptHeader) + size_t(h->lat.Q) * size_t(h->nstored) * h->elem;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_checkpoint_bytes: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_checkpoint_bytes: unexpected host exception");
    }
}

lbm_status lbm_get_state(lbm_t h, void* buf, size_t bytes)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        size_t need = 0;
        lbm_checkpoint_bytes(h, &need);
        if (!buf || bytes < need) return fail(LBM_EINVAL, "checkpoint buffer needs %zu bytes", need);
        if (!h->initialized) return fail(LBM_ESTATE, "lbm_get_state before lbm_init");
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        CkptHeader hd;
        std::memset(&hd, 0, sizeof(hd));
        hd.magic = kCkptMagic;
        hd.lattice = h->lattice;
        hd.dtype = h->dtype;
        hd.K = h->K;
        hd.nbox = h->nbox;
        hd.nsites = h->nsites;
        hd.t = h->t;
        hd.geometry_hash = geometry_hash(h);
        hd.payload_bytes = need - sizeof(CkptHeader);
        std::memcpy(buf, &hd, sizeof(hd));
        char* dst = static_cast<char*>(buf) + sizeof(hd);
        const void* state = nullptr;
        int layout = kNatural;
        state_view(h, &state, &layout);
        const size_t payload = size_t(h->lat.Q) * size_t(h->nstored) * h->elem;
        if (layout == kNatural) {
            HIP_TRY(hipMemcpyAsync(dst, state, payload, hipMemcpyDeviceToHost, h->stream), "copy state to host");
            HIP_TRY(hipStreamSynchronize(h->stream), "get_state synchronize");
        } else {
            // an in-place step left the state in one of its layouts: copy it out
            // as it is and put it into the natural layout on the host (no second
            // device buffer)
            std::vector<char> tmp;
            try {
                tmp.resize(payload);
            } catch (const std::bad_alloc&) {
                return fail(LBM_ENOMEM, "host staging for the checkpoint");
            }
            HIP_TRY(hipMemcpyAsync(tmp.data(), state, payload, hipMemcpyDeviceToHost, h->stream), "copy state to host");
            HIP_TRY(hipStreamSynchronize(h->stream), "get_state synchronize");
            relayout_host(h, layout, true, tmp.data(), dst);
        }
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_get_state: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_get_state: unexpected host exception");
    }
}

lbm_status lbm_set_state(lbm_t h, const void* buf, size_t bytes)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        size_t need = 0;
        lbm_checkpoint_bytes(h, &need);
        CkptHeader expect;
        std::memset(&expect, 0, sizeof(expect));
        expect.lattice = h->lattice;
        expect.dtype = h->dtype;
        expect.K = h->K;
        expect.nbox = h->nbox;
        expect.nsites = h->nsites;
        expect.geometry_hash = geometry_hash(h);
        expect.payload_bytes = need - sizeof(CkptHeader);
        std::string why;
        if (!check_checkpoint(buf, bytes, expect, &why)) return fail(LBM_EINVAL, "%s", why.c_str());
        CkptHeader hd;
        std::memcpy(&hd, buf, sizeof(hd));
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        if (lbm_status st = ensure_buffers(h)) return st;
        if (lbm_status st = build_tiles(h)) return st;
        const char* src = static_cast<const char*>(buf) + sizeof(hd);
        if (lbm_status st = clear_padding(h)) return st;
        const size_t payload = size_t(h->lat.Q) * size_t(h->nstored) * h->elem;
        std::vector<char> tmp;
        if (twisted(h)) {
            // the twist step starts from its even-time layout: rearrange the
            // natural checkpoint on the host (no second device buffer)
            try {
                tmp.resize(payload);
            } catch (const std::bad_alloc&) {
                return fail(LBM_ENOMEM, "host staging for the checkpoint");
            }
            relayout_host(h, kTwistEven, false, src, tmp.data());
            src = tmp.data();
        }
        HIP_TRY(hipMemcpyAsync(h->buf[0], src, payload, hipMemcpyHostToDevice, h->stream), "copy state to device");
        HIP_TRY(hipStreamSynchronize(h->stream), "set_state synchronize");
        h->cur = 0;
        h->t = hd.t;
        h->initialized = true;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_set_state: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_set_state: unexpected host exception");
    }
}

lbm_status lbm_get_info(lbm_t h, lbm_info* info)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        if (!info) return fail(LBM_EINVAL, "info is NULL");
        std::memset(info, 0, sizeof(*info));
        info->lattice = h->lattice;
        info->dtype = h->dtype;
        info->D = h->lat.D;
        info->Q = h->lat.Q;
        info->two_n = h->lat.two_n;
        info->K = h->K;
        info->T0 = h->lat.T0;
        info->nbox = h->nbox;
        for (int a = 0; a < 3; ++a) info->dims[a] = h->dims[a];
        info->nsites = h->nsites;
        info->t = h->t;
        info->bytes_per_site_update = int64_t(2 * h->lat.Q) * int64_t(h->elem);
        info->state_bytes = h->state_bytes;
        info->block = effective_block(h);
        info->grid = two_step(h) ? two_step_grid(h) : h->grid;
        info->graph_chunk = h->graph_chunk;
        info->kernel = effective_kernel(h);
        info->collision = h->collision;
        info->theta = h->theta;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_get_info: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_get_info: unexpected host exception");
    }
}

lbm_status lbm_sync(lbm_t h)
{
    try {
        if (lbm_status st = check_handle(h)) return st;
        HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_sync: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_sync: unexpected host exception");
    }
}

lbm_status lbm_destroy(lbm_t h)
{
    try {
        if (!h) return LBM_OK;
        (void)hipSetDevice(h->device);
        (void)hipStreamSynchronize(h->stream);
        free_all(h);
        delete h;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_destroy: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_destroy: unexpected host exception");
    }
}

const char* lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_lattice_table(int32_t lattice, int32_t* D, int32_t* Q, double* T0, int32_t* two_n, int32_t* c,
                             double* w)
{
    try {
        LatticeInfo L;
        if (!lattice_info(lattice, &L)) return fail(LBM_EINVAL, "unknown lattice %d", lattice);
        if (D) *D = L.D;
        if (Q) *Q = L.Q;
        if (T0) *T0 = L.T0;
        if (two_n) *two_n = L.two_n;
        for (int i = 0; i < L.Q; ++i) {
            if (c)
                for (int a = 0; a < 3; ++a) c[i * 3 + a] = L.c[i * 3 + a];
            if (w) w[i] = L.w[i];
        }
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_lattice_table: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_lattice_table: unexpected host exception");
    }
}

lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, int32_t reps, void* hip_stream,
                          double* ms_per_copy)
{
    try {
        if (!dst || !src || !ms_per_copy || reps < 1 || bytes == 0 || (bytes % 16) != 0)
            return fail(LBM_EINVAL, "copy probe needs non-NULL buffers, reps >= 1 and bytes a positive multiple of 16");
        int dev = 0;
        if (lbm_status st = device_check(&dev)) return st;
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
        hipError_t e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail_hip(e, "hipEventCreate");
        }
        e = launch_copy(dst, src, bytes, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(dst, src, bytes, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (e != hipSuccess) return fail_hip(e, "copy probe");
        *ms_per_copy = double(ms) / reps;
        return LBM_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "lbm_copy_probe: host memory allocation failed");
    } catch (...) {
        return fail(LBM_EDEVICE, "lbm_copy_probe: unexpected host exception");
    }
}

}  // extern "C"
