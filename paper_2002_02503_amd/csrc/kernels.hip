// HIP kernels for gfx950 (MI355X) around the step: initialisation, moments,
// FP64 reductions and a copy kernel used to calibrate bandwidth measurements.
// The step kernels are in step.hpp (single box) and step_batch.hpp (batch).
//
// Data layout: blocked structure of arrays, row tiles for a single box and
// 64-site blocks for a batch (see internal.hpp, BoxDesc).  Two buffers
// alternate: a step reads one and writes the other, so a step never reads what
// it writes.  The stored value is G_i = S (f_i - w_i), the deviation from the
// rest weights in units of the lattice's weight quantum 1/S.
//
// The step is bandwidth bound (about 400 single-precision operations against
// 2 Q S bytes per site, far below the FP32 ridge of the chip), so it uses no
// matrix cores: every population is read once (pull form of eq. lbe, periodic
// wrap) and written once, and the collision runs entirely in registers.
#include "device.hpp"
#include "step_launch.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Set-up, moments and reductions work on chunks: runs of consecutive sites
// of one box, one block per chunk.
// ---------------------------------------------------------------------------

// Element index of population 0 of a site, relative to the box's first
// element, in a layout of w-site blocks (BoxDesc): block local / w, position
// local % w; population i is m(i) * w further on.
__device__ __forceinline__ long long site_elem(long long local, int w, int Q)
{
    const long long r = local / w;
    const long long x = local - r * w;
    return r * Q * w + x;
}

// Element of population i of the site `local` of a single box (row tiles,
// w = nx) when the state is in layout LAYOUT (StateLayout, internal.hpp):
// natural: the site's own cell, tile row m(i); swapped: cell x + c_i, tile row
// m(opp(i)); twisted: cell x + b_i (b_i the positive part of c_i), tile row
// m(i) at even times and m(opp(i)) at odd times.
template <class L, int LAYOUT, int I>
__device__ __forceinline__ long long layout_elem(long long local, const BoxDesc& b)
{
    const long long r = local / b.nx;
    const int x = int(local - r * b.nx);
    const int y = int(r % b.ny);
    const int z = int(r / b.ny);
    const long long tile = (long long)L::Q * b.nx;
    constexpr bool SW = (LAYOUT == kSwapped);
    constexpr int ox = SW ? L::c[I][0] : twist_offset<L>(I, 0);
    constexpr int oy = SW ? L::c[I][1] : twist_offset<L>(I, 1);
    constexpr int oz = SW ? L::c[I][2] : twist_offset<L>(I, 2);
    constexpr int m = (LAYOUT == kTwistEven) ? mem_row<L>(I) : mem_row<L>(opp(I));
    const int xs = wrap_coord(x + ox, b.nx), ys = wrap_coord(y + oy, b.ny), zs = wrap_coord(z + oz, b.nz);
    return ((long long)zs * b.ny + ys) * tile + (long long)m * b.nx + xs;
}

// Initialisation: f := f^eq_K(rho, u) (eq. hermite), evaluated in double and
// rounded once to the storage type (set-up, not part of the step), written in
// the natural layout or (single box) the twisted layout of an even time.
template <class L, class S, int K, int LAYOUT>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ rho, const double* __restrict__ u,
                                              S* __restrict__ dst, const ChunkDesc* __restrict__ chunks,
                                              const BoxDesc* __restrict__ boxes, long long nsites)
{
    using ST = Store<S>;
    static_assert(LAYOUT == kNatural || LAYOUT == kTwistEven, "init writes a layout of time 0");
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    S* base = dst + b.mem;
    for (int k = threadIdx.x; k < ch.count; k += blockDim.x) {
        const long long s = ch.start + k;
        const long long local = s - b.offset;
        const long long e = site_elem(local, b.w, L::Q);
        const double ux = u[s];
        const double uy = u[nsites + s];
        const double uz = (L::D == 3) ? u[2 * nsites + s] : 0.0;
        double g[L::Q];
        equilibrium_scaled<L, K, double>(rho[s] - 1.0, ux, uy, uz, g);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (LAYOUT == kNatural) ST::put_d(base + e + (long long)mem_row<L>(i) * b.w, g[i]);
            else ST::put_d(base + layout_elem<L, LAYOUT, i>(local, b), g[i]);
        });
    }
}

// rho - 1 and rho u (eq. mme) of one stored site, in double (outside the
// step, for output and reductions).  `p` points at population 0 of the site,
// w is the block width of the box's layout.
template <class L, class S>
__device__ __forceinline__ void site_moments(const S* __restrict__ p, int w, double& dsum, double (&j)[3])
{
    using ST = Store<S>;
    dsum = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        constexpr int m = mem_row<L>(i);
        const double gi = double(ST::get(p + (long long)m * w));
        dsum += gi;
        if constexpr (cx != 0) j[0] += double(cx) * gi;
        if constexpr (cy != 0) j[1] += double(cy) * gi;
        if constexpr (cz != 0) j[2] += double(cz) * gi;
    });
    // stored units are 1/S of a population
    dsum /= double(L::S);
    j[0] /= double(L::S);
    j[1] /= double(L::S);
    j[2] /= double(L::S);
}

// The same for a single box whose state is in one of the in-place steps'
// layouts (layout_elem).  `local` is the site's index inside its box.
template <class L, class S, int LAYOUT>
__device__ __forceinline__ void relaid_site_moments(const S* __restrict__ base, long long local, const BoxDesc& b,
                                                    double& dsum, double (&j)[3])
{
    using ST = Store<S>;
    dsum = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const double gi = double(ST::get(base + layout_elem<L, LAYOUT, i>(local, b)));
        dsum += gi;
        if constexpr (cx != 0) j[0] += double(cx) * gi;
        if constexpr (cy != 0) j[1] += double(cy) * gi;
        if constexpr (cz != 0) j[2] += double(cz) * gi;
    });
    dsum /= double(L::S);
    j[0] /= double(L::S);
    j[1] /= double(L::S);
    j[2] /= double(L::S);
}

template <class L, class S, int LAYOUT>
__device__ __forceinline__ void stored_site_moments(const S* __restrict__ base, long long local, const BoxDesc& b,
                                                    double& dsum, double (&j)[3])
{
    if constexpr (LAYOUT != kNatural) relaid_site_moments<L, S, LAYOUT>(base, local, b, dsum, j);
    else site_moments<L, S>(base + site_elem(local, b.w, L::Q), b.w, dsum, j);
}

template <class L, class S, int LAYOUT>
__global__ __launch_bounds__(256) void k_moments(const S* __restrict__ src, double* __restrict__ rho,
                                                 double* __restrict__ u, const ChunkDesc* __restrict__ chunks,
                                                 const BoxDesc* __restrict__ boxes, long long nsites)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    const S* base = src + b.mem;
    for (int k = threadIdx.x; k < ch.count; k += blockDim.x) {
        const long long s = ch.start + k;
        double d, j[3];
        stored_site_moments<L, S, LAYOUT>(base, s - b.offset, b, d, j);
        const double r = 1.0 + d;
        rho[s] = r;
#pragma unroll
        for (int a = 0; a < L::D; ++a) u[a * nsites + s] = j[a] / r;
    }
}

// ---------------------------------------------------------------------------
// FP64 reductions with a fixed order: per-chunk partials (one block per
// chunk, LDS tree), then per-box (or global) sums over chunks in order.
// ---------------------------------------------------------------------------

constexpr int kRedBlock = 256;

template <int NV>
__device__ __forceinline__ void block_tree(double (&acc)[NV], const bool (&is_max)[NV])
{
    __shared__ double sh[NV][kRedBlock];
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][tid] = acc[k];
    __syncthreads();
    for (int off = kRedBlock / 2; off > 0; off >>= 1) {
        if (tid < off) {
#pragma unroll
            for (int k = 0; k < NV; ++k)
                sh[k][tid] = is_max[k] ? fmax(sh[k][tid], sh[k][tid + off]) : sh[k][tid] + sh[k][tid + off];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = sh[k][0];
}

template <class L, class S, int LAYOUT>
__global__ __launch_bounds__(kRedBlock) void k_totals_partial(const S* __restrict__ src,
                                                              const ChunkDesc* __restrict__ chunks,
                                                              const BoxDesc* __restrict__ boxes,
                                                              double* __restrict__ partial)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    const S* base = src + b.mem;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < ch.count; k += kRedBlock) {
        double d, j[3];
        stored_site_moments<L, S, LAYOUT>(base, ch.start + k - b.offset, b, d, j);
        acc[0] += d;
        acc[1] += j[0];
        acc[2] += j[1];
        acc[3] += j[2];
    }
    const bool is_max[4] = {false, false, false, false};
    block_tree<4>(acc, is_max);
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 4 + 0] = double(ch.count) + acc[0];  // sum rho = sites + sum (rho - 1)
        partial[blockIdx.x * 4 + 1] = acc[1];
        partial[blockIdx.x * 4 + 2] = acc[2];
        partial[blockIdx.x * 4 + 3] = acc[3];
    }
}

__global__ __launch_bounds__(kRedBlock) void k_totals_final(const double* __restrict__ partial,
                                                            const int* __restrict__ box_chunk_begin,
                                                            double* __restrict__ out)
{
    const int b = blockIdx.x;
    const int c0 = box_chunk_begin[b], c1 = box_chunk_begin[b + 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = c0 + int(threadIdx.x); c < c1; c += kRedBlock)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += partial[c * 4 + k];
    const bool is_max[4] = {false, false, false, false};
    block_tree<4>(acc, is_max);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) out[b * 4 + k] = acc[k];
}

template <class L, class S, int LAYOUT>
__global__ __launch_bounds__(kRedBlock) void k_residual_partial(const S* __restrict__ src,
                                                                const double* __restrict__ rho_ref,
                                                                const double* __restrict__ u_ref,
                                                                const ChunkDesc* __restrict__ chunks,
                                                                const BoxDesc* __restrict__ boxes,
                                                                long long nsites, double* __restrict__ partial)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    const S* base = src + b.mem;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // max |du|, sum du^2, max |drho|, sum drho^2
    for (int k = threadIdx.x; k < ch.count; k += kRedBlock) {
        const long long s = ch.start + k;
        double d, j[3];
        stored_site_moments<L, S, LAYOUT>(base, s - b.offset, b, d, j);
        const double r = 1.0 + d;
#pragma unroll
        for (int a = 0; a < L::D; ++a) {
            const double du = j[a] / r - u_ref[a * nsites + s];
            acc[0] = fmax(acc[0], fabs(du));
            acc[1] += du * du;
        }
        const double dr = r - rho_ref[s];
        acc[2] = fmax(acc[2], fabs(dr));
        acc[3] += dr * dr;
    }
    const bool is_max[4] = {true, false, true, false};
    block_tree<4>(acc, is_max);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) partial[blockIdx.x * 4 + k] = acc[k];
}

// sqrt_l2: write the square roots of the two sums (the L2 norms) instead of
// the sums themselves.
__global__ __launch_bounds__(kRedBlock) void k_residual_final(const double* __restrict__ partial, int nchunks,
                                                              double* __restrict__ out, int sqrt_l2)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < nchunks; c += kRedBlock) {
        acc[0] = fmax(acc[0], partial[c * 4 + 0]);
        acc[1] += partial[c * 4 + 1];
        acc[2] = fmax(acc[2], partial[c * 4 + 2]);
        acc[3] += partial[c * 4 + 3];
    }
    const bool is_max[4] = {true, false, true, false};
    block_tree<4>(acc, is_max);
    if (threadIdx.x == 0) {
        out[0] = acc[0];
        out[1] = sqrt_l2 ? sqrt(acc[1]) : acc[1];
        out[2] = acc[2];
        out[3] = sqrt_l2 ? sqrt(acc[3]) : acc[3];
    }
}

// ---------------------------------------------------------------------------
// Plain 16-byte-vector copy with non-temporal accesses, one vector per thread.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

// Calls f(integral_constant layout) for a runtime StateLayout.
template <class F>
static hipError_t by_layout(int layout, F&& f)
{
    switch (layout) {
    case kNatural: return f(ic<kNatural>{});
    case kSwapped: return f(ic<kSwapped>{});
    case kTwistEven: return f(ic<kTwistEven>{});
    case kTwistOdd: return f(ic<kTwistOdd>{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(int lat, int dtype, int K, int layout, const double* rho, const double* u, void* dst,
                       const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites, hipStream_t s)
{
    if (layout != kNatural && layout != kTwistEven) return hipErrorInvalidValue;
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        constexpr int KK = decltype(Kc)::value;
        if (layout == kTwistEven)
            k_init<L, S, KK, kTwistEven><<<nchunks, 256, 0, s>>>(rho, u, static_cast<S*>(dst), chunks, boxes, nsites);
        else
            k_init<L, S, KK, kNatural><<<nchunks, 256, 0, s>>>(rho, u, static_cast<S*>(dst), chunks, boxes, nsites);
        return hipGetLastError();
    });
}

hipError_t launch_moments(int lat, int dtype, const void* src, int layout, double* rho, double* u,
                          const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return by_layout(layout, [&](auto Lay) -> hipError_t {
            constexpr int LAY = decltype(Lay)::value;
            k_moments<L, S, LAY><<<nchunks, 256, 0, s>>>(static_cast<const S*>(src), rho, u, chunks, boxes, nsites);
            return hipGetLastError();
        });
    });
}

hipError_t launch_totals(int lat, int dtype, const void* src, int layout, const ChunkDesc* chunks, int nchunks,
                         const int* box_chunk_begin, int nbox, const BoxDesc* boxes, double* partial, double* out,
                         hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        hipError_t e = by_layout(layout, [&](auto Lay) -> hipError_t {
            constexpr int LAY = decltype(Lay)::value;
            k_totals_partial<L, S, LAY><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), chunks, boxes,
                                                                      partial);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        k_totals_final<<<nbox, kRedBlock, 0, s>>>(partial, box_chunk_begin, out);
        return hipGetLastError();
    });
}

hipError_t launch_residual(int lat, int dtype, const void* src, int layout, const double* rho_ref,
                           const double* u_ref, const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes,
                           long long nsites, double* partial, double* out, bool sqrt_l2, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        hipError_t e = by_layout(layout, [&](auto Lay) -> hipError_t {
            constexpr int LAY = decltype(Lay)::value;
            k_residual_partial<L, S, LAY><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), rho_ref, u_ref,
                                                                        chunks, boxes, nsites, partial);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        k_residual_final<<<1, kRedBlock, 0, s>>>(partial, nchunks, out, sqrt_l2 ? 1 : 0);
        return hipGetLastError();
    });
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    const size_t g = (n + 255) / 256;
    if (g == 0 || g > 0x7fffffffu) return hipErrorInvalidValue;
    k_copy<<<unsigned(g), 256, 0, s>>>(static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n);
    return hipGetLastError();
}

// Layout conversions of a single box's state between the natural layout and
// one of the in-place steps' layouts (layout_elem), into another buffer: a
// pure permutation of stored values (bit-exact).  TO_NATURAL: population i of
// site x is read at its element in LAYOUT and written to its natural element;
// otherwise the other way round.  One thread per site.
template <class L, class S, int LAYOUT, bool TO_NATURAL>
__global__ __launch_bounds__(256) void k_relayout(const S* __restrict__ src, S* __restrict__ dst, BoxDesc b)
{
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const int x = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (x >= b.nx) return;
    const long long local = ((long long)z * b.ny + y) * b.nx + x;
    const long long nat = site_elem(local, b.nx, L::Q);
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const long long e = layout_elem<L, LAYOUT, i>(local, b);
        const long long n = nat + (long long)mem_row<L>(i) * b.nx;
        if constexpr (TO_NATURAL) dst[n] = src[e];
        else dst[e] = src[n];
    });
}

hipError_t launch_relayout(int lat, int dtype, int layout, bool to_natural, const void* src, void* dst,
                           const StepGeom& geo, int block, hipStream_t s)
{
    if (layout == kNatural) return hipErrorInvalidValue;
    BoxDesc b{};
    b.nx = geo.nx;
    b.ny = geo.ny;
    b.nz = geo.nz;
    b.w = geo.nx;
    const dim3 grid(unsigned(geo.xblocks), unsigned(geo.ny), unsigned(geo.nz));
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return by_layout(layout, [&](auto Lay) -> hipError_t {
            constexpr int LAY = decltype(Lay)::value;
            if constexpr (LAY != kNatural) {
                if (to_natural)
                    k_relayout<L, S, LAY, true><<<grid, block, 0, s>>>(static_cast<const S*>(src),
                                                                       static_cast<S*>(dst), b);
                else
                    k_relayout<L, S, LAY, false><<<grid, block, 0, s>>>(static_cast<const S*>(src),
                                                                        static_cast<S*>(dst), b);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        });
    });
}

// ---------------------------------------------------------------------------
// Runtime-lattice entry points of the step kernels (instances compiled per
// lattice in step_<lattice>.hip and batch_<lattice>.hip).
// ---------------------------------------------------------------------------

// Calls f(L{}, (S*)nullptr) for a runtime (lattice, dtype).
template <class F>
static hipError_t by_pair(int lat, int dtype, F&& f)
{
    return dispatch_kind(lat, dtype, 2, kFiltered,
                         [&](auto Lt, auto* Sp, auto, auto) -> hipError_t { return f(Lt, Sp); });
}

hipError_t launch_step(int lat, int dtype, int K, int kind, const void* src, void* dst, const StepGeom& geo,
                       double omega, double theta, int block, bool pair, hipStream_t s)
{
    return by_pair(lat, dtype, [&](auto Lt, auto* Sp) {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return launch_step_l<L, S>(K, kind, src, dst, geo, omega, theta, block, pair, s);
    });
}

hipError_t launch_step2(int lat, int dtype, int K, int kind, const void* src, void* dst, const Step2Geom& geo,
                        double omega, double theta, int grid, hipStream_t s)
{
    return by_pair(lat, dtype, [&](auto Lt, auto* Sp) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        if constexpr (std::is_same<L, D3Q15>::value || std::is_same<L, D3Q19>::value)
            return launch_step2_l<L, S>(K, kind, src, dst, geo, omega, theta, grid, s);
        else
            return hipErrorInvalidValue;
    });
}

int vec_sites_per_lane(int lat, int dtype)
{
    int v = 0;
    (void)by_pair(lat, dtype, [&](auto Lt, auto* Sp) {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        v = vec_sites_l<L, S>();
        return hipSuccess;
    });
    return v;
}

hipError_t launch_step_vec(int lat, int dtype, int K, int kind, const void* src, void* dst, const VecGeom& geo,
                           double omega, double theta, hipStream_t s)
{
    return by_pair(lat, dtype, [&](auto Lt, auto* Sp) {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return launch_step_vec_l<L, S>(K, kind, src, dst, geo, omega, theta, s);
    });
}

hipError_t launch_step_ip(int lat, int dtype, int K, int kind, void* buf, bool from_natural, const StepGeom& geo,
                          double omega, double theta, int block, hipStream_t s)
{
    return by_pair(lat, dtype, [&](auto Lt, auto* Sp) {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return launch_step_ip_l<L, S>(K, kind, buf, from_natural, geo, omega, theta, block, s);
    });
}

hipError_t launch_step_tw(int lat, int dtype, int K, int kind, void* buf, bool even, const StepGeom& geo,
                          double omega, double theta, int block, hipStream_t s)
{
    return by_pair(lat, dtype, [&](auto Lt, auto* Sp) {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return launch_step_tw_l<L, S>(K, kind, buf, even, geo, omega, theta, block, s);
    });
}

hipError_t launch_step_batch(int lat, int dtype, int K, int kind, const void* src, void* dst, const TileDesc* tiles,
                             int ntiles, double theta, int block, int grid, bool aligned_rows, hipStream_t s)
{
    return by_pair(lat, dtype, [&](auto Lt, auto* Sp) {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return launch_step_batch_l<L, S>(K, kind, src, dst, tiles, ntiles, theta, block, grid, aligned_rows, s);
    });
}

}  // namespace lbm
