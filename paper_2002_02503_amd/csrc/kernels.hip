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

// Initialisation: f := f^eq_K(rho, u) (eq. hermite), evaluated in double and
// rounded once to the storage type (set-up, not part of the step).
template <class L, class S, int K>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ rho, const double* __restrict__ u,
                                              S* __restrict__ dst, const ChunkDesc* __restrict__ chunks,
                                              const BoxDesc* __restrict__ boxes, long long nsites)
{
    using ST = Store<S>;
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    S* base = dst + b.mem;
    for (int k = threadIdx.x; k < ch.count; k += blockDim.x) {
        const long long s = ch.start + k;
        const long long e = site_elem(s - b.offset, b.w, L::Q);
        const double ux = u[s];
        const double uy = u[nsites + s];
        const double uz = (L::D == 3) ? u[2 * nsites + s] : 0.0;
        double g[L::Q];
        equilibrium_scaled<L, K, double>(rho[s] - 1.0, ux, uy, uz, g);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int m = mem_row<L>(i);
            ST::put_d(base + e + (long long)m * b.w, g[i]);
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

// The same for a box whose state the in-place step left in the swapped layout:
// population i of site (x, y, z) sits at site (x, y, z) + c_i, tile row
// m(opp(i)).  `local` is the site's index inside its box.  Single boxes only
// (row tiles, w = nx).
template <class L, class S>
__device__ __forceinline__ void swapped_site_moments(const S* __restrict__ base, long long local, const BoxDesc& b,
                                                     double& dsum, double (&j)[3])
{
    using ST = Store<S>;
    const long long r = local / b.nx;
    const int x = int(local - r * b.nx);
    const int y = int(r % b.ny);
    const int z = int(r / b.ny);
    const long long tile = (long long)L::Q * b.nx;
    dsum = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        constexpr int m = mem_row<L>(opp(i));
        const int xs = wrap_coord(x + cx, b.nx), ys = wrap_coord(y + cy, b.ny), zs = wrap_coord(z + cz, b.nz);
        const double gi = double(ST::get(base + ((long long)zs * b.ny + ys) * tile + (long long)m * b.nx + xs));
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

template <class L, class S, bool SWAPPED>
__device__ __forceinline__ void stored_site_moments(const S* __restrict__ base, long long local, const BoxDesc& b,
                                                    double& dsum, double (&j)[3])
{
    if constexpr (SWAPPED) swapped_site_moments<L, S>(base, local, b, dsum, j);
    else site_moments<L, S>(base + site_elem(local, b.w, L::Q), b.w, dsum, j);
}

template <class L, class S, bool SWAPPED>
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
        stored_site_moments<L, S, SWAPPED>(base, s - b.offset, b, d, j);
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

template <class L, class S, bool SWAPPED>
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
        stored_site_moments<L, S, SWAPPED>(base, ch.start + k - b.offset, b, d, j);
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

template <class L, class S, bool SWAPPED>
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
        stored_site_moments<L, S, SWAPPED>(base, s - b.offset, b, d, j);
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

hipError_t launch_init(int lat, int dtype, int K, const double* rho, const double* u, void* dst,
                       const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites, hipStream_t s)
{
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        constexpr int KK = decltype(Kc)::value;
        k_init<L, S, KK><<<nchunks, 256, 0, s>>>(rho, u, static_cast<S*>(dst), chunks, boxes, nsites);
        return hipGetLastError();
    });
}

hipError_t launch_moments(int lat, int dtype, const void* src, bool swapped, double* rho, double* u,
                          const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        if (swapped)
            k_moments<L, S, true><<<nchunks, 256, 0, s>>>(static_cast<const S*>(src), rho, u, chunks, boxes, nsites);
        else
            k_moments<L, S, false><<<nchunks, 256, 0, s>>>(static_cast<const S*>(src), rho, u, chunks, boxes, nsites);
        return hipGetLastError();
    });
}

hipError_t launch_totals(int lat, int dtype, const void* src, bool swapped, const ChunkDesc* chunks, int nchunks,
                         const int* box_chunk_begin, int nbox, const BoxDesc* boxes, double* partial, double* out,
                         hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        if (swapped)
            k_totals_partial<L, S, true><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), chunks, boxes,
                                                                       partial);
        else
            k_totals_partial<L, S, false><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), chunks, boxes,
                                                                        partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_totals_final<<<nbox, kRedBlock, 0, s>>>(partial, box_chunk_begin, out);
        return hipGetLastError();
    });
}

hipError_t launch_residual(int lat, int dtype, const void* src, bool swapped, const double* rho_ref,
                           const double* u_ref, const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes,
                           long long nsites, double* partial, double* out, bool sqrt_l2, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        if (swapped)
            k_residual_partial<L, S, true><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), rho_ref, u_ref,
                                                                         chunks, boxes, nsites, partial);
        else
            k_residual_partial<L, S, false><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), rho_ref, u_ref,
                                                                          chunks, boxes, nsites, partial);
        hipError_t e = hipGetLastError();
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

// Swapped layout of the in-place step -> natural layout, into another buffer:
// population j of site x is read from site x + c_j, tile row m(opp(j)).  A
// pure permutation of stored values (bit-exact), single box.
template <class L, class S>
__global__ __launch_bounds__(256) void k_unswap(const S* __restrict__ src, S* __restrict__ dst, StepGeom geo)
{
    constexpr int RR = L::R;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const int x = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (x >= geo.nx) return;
    const long long tile = (long long)L::Q * geo.nx;
    int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * RR; ++k) {
        xw[k] = wrap_coord(x + k - RR, geo.nx);
        yw[k] = wrap_coord(y + k - RR, geo.ny);
        zw[k] = wrap_coord(z + k - RR, geo.nz);
    }
    S* q = dst + (long long)(z * geo.ny + y) * tile;
    unroll<L::Q>([&](auto J) {
        constexpr int j = decltype(J)::value;
        constexpr int cx = L::c[j][0], cy = L::c[j][1], cz = L::c[j][2];
        const int row = zw[RR + cz] * geo.ny + yw[RR + cy];
        constexpr int m_src = mem_row<L>(opp(j));
        constexpr int m_dst = mem_row<L>(j);
        const S* p = src + row * tile + (long long)m_src * geo.nx;
        q[(long long)m_dst * geo.nx + x] = p[xw[RR + cx]];
    });
}

hipError_t launch_unswap(int lat, int dtype, const void* src, void* dst, const StepGeom& geo, int block,
                         hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        k_unswap<L, S><<<dim3(unsigned(geo.xblocks), unsigned(geo.ny), unsigned(geo.nz)), block, 0, s>>>(
            static_cast<const S*>(src), static_cast<S*>(dst), geo);
        return hipGetLastError();
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

hipError_t launch_step_batch(int lat, int dtype, int K, int kind, const void* src, void* dst, const TileDesc* tiles,
                             int ntiles, double theta, int block, int grid, bool aligned_rows, hipStream_t s)
{
    return by_pair(lat, dtype, [&](auto Lt, auto* Sp) {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        return launch_step_batch_l<L, S>(K, kind, src, dst, tiles, ntiles, theta, block, grid, aligned_rows, s);
    });
}

// ---------------------------------------------------------------------------
// Host copies of the descriptors.
// ---------------------------------------------------------------------------

template <class L>
static void fill_info(LatticeInfo* out)
{
    out->D = L::D;
    out->Q = L::Q;
    out->two_n = L::TWO_N;
    out->k_default = L::K_DEFAULT;
    out->k_max = L::K_MAX;
    out->R = L::R;
    out->T0 = L::T0;
    out->c.resize(L::Q * 3);
    out->w.resize(L::Q);
    out->mrow.resize(L::Q);
    for (int i = 0; i < L::Q; ++i) {
        for (int a = 0; a < 3; ++a) out->c[i * 3 + a] = L::c[i][a];
        out->w[i] = L::w[i];
        out->mrow[i] = mem_row<L>(i);
    }
}

bool lattice_info(int lat, LatticeInfo* out)
{
    switch (lat) {
    case kD2Q9: fill_info<D2Q9>(out); return true;
    case kD3Q15: fill_info<D3Q15>(out); return true;
    case kD3Q19: fill_info<D3Q19>(out); return true;
    case kD3Q39: fill_info<D3Q39>(out); return true;
    default: return false;
    }
}

size_t storage_bytes(int dtype)
{
    switch (dtype) {
    case 0: return 8;
    case 1: return 4;
    case 2: return 2;
    case 3: return 2;
    default: return 0;
    }
}

}  // namespace lbm
