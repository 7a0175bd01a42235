// HIP kernels for gfx950 (MI355X): the fused pull-stream + collide step
// (single box and batched), initialisation, moments, FP64 reductions and a
// copy kernel used to calibrate bandwidth measurements.
//
// Data layout: structure of arrays.  Population i of site s lives at
// buf[i * plane + s], s = (z * ny + y) * nx + x (x fastest); plane is the site
// count rounded up so every plane starts on a 256-byte boundary.  Two buffers
// alternate: a step reads one and writes the other, so a step never reads
// what it writes.  The stored value is G_i = S (f_i - w_i), the deviation from
// the rest weights in units of the lattice's weight quantum 1/S.
//
// The step is bandwidth bound (about 600 flops against 2 Q S bytes per site,
// far below the FP32 ridge of the chip), so it uses no matrix cores: one thread
// per site, every population read once (pull form of eq. lbe, periodic wrap)
// and written once, the collision entirely in registers.
#include <type_traits>

#include "collide.hpp"
#include "internal.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Storage types.  FP16 and BF16 are converted with round-to-nearest-even,
// keeping subnormals.
// ---------------------------------------------------------------------------

struct bf16_t {
    uint16_t bits;
};

template <class S>
struct Store;

template <>
struct Store<double> {
    using R = double;
    static __device__ __forceinline__ R get(const double* p) { return *p; }
    static __device__ __forceinline__ void put(double* p, R v) { *p = v; }
    static __device__ __forceinline__ void put_d(double* p, double v) { *p = v; }
};

template <>
struct Store<float> {
    using R = float;
    static __device__ __forceinline__ R get(const float* p) { return *p; }
    static __device__ __forceinline__ void put(float* p, R v) { *p = v; }
    static __device__ __forceinline__ void put_d(float* p, double v) { *p = float(v); }
};

template <>
struct Store<_Float16> {
    using R = float;
    static __device__ __forceinline__ R get(const _Float16* p) { return float(*p); }
    static __device__ __forceinline__ void put(_Float16* p, R v) { *p = _Float16(v); }
    static __device__ __forceinline__ void put_d(_Float16* p, double v) { *p = _Float16(v); }
};

template <>
struct Store<bf16_t> {
    using R = float;
    static __device__ __forceinline__ R get(const bf16_t* p) { return __uint_as_float(uint32_t(p->bits) << 16); }
    static __device__ __forceinline__ uint16_t round_bf16(float v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);  // quiet NaN
        u += 0x7fffu + ((u >> 16) & 1u);
        return uint16_t(u >> 16);
    }
    static __device__ __forceinline__ void put(bf16_t* p, R v) { p->bits = round_bf16(v); }
    static __device__ __forceinline__ void put_d(bf16_t* p, double v) { p->bits = round_bf16(float(v)); }
};

// Periodic wrap of a coordinate v in [-3, n + 2] onto [0, n).
__device__ __forceinline__ int wrap_coord(int v, int n)
{
    if (n >= 3) {
        v += (v < 0) ? n : 0;
        v -= (v >= n) ? n : 0;
        return v;
    }
    v %= n;
    return v < 0 ? v + n : v;
}

// ---------------------------------------------------------------------------
// Fused step, single box.  One block covers `blockDim.x` sites of one x-row,
// so y and z (and every y/z neighbour offset) are block-uniform scalars; only
// the x wrap is per lane.
// ---------------------------------------------------------------------------

template <class L, class S, int K>
__global__ __launch_bounds__(256) void k_step(const S* __restrict__ src, S* __restrict__ dst, StepGeom geo,
                                              typename Store<S>::R omega)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    const int bid = blockIdx.x;
    const int row = bid / geo.xblocks;
    const int xb = bid - row * geo.xblocks;
    const int y = row % geo.ny;
    const int z = row / geo.ny;
    const int x = xb * int(blockDim.x) + int(threadIdx.x);
    if (x >= geo.nx) return;

    int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * RR; ++k) {
        xw[k] = wrap_coord(x + k - RR, geo.nx);
        yw[k] = wrap_coord(y + k - RR, geo.ny);
        zw[k] = wrap_coord(z + k - RR, geo.nz);
    }

    R g[L::Q];
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const long long rowoff = (long long)i * geo.plane +
                                 ((long long)zw[RR - cz] * geo.ny + yw[RR - cy]) * (long long)geo.nx;
        g[i] = ST::get(src + rowoff + xw[RR - cx]);
    });

    collide_site<L, K, PROJ, R>(g, omega);

    const long long site = ((long long)z * geo.ny + y) * (long long)geo.nx + x;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        ST::put(dst + (long long)i * geo.plane + site, g[i]);
    });
}

// ---------------------------------------------------------------------------
// Fused step, batch of boxes.  A tile is up to blockDim.x consecutive sites
// of one box; a fixed grid walks the tile table (grid-stride), so one launch
// advances every box by one step.  Each box carries its own tau.
// ---------------------------------------------------------------------------

template <class L, class S, int K>
__global__ __launch_bounds__(256) void k_step_batch(const S* __restrict__ src, S* __restrict__ dst,
                                                    const TileDesc* __restrict__ tiles, int ntiles,
                                                    const BoxDesc* __restrict__ boxes, long long plane)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileDesc td = tiles[t];
        const BoxDesc b = boxes[td.box];
        const int local = td.start + int(threadIdx.x);
        const int nxy = b.nx * b.ny;
        if (local >= nxy * b.nz) continue;
        const int z = local / nxy;
        const int rem = local - z * nxy;
        const int y = rem / b.nx;
        const int x = rem - y * b.nx;

        int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
        for (int k = 0; k <= 2 * RR; ++k) {
            xw[k] = wrap_coord(x + k - RR, b.nx);
            yw[k] = wrap_coord(y + k - RR, b.ny);
            zw[k] = wrap_coord(z + k - RR, b.nz);
        }
        R g[L::Q];
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            const int s = (zw[RR - cz] * b.ny + yw[RR - cy]) * b.nx + xw[RR - cx];
            g[i] = ST::get(src + (long long)i * plane + b.offset + s);
        });

        collide_site<L, K, PROJ, R>(g, R(b.omega));

        const long long site = b.offset + local;
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            ST::put(dst + (long long)i * plane + site, g[i]);
        });
    }
}

// ---------------------------------------------------------------------------
// Initialisation: f := f^eq_K(rho, u) (eq. hermite), evaluated in double and
// rounded once to the storage type (set-up, not part of the step).
// ---------------------------------------------------------------------------

template <class L, class S, int K>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ rho, const double* __restrict__ u,
                                              S* __restrict__ dst, long long nsites, long long plane)
{
    using ST = Store<S>;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < nsites;
         s += (long long)gridDim.x * blockDim.x) {
        const double ux = u[s];
        const double uy = u[nsites + s];
        const double uz = (L::D == 3) ? u[2 * nsites + s] : 0.0;
        double g[L::Q];
        equilibrium_scaled<L, K, double>(rho[s] - 1.0, ux, uy, uz, g);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            ST::put_d(dst + (long long)i * plane + s, g[i]);
        });
    }
}

// ---------------------------------------------------------------------------
// Moments rho, u (eq. mme) of the stored state, in double (outside the step,
// for output and reductions).
// ---------------------------------------------------------------------------

template <class L, class S>
__device__ __forceinline__ void site_moments(const S* __restrict__ src, long long s, long long plane,
                                             double& dsum, double (&j)[3])
{
    using ST = Store<S>;
    dsum = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const double gi = double(ST::get(src + (long long)i * plane + s));
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

template <class L, class S>
__global__ __launch_bounds__(256) void k_moments(const S* __restrict__ src, double* __restrict__ rho,
                                                 double* __restrict__ u, long long nsites, long long plane)
{
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < nsites;
         s += (long long)gridDim.x * blockDim.x) {
        double d, j[3];
        site_moments<L, S>(src, s, plane, d, j);
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

template <class L, class S>
__global__ __launch_bounds__(kRedBlock) void k_totals_partial(const S* __restrict__ src,
                                                              const ChunkDesc* __restrict__ chunks,
                                                              long long plane, double* __restrict__ partial)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < ch.count; k += kRedBlock) {
        double d, j[3];
        site_moments<L, S>(src, ch.start + k, plane, d, j);
        acc[0] += d;
        acc[1] += j[0];
        acc[2] += j[1];
        acc[3] += j[2];
    }
    const bool is_max[4] = {false, false, false, false};
    block_tree<4>(acc, is_max);
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 4 + 0] = double(ch.count) + acc[0];  // sum rho = sites + sum g
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

template <class L, class S>
__global__ __launch_bounds__(kRedBlock) void k_residual_partial(const S* __restrict__ src,
                                                                const double* __restrict__ rho_ref,
                                                                const double* __restrict__ u_ref,
                                                                const ChunkDesc* __restrict__ chunks,
                                                                long long nsites, long long plane,
                                                                double* __restrict__ partial)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // max |du|, sum du^2, max |drho|, sum drho^2
    for (int k = threadIdx.x; k < ch.count; k += kRedBlock) {
        const long long s = ch.start + k;
        double d, j[3];
        site_moments<L, S>(src, s, plane, d, j);
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

__global__ __launch_bounds__(kRedBlock) void k_residual_final(const double* __restrict__ partial, int nchunks,
                                                              double* __restrict__ out)
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
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = acc[k];
}

// ---------------------------------------------------------------------------
// Plain 16-byte-vector copy, grid-stride.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// Dispatch from runtime (lattice, dtype, K) to template instances.
// ---------------------------------------------------------------------------

template <class L, class S, class F>
static hipError_t by_k(int K, F&& f)
{
    switch (K) {
    case 2: return f(L{}, (S*)nullptr, std::integral_constant<int, 2>{});
    case 3: return f(L{}, (S*)nullptr, std::integral_constant<int, 3>{});
    case 4:
        if constexpr (L::K_MAX >= 4) return f(L{}, (S*)nullptr, std::integral_constant<int, 4>{});
        break;
    case 5:
        if constexpr (L::K_MAX >= 5) return f(L{}, (S*)nullptr, std::integral_constant<int, 5>{});
        break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <class L, class F>
static hipError_t by_dtype(int dtype, int K, F&& f)
{
    switch (dtype) {
    case 0: return by_k<L, double>(K, f);
    case 1: return by_k<L, float>(K, f);
    case 2: return by_k<L, _Float16>(K, f);
    case 3: return by_k<L, bf16_t>(K, f);
    default: return hipErrorInvalidValue;
    }
}

template <class F>
static hipError_t dispatch(int lat, int dtype, int K, F&& f)
{
    switch (lat) {
    case kD2Q9: return by_dtype<D2Q9>(dtype, K, f);
    case kD3Q19: return by_dtype<D3Q19>(dtype, K, f);
    case kD3Q39: return by_dtype<D3Q39>(dtype, K, f);
    default: return hipErrorInvalidValue;
    }
}

// (lattice, dtype) only: K fixed to 2, ignored by the callee.
template <class F>
static hipError_t dispatch_ld(int lat, int dtype, F&& f)
{
    return dispatch(lat, dtype, 2, f);
}

static int grid_for(long long n, int block)
{
    long long g = (n + block - 1) / block;
    const long long cap = 256LL * 64;  // enough blocks to fill 256 CUs many times over
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return int(g);
}

hipError_t launch_init(int lat, int dtype, int K, const double* rho, const double* u, void* dst,
                       long long nsites, long long plane, hipStream_t s)
{
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        constexpr int KK = decltype(Kc)::value;
        k_init<L, S, KK><<<grid_for(nsites, 256), 256, 0, s>>>(rho, u, static_cast<S*>(dst), nsites, plane);
        return hipGetLastError();
    });
}

hipError_t launch_step(int lat, int dtype, int K, const void* src, void* dst, const StepGeom& geo, double omega,
                       int block, hipStream_t s)
{
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        const long long nblocks = (long long)geo.xblocks * geo.ny * geo.nz;
        k_step<L, S, KK><<<dim3((unsigned)nblocks), block, 0, s>>>(static_cast<const S*>(src), static_cast<S*>(dst),
                                                                   geo, R(omega));
        return hipGetLastError();
    });
}

hipError_t launch_step_batch(int lat, int dtype, int K, const void* src, void* dst, const TileDesc* tiles,
                             int ntiles, const BoxDesc* boxes, long long plane, int block, int grid,
                             hipStream_t s)
{
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        constexpr int KK = decltype(Kc)::value;
        const int g = (grid > 0 && grid < ntiles) ? grid : ntiles;
        k_step_batch<L, S, KK><<<g, block, 0, s>>>(static_cast<const S*>(src), static_cast<S*>(dst), tiles, ntiles,
                                                   boxes, plane);
        return hipGetLastError();
    });
}

hipError_t launch_moments(int lat, int dtype, const void* src, double* rho, double* u, long long nsites,
                          long long plane, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        k_moments<L, S><<<grid_for(nsites, 256), 256, 0, s>>>(static_cast<const S*>(src), rho, u, nsites, plane);
        return hipGetLastError();
    });
}

hipError_t launch_totals(int lat, int dtype, const void* src, const ChunkDesc* chunks, int nchunks,
                         const int* box_chunk_begin, int nbox, long long plane, double* partial, double* out,
                         hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        k_totals_partial<L, S><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), chunks, plane, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_totals_final<<<nbox, kRedBlock, 0, s>>>(partial, box_chunk_begin, out);
        return hipGetLastError();
    });
}

hipError_t launch_residual(int lat, int dtype, const void* src, const double* rho_ref, const double* u_ref,
                           const ChunkDesc* chunks, int nchunks, long long nsites, long long plane,
                           double* partial, double* out, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        k_residual_partial<L, S><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), rho_ref, u_ref, chunks,
                                                               nsites, plane, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_residual_final<<<1, kRedBlock, 0, s>>>(partial, nchunks, out);
        return hipGetLastError();
    });
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    long long g = (long long)((n + 255) / 256);
    if (g > 256LL * 32) g = 256LL * 32;
    if (g < 1) g = 1;
    k_copy<<<int(g), 256, 0, s>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
    return hipGetLastError();
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
    for (int i = 0; i < L::Q; ++i) {
        for (int a = 0; a < 3; ++a) out->c[i * 3 + a] = L::c[i][a];
        out->w[i] = L::w[i];
    }
}

bool lattice_info(int lat, LatticeInfo* out)
{
    switch (lat) {
    case kD2Q9: fill_info<D2Q9>(out); return true;
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
