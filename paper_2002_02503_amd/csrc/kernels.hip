// HIP kernels for gfx950 (MI355X): the fused pull-stream + collide step
// (single box, one site per thread or row-wave; batches of boxes),
// initialisation, moments, FP64 reductions and a copy kernel used to
// calibrate bandwidth measurements.
//
// Data layout: row-tiled structure of arrays (see internal.hpp).  Two buffers
// alternate: a step reads one and writes the other, so a step never reads what
// it writes.  The stored value is G_i = S (f_i - w_i), the deviation from the
// rest weights in units of the lattice's weight quantum 1/S.
//
// The step is bandwidth bound (about 400 single-precision operations against
// 2 Q S bytes per site, far below the FP32 ridge of the chip), so it uses no
// matrix cores: every population is read once (pull form of eq. lbe, periodic
// wrap) and written once, and the collision runs entirely in registers.
#include <type_traits>

#include "collide.hpp"
#include "internal.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Storage types.  FP16 and BF16 are converted with round-to-nearest-even,
// keeping subnormals.
// ---------------------------------------------------------------------------

// The FP32 value v, materialised in a register.  A narrowing store rounds the
// finished FP32 result: without this the compiler may fold the last
// multiply-add into the conversion (a mixed-precision FMA that rounds the exact
// product-sum once to 16 bits), in some kernels and not in others, and the
// step forms would then disagree in the last bit of the stored value.
__device__ __forceinline__ float rounded_f32(float v)
{
    asm("" : "+v"(v));
    return v;
}

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
    static __device__ __forceinline__ void put_nt(double* p, R v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ void put_d(double* p, double v) { *p = v; }
};

template <>
struct Store<float> {
    using R = float;
    static __device__ __forceinline__ R get(const float* p) { return *p; }
    static __device__ __forceinline__ void put(float* p, R v) { *p = v; }
    static __device__ __forceinline__ void put_nt(float* p, R v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ void put_d(float* p, double v) { *p = float(v); }
};

template <>
struct Store<_Float16> {
    using R = float;
    static __device__ __forceinline__ R get(const _Float16* p) { return float(*p); }
    static __device__ __forceinline__ void put(_Float16* p, R v) { *p = _Float16(rounded_f32(v)); }
    static __device__ __forceinline__ void put_nt(_Float16* p, R v)
    {
        __builtin_nontemporal_store(_Float16(rounded_f32(v)), p);
    }
    static __device__ __forceinline__ void put_d(_Float16* p, double v) { *p = _Float16(v); }
};

template <>
struct Store<bf16_t> {
    using R = float;
    static __device__ __forceinline__ R get(const bf16_t* p) { return __uint_as_float(uint32_t(p->bits) << 16); }
    // round to nearest even (gfx950 converts in one instruction)
    static __device__ __forceinline__ uint16_t round_bf16(float v)
    {
        return __builtin_bit_cast(uint16_t, static_cast<__bf16>(rounded_f32(v)));
    }
    static __device__ __forceinline__ void put(bf16_t* p, R v) { p->bits = round_bf16(v); }
    static __device__ __forceinline__ void put_nt(bf16_t* p, R v)
    {
        __builtin_nontemporal_store(round_bf16(v), reinterpret_cast<uint16_t*>(p));
    }
    static __device__ __forceinline__ void put_d(bf16_t* p, double v) { p->bits = round_bf16(float(v)); }
};

// p + i for a uniform pointer p and a 32-bit element index i, with the byte
// offset formed in 32 bits, so the access is a scalar base plus a 32-bit
// vector offset.  Callers keep i * sizeof(T) below 4 GiB.
template <class T>
__device__ __forceinline__ T* at32(T* p, unsigned i)
{
    using B = std::conditional_t<std::is_const<T>::value, const char, char>;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(p) + unsigned(i * unsigned(sizeof(T))));
}

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
// Fused step, single box, one site per thread.  The grid is (x-blocks, ny,
// nz): a block covers blockDim.x sites of one x-row, so y, z and the source
// row of every population are block-uniform; only the x wrap is per lane.
// Every access is a uniform 64-bit pointer (row tile + population row) plus a
// 32-bit lane offset.
// ---------------------------------------------------------------------------

template <class L, class S, int K>
__global__ __launch_bounds__(256) void k_step(const S* __restrict__ src, S* __restrict__ dst, StepGeom geo,
                                              typename Store<S>::R omega)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    const int y = blockIdx.y;
    const int z = blockIdx.z;
    const int x = int(blockIdx.x) * int(blockDim.x) + int(threadIdx.x);
    if (x >= geo.nx) return;
    const long long tile = (long long)L::Q * geo.nx;  // elements per row tile

    int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * RR; ++k) {
        xw[k] = wrap_coord(x + k - RR, geo.nx);
        yw[k] = wrap_coord(y + k - RR, geo.ny);
        zw[k] = wrap_coord(z + k - RR, geo.nz);
    }

    R g[L::Q];
    unroll<L::Q>([&](auto M) {  // in tile-row order
        constexpr int m = decltype(M)::value;
        constexpr int i = mem_pop<L>(m);
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const int row = zw[RR - cz] * geo.ny + yw[RR - cy];
        const S* p = src + row * tile + (long long)m * geo.nx;
        g[i] = ST::get(at32(p, unsigned(xw[RR - cx])));
    });

    collide_site<L, K, PROJ, R>(g, omega);

    S* q = dst + (long long)(z * geo.ny + y) * tile;
    unroll<L::Q>([&](auto M) {
        constexpr int m = decltype(M)::value;
        ST::put_nt(at32(q + (long long)m * geo.nx, unsigned(x)), g[mem_pop<L>(m)]);
    });
}

// ---------------------------------------------------------------------------
// Fused step, single box, row-wave form.  Each wavefront owns whole x-rows;
// each lane owns V consecutive sites of a row and moves them with one aligned
// 8- or 16-byte access per population.  A population shifted along x by
// c_x = +-1..3 (< V) needs V - |c_x| of its values from the lane itself and
// |c_x| from the neighbouring lane of the same row (periodic within the row),
// exchanged with a cross-lane shuffle instead of a second, misaligned load.
// ---------------------------------------------------------------------------

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <class S, int V>
struct VecIO;

// V floats in 16 bytes
template <>
struct VecIO<float, 4> {
    using VT = u32x4;
    static __device__ __forceinline__ void unpack(VT w, float (&o)[4])
    {
        o[0] = __uint_as_float(w.x);
        o[1] = __uint_as_float(w.y);
        o[2] = __uint_as_float(w.z);
        o[3] = __uint_as_float(w.w);
    }
    static __device__ __forceinline__ VT pack(const float (&v)[4])
    {
        VT w;
        w.x = __float_as_uint(v[0]);
        w.y = __float_as_uint(v[1]);
        w.z = __float_as_uint(v[2]);
        w.w = __float_as_uint(v[3]);
        return w;
    }
};

// V doubles in 16 bytes
template <>
struct VecIO<double, 2> {
    using VT = u32x4;
    static __device__ __forceinline__ void unpack(VT w, double (&o)[2])
    {
        o[0] = __hiloint2double(int(w.y), int(w.x));
        o[1] = __hiloint2double(int(w.w), int(w.z));
    }
    static __device__ __forceinline__ VT pack(const double (&v)[2])
    {
        VT w;
        w.x = uint32_t(__double2loint(v[0]));
        w.y = uint32_t(__double2hiint(v[0]));
        w.z = uint32_t(__double2loint(v[1]));
        w.w = uint32_t(__double2hiint(v[1]));
        return w;
    }
};

// four 16-bit values in 8 bytes, FP16 or BF16
template <class H>
struct VecIO16 {
    using VT = u32x2;
    static __device__ __forceinline__ float half_to_float(uint32_t bits16)
    {
        if constexpr (std::is_same<H, bf16_t>::value) {
            return __uint_as_float(bits16 << 16);
        } else {
            const uint16_t b = uint16_t(bits16);
            return float(__builtin_bit_cast(_Float16, b));
        }
    }
    static __device__ __forceinline__ uint32_t float_to_half(float v)
    {
        if constexpr (std::is_same<H, bf16_t>::value) {
            return Store<bf16_t>::round_bf16(v);
        } else {
            return uint32_t(__builtin_bit_cast(uint16_t, _Float16(rounded_f32(v))));
        }
    }
    static __device__ __forceinline__ void unpack(VT w, float (&o)[4])
    {
        o[0] = half_to_float(w.x & 0xffffu);
        o[1] = half_to_float(w.x >> 16);
        o[2] = half_to_float(w.y & 0xffffu);
        o[3] = half_to_float(w.y >> 16);
    }
    static __device__ __forceinline__ VT pack(const float (&v)[4])
    {
        VT w;
        w.x = float_to_half(v[0]) | (float_to_half(v[1]) << 16);
        w.y = float_to_half(v[2]) | (float_to_half(v[3]) << 16);
        return w;
    }
};
template <>
struct VecIO<_Float16, 4> : VecIO16<_Float16> {};
template <>
struct VecIO<bf16_t, 4> : VecIO16<bf16_t> {};

// Sites per lane of the row-wave kernel for each storage type.
template <class S>
constexpr int vec_sites()
{
    return std::is_same<S, double>::value ? 2 : 4;
}

template <class L, class S, int K>
__global__ __launch_bounds__(256) void k_step_vec(const S* __restrict__ src, S* __restrict__ dst, VecGeom geo,
                                                  typename Store<S>::R omega)
{
    using R = typename Store<S>::R;
    constexpr int V = vec_sites<S>();
    using IO = VecIO<S, V>;
    using VT = typename IO::VT;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;
    static_assert(RR < V, "a shifted population must come from at most one neighbouring lane");

    const int lane = int(threadIdx.x) & 63;
    const int wave = int(blockIdx.x) * (int(blockDim.x) >> 6) + (int(threadIdx.x) >> 6);
    const int lpr = geo.lanes_per_row;
    const int r = lane / lpr;          // row within the wave
    const int li = lane - r * lpr;     // lane within the row
    const int row = wave * geo.rows_per_wave + r;
    // Lanes past the last row of the wave, or past the last row of the box,
    // leave now; every lane that stays only reads lanes of its own row.
    if (r >= geo.rows_per_wave || row >= geo.nrows) return;
    const int prev = r * lpr + (li == 0 ? lpr - 1 : li - 1);
    const int next = r * lpr + (li == lpr - 1 ? 0 : li + 1);
    const int y = row % geo.ny;
    const int z = row / geo.ny;
    const long long tile = (long long)L::Q * geo.nx;
    int yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
    for (int k = 0; k <= 2 * RR; ++k) {
        yw[k] = wrap_coord(y + k - RR, geo.ny);
        zw[k] = wrap_coord(z + k - RR, geo.nz);
    }

    R g[V][L::Q];
    unroll<L::Q>([&](auto M) {  // in tile-row order
        constexpr int m = decltype(M)::value;
        constexpr int i = mem_pop<L>(m);
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const long long srow = zw[RR - cz] * geo.ny + yw[RR - cy];
        const S* p = src + srow * tile + (long long)m * geo.nx;
        R own[V];
        IO::unpack(*reinterpret_cast<const VT*>(p + (long long)li * V), own);
        // site j pulls from x_j - c_x: element j - c_x of this lane when it is
        // in [0, V), otherwise the wrapped element of the neighbouring lane
        unroll<V>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr int e = j - cx;
            if constexpr (e >= 0 && e < V) {
                g[j][i] = own[e];
            } else if constexpr (e < 0) {
                g[j][i] = __shfl(own[e + V], prev, 64);
            } else {
                g[j][i] = __shfl(own[e - V], next, 64);
            }
        });
    });

    unroll<V>([&](auto J) {
        constexpr int j = decltype(J)::value;
        collide_site<L, K, PROJ, R>(g[j], omega);
    });

    S* q = dst + (long long)row * tile + (long long)li * V;
    unroll<L::Q>([&](auto M) {
        constexpr int m = decltype(M)::value;
        constexpr int i = mem_pop<L>(m);
        R v[V];
        unroll<V>([&](auto J) {
            constexpr int j = decltype(J)::value;
            v[j] = g[j][i];
        });
        __builtin_nontemporal_store(IO::pack(v), reinterpret_cast<VT*>(q + (long long)m * geo.nx));
    });
}

// ---------------------------------------------------------------------------
// Fused step, batch of boxes.  A tile is a run of whole x-rows of one z-plane
// of one box (or a block-wide piece of one row when nx exceeds the block), so
// z and the box are uniform and each lane finds its row with one exact
// reciprocal multiply.  A fixed grid walks the tile table (grid-stride): one
// launch advances every box by one step, each with its own tau.  Offsets
// inside a box fit 32 bits (checked on the host).
// ---------------------------------------------------------------------------

template <class L, class S, int K>
__global__ __launch_bounds__(256) void k_step_batch(const S* __restrict__ src, S* __restrict__ dst,
                                                    const TileDesc* __restrict__ tiles, int ntiles,
                                                    const BoxDesc* __restrict__ boxes)
{
    using ST = Store<S>;
    using R = typename ST::R;
    constexpr bool PROJ = !std::is_same<R, double>::value;
    constexpr int RR = L::R;

    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileDesc td = tiles[t];
        const BoxDesc b = boxes[td.box];
        const int tid = int(threadIdx.x);
        int r, x;
        if (b.nx <= int(blockDim.x)) {
            // (tid + 1/2) / nx is at least 1/(2 nx) away from an integer, far
            // more than the float rounding of the product: the floor is exact
            r = int((float(tid) + 0.5f) * b.inv_nx);
            x = tid - r * b.nx;
        } else {
            r = 0;
            x = td.x0 + tid;
        }
        if (r >= td.rows || x >= b.nx) continue;
        const int y = td.y0 + r;
        const int z = td.z;
        const S* sb = src + (long long)L::Q * b.offset;
        S* db = dst + (long long)L::Q * b.offset;

        int xw[2 * RR + 1], yw[2 * RR + 1], zw[2 * RR + 1];
#pragma unroll
        for (int k = 0; k <= 2 * RR; ++k) {
            xw[k] = wrap_coord(x + k - RR, b.nx);
            yw[k] = wrap_coord(y + k - RR, b.ny);
            zw[k] = wrap_coord(z + k - RR, b.nz);
        }
        // element offset of a row tile = plane part (uniform) + row part (per lane)
        const int tq = L::Q * b.nx;
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
            g[i] = ST::get(at32(sb, unsigned(off)));
        });

        collide_site<L, K, PROJ, R>(g, R(b.omega));

        const int out_off = (z * b.ny + y) * tq + x;
        unroll<L::Q>([&](auto M) {
            constexpr int m = decltype(M)::value;
            ST::put_nt(at32(db, unsigned(out_off + m * b.nx)), g[mem_pop<L>(m)]);
        });
    }
}

// ---------------------------------------------------------------------------
// Set-up, moments and reductions work on chunks: runs of consecutive sites
// of one box, one block per chunk.
// ---------------------------------------------------------------------------

// Element index of population 0 of a site, relative to the box's first
// element: row tile r = local / nx, x = local % nx.
__device__ __forceinline__ long long site_elem(long long local, int nx, int Q)
{
    const long long r = local / nx;
    const long long x = local - r * nx;
    return r * Q * nx + x;
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
    S* base = dst + (long long)L::Q * b.offset;
    for (int k = threadIdx.x; k < ch.count; k += blockDim.x) {
        const long long s = ch.start + k;
        const long long e = site_elem(s - b.offset, b.nx, L::Q);
        const double ux = u[s];
        const double uy = u[nsites + s];
        const double uz = (L::D == 3) ? u[2 * nsites + s] : 0.0;
        double g[L::Q];
        equilibrium_scaled<L, K, double>(rho[s] - 1.0, ux, uy, uz, g);
        unroll<L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            ST::put_d(base + e + (long long)mem_row<L>(i) * b.nx, g[i]);
        });
    }
}

// rho - 1 and rho u (eq. mme) of one stored site, in double (outside the
// step, for output and reductions).  `p` points at population 0 of the site.
template <class L, class S>
__device__ __forceinline__ void site_moments(const S* __restrict__ p, int nx, double& dsum, double (&j)[3])
{
    using ST = Store<S>;
    dsum = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    unroll<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const double gi = double(ST::get(p + (long long)mem_row<L>(i) * nx));
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
                                                 double* __restrict__ u, const ChunkDesc* __restrict__ chunks,
                                                 const BoxDesc* __restrict__ boxes, long long nsites)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    const S* base = src + (long long)L::Q * b.offset;
    for (int k = threadIdx.x; k < ch.count; k += blockDim.x) {
        const long long s = ch.start + k;
        double d, j[3];
        site_moments<L, S>(base + site_elem(s - b.offset, b.nx, L::Q), b.nx, d, j);
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
                                                              const BoxDesc* __restrict__ boxes,
                                                              double* __restrict__ partial)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    const S* base = src + (long long)L::Q * b.offset;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < ch.count; k += kRedBlock) {
        double d, j[3];
        site_moments<L, S>(base + site_elem(ch.start + k - b.offset, b.nx, L::Q), b.nx, d, j);
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

template <class L, class S>
__global__ __launch_bounds__(kRedBlock) void k_residual_partial(const S* __restrict__ src,
                                                                const double* __restrict__ rho_ref,
                                                                const double* __restrict__ u_ref,
                                                                const ChunkDesc* __restrict__ chunks,
                                                                const BoxDesc* __restrict__ boxes,
                                                                long long nsites, double* __restrict__ partial)
{
    const ChunkDesc ch = chunks[blockIdx.x];
    const BoxDesc b = boxes[ch.box];
    const S* base = src + (long long)L::Q * b.offset;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // max |du|, sum du^2, max |drho|, sum drho^2
    for (int k = threadIdx.x; k < ch.count; k += kRedBlock) {
        const long long s = ch.start + k;
        double d, j[3];
        site_moments<L, S>(base + site_elem(s - b.offset, b.nx, L::Q), b.nx, d, j);
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
// Plain 16-byte-vector copy with non-temporal accesses, one vector per thread.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
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

hipError_t launch_step(int lat, int dtype, int K, const void* src, void* dst, const StepGeom& geo, double omega,
                       int block, hipStream_t s)
{
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        k_step<L, S, KK><<<dim3(unsigned(geo.xblocks), unsigned(geo.ny), unsigned(geo.nz)), block, 0, s>>>(
            static_cast<const S*>(src), static_cast<S*>(dst), geo, R(omega));
        return hipGetLastError();
    });
}

int vec_sites_per_lane(int lat, int dtype)
{
    int v = 0;
    (void)dispatch(lat, dtype, 2, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        constexpr int V = vec_sites<S>();
        v = (L::R < V) ? V : 0;
        return hipSuccess;
    });
    return v;
}

hipError_t launch_step_vec(int lat, int dtype, int K, const void* src, void* dst, const VecGeom& geo, double omega,
                           hipStream_t s)
{
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        using R = typename Store<S>::R;
        constexpr int KK = decltype(Kc)::value;
        if constexpr (L::R < vec_sites<S>()) {
            const long long waves = (geo.nrows + geo.rows_per_wave - 1) / geo.rows_per_wave;
            const long long nblocks = (waves + 3) / 4;
            k_step_vec<L, S, KK><<<dim3((unsigned)nblocks), 256, 0, s>>>(static_cast<const S*>(src),
                                                                       static_cast<S*>(dst), geo, R(omega));
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

hipError_t launch_step_batch(int lat, int dtype, int K, const void* src, void* dst, const TileDesc* tiles,
                             int ntiles, const BoxDesc* boxes, int block, int grid, hipStream_t s)
{
    return dispatch(lat, dtype, K, [&](auto Lt, auto* Sp, auto Kc) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        constexpr int KK = decltype(Kc)::value;
        const int g = (grid > 0 && grid < ntiles) ? grid : ntiles;
        k_step_batch<L, S, KK><<<g, block, 0, s>>>(static_cast<const S*>(src), static_cast<S*>(dst), tiles, ntiles,
                                                   boxes);
        return hipGetLastError();
    });
}

hipError_t launch_moments(int lat, int dtype, const void* src, double* rho, double* u, const ChunkDesc* chunks,
                          int nchunks, const BoxDesc* boxes, long long nsites, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        k_moments<L, S><<<nchunks, 256, 0, s>>>(static_cast<const S*>(src), rho, u, chunks, boxes, nsites);
        return hipGetLastError();
    });
}

hipError_t launch_totals(int lat, int dtype, const void* src, const ChunkDesc* chunks, int nchunks,
                         const int* box_chunk_begin, int nbox, const BoxDesc* boxes, double* partial, double* out,
                         hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        k_totals_partial<L, S><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), chunks, boxes, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_totals_final<<<nbox, kRedBlock, 0, s>>>(partial, box_chunk_begin, out);
        return hipGetLastError();
    });
}

hipError_t launch_residual(int lat, int dtype, const void* src, const double* rho_ref, const double* u_ref,
                           const ChunkDesc* chunks, int nchunks, const BoxDesc* boxes, long long nsites,
                           double* partial, double* out, hipStream_t s)
{
    return dispatch_ld(lat, dtype, [&](auto Lt, auto* Sp, auto) -> hipError_t {
        using L = decltype(Lt);
        using S = std::remove_pointer_t<decltype(Sp)>;
        k_residual_partial<L, S><<<nchunks, kRedBlock, 0, s>>>(static_cast<const S*>(src), rho_ref, u_ref, chunks,
                                                               boxes, nsites, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_residual_final<<<1, kRedBlock, 0, s>>>(partial, nchunks, out);
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
