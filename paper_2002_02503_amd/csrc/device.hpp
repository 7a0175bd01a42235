// Device-side building blocks shared by the kernel translation units:
// storage types and their conversions, addressing helpers, the vector
// accessors of the row-wave step, and the dispatch from a runtime (lattice,
// dtype, K) to template instances.
#pragma once

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
    static __device__ __forceinline__ R get_nt(const double* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void put(double* p, R v) { *p = v; }
    static __device__ __forceinline__ void put_nt(double* p, R v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ void put_d(double* p, double v) { *p = v; }
};

template <>
struct Store<float> {
    using R = float;
    static __device__ __forceinline__ R get(const float* p) { return *p; }
    static __device__ __forceinline__ R get_nt(const float* p) { return __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void put(float* p, R v) { *p = v; }
    static __device__ __forceinline__ void put_nt(float* p, R v) { __builtin_nontemporal_store(v, p); }
    static __device__ __forceinline__ void put_d(float* p, double v) { *p = float(v); }
};

template <>
struct Store<_Float16> {
    using R = float;
    static __device__ __forceinline__ R get(const _Float16* p) { return float(*p); }
    static __device__ __forceinline__ R get_nt(const _Float16* p) { return float(__builtin_nontemporal_load(p)); }
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
    static __device__ __forceinline__ R get_nt(const bf16_t* p)
    {
        return __uint_as_float(uint32_t(__builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p))) << 16);
    }
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

// A population the step pulls.  Rows read at their own x (c_x = 0) are read
// by exactly one wavefront and are loaded non-temporally; x-shifted rows
// share each wavefront's edge cache lines with the neighbouring wavefront and
// keep the default policy.  (Measured on the D3Q19 FP32 step: +4% over plain
// loads, +1% over non-temporal loads everywhere.)
template <class ST, int CX, class S>
__device__ __forceinline__ typename ST::R load_population(const S* p)
{
    if constexpr (CX == 0) return ST::get_nt(p);
    else return ST::get(p);
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

// ---------------------------------------------------------------------------
// Dispatch from runtime (dtype, K, collision kind) to template instances of
// one lattice, and from a runtime lattice to that.  The callee gets
// (L{}, (S*)nullptr, integral_constant K, integral_constant kind).  The
// energy-flux kind exists for K >= 3 only (its Hermite series starts at
// n = 3).
// ---------------------------------------------------------------------------

template <int V>
using ic = std::integral_constant<int, V>;

template <class L, class S, int KK, class F>
hipError_t by_kind(int kind, F&& f)
{
    switch (kind) {
    case kFiltered: return f(L{}, (S*)nullptr, ic<KK>{}, ic<kFiltered>{});
    case kBGK: return f(L{}, (S*)nullptr, ic<KK>{}, ic<kBGK>{});
    case kFilteredQ:
        if constexpr (KK >= 3) return f(L{}, (S*)nullptr, ic<KK>{}, ic<kFilteredQ>{});
        break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <class L, class S, class F>
hipError_t by_k(int K, int kind, F&& f)
{
    switch (K) {
    case 2: return by_kind<L, S, 2>(kind, f);
    case 3: return by_kind<L, S, 3>(kind, f);
    case 4:
        if constexpr (L::K_MAX >= 4) return by_kind<L, S, 4>(kind, f);
        break;
    case 5:
        if constexpr (L::K_MAX >= 5) return by_kind<L, S, 5>(kind, f);
        break;
    default: break;
    }
    return hipErrorInvalidValue;
}

// (K, kind) for a fixed (lattice, storage type).
template <class L, class S, class F>
hipError_t dispatch_pair(int K, int kind, F&& f)
{
    return by_k<L, S>(K, kind, f);
}

template <class L, class F>
hipError_t dispatch_lattice(int dtype, int K, int kind, F&& f)
{
    switch (dtype) {
    case 0: return by_k<L, double>(K, kind, f);
    case 1: return by_k<L, float>(K, kind, f);
    case 2: return by_k<L, _Float16>(K, kind, f);
    case 3: return by_k<L, bf16_t>(K, kind, f);
    default: return hipErrorInvalidValue;
    }
}

template <class F>
hipError_t dispatch_kind(int lat, int dtype, int K, int kind, F&& f)
{
    switch (lat) {
    case kD2Q9: return dispatch_lattice<D2Q9>(dtype, K, kind, f);
    case kD3Q15: return dispatch_lattice<D3Q15>(dtype, K, kind, f);
    case kD3Q19: return dispatch_lattice<D3Q19>(dtype, K, kind, f);
    case kD3Q39: return dispatch_lattice<D3Q39>(dtype, K, kind, f);
    default: return hipErrorInvalidValue;
    }
}

// (lattice, dtype, K) for callees that take (L{}, (S*)nullptr, K constant).
template <class F>
hipError_t dispatch(int lat, int dtype, int K, F&& f)
{
    return dispatch_kind(lat, dtype, K, kFiltered,
                         [&](auto Lt, auto* Sp, auto Kc, auto) -> hipError_t { return f(Lt, Sp, Kc); });
}

// (lattice, dtype) only: K fixed to 2, ignored by the callee.
template <class F>
hipError_t dispatch_ld(int lat, int dtype, F&& f)
{
    return dispatch(lat, dtype, 2, f);
}

}  // namespace lbm
