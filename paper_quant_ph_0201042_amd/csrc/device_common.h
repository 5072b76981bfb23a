// Device-side helpers shared by the gfx950 kernels of this library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sv_internal.h"

namespace svd {

// Amplitude types as clang vector types, so that the nontemporal builtins
// (which need scalar or vector operands) apply to whole 8- or 16-byte
// amplitudes.
typedef double c128 __attribute__((ext_vector_type(2)));
typedef float c64 __attribute__((ext_vector_type(2)));

template <typename T>
struct RealOf;
template <>
struct RealOf<c128> {
    using type = double;
};
template <>
struct RealOf<c64> {
    using type = float;
};

// The state is far larger than every cache (a 30-qubit complex128 register is
// 16 GiB against 256 MB of Infinity Cache), so amplitudes are streamed with
// nontemporal loads and stores; on gfx950 this raised in-place sweeps from
// ~5.4 to ~6.6 TB/s.
template <typename T>
__device__ __forceinline__ T ldnt(const T *p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void stnt(T v, T *p) {
    __builtin_nontemporal_store(v, p);
}

// t with a zero bit inserted at position p.
__device__ __forceinline__ uint64_t insert_zero(uint64_t t, int p) {
    const uint64_t lo = t & ((uint64_t(1) << p) - 1);
    return ((t & ~lo) << 1) | lo;
}

// t with zero bits inserted at every (ascending) position of s.
__device__ __forceinline__ uint64_t insert_zeros(uint64_t t, const BitSpec &s) {
    for (int i = 0; i < s.count; ++i) t = insert_zero(t, s.pos[i]);
    return t;
}

// m[o] * x + m[o+2] * y for complex entries stored as (re, im) pairs.
template <typename T, typename R>
__device__ __forceinline__ T mac2(const R *m, int o, T x, T y) {
    T r;
    r.x = m[o] * x.x - m[o + 1] * x.y + m[o + 2] * y.x - m[o + 3] * y.y;
    r.y = m[o] * x.y + m[o + 1] * x.x + m[o + 2] * y.y + m[o + 3] * y.x;
    return r;
}

template <typename T, typename R>
__device__ __forceinline__ T cscale(R re, R im, T x) {
    T r;
    r.x = re * x.x - im * x.y;
    r.y = re * x.y + im * x.x;
    return r;
}

template <typename T>
__device__ __forceinline__ T shfl_xor_c(T v, int m) {
    T r;
    r.x = __shfl_xor(v.x, m, 64);
    r.y = __shfl_xor(v.y, m, 64);
    return r;
}

}  // namespace svd
