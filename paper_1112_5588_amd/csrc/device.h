// Device helpers shared by the HIP kernels of libpjds (gfx950: 64-lane wavefronts, 8 XCDs).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace pjds {

// Values and column indices are read once per product: non-temporal loads.
template <class T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }

// Rows are sorted by length, longest first, inside windows that hold whole waves, so lane 0
// of a wave holds the wave's longest row: its length bounds the wave's loop and its slot is
// the one lanes past their own row re-read.  Both are wave-uniform values.
__device__ __forceinline__ int wave_first(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t wave_first(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// A value (or VPL-wide vector V) from LDS when its staged row d is below n, else from global
// memory at x + xoff.  The LDS row holds `stride` vectors, the first at `staged`.  The two
// loads are separate instructions -- a ds_read for the staged lanes and an exec-masked global
// load for the others -- so no generic (flat) load serves both; the LDS index is clamped to
// row 0 for lanes that do not use it.
template <class V, class T>
__device__ __forceinline__ V staged_or_global(const T *staged, uint32_t d, uint32_t n, uint32_t stride,
                                              const T *x, int64_t xoff) {
    typedef __attribute__((address_space(3))) const V LdsV;
    const bool in = d < n;
    V v = ((const LdsV *)(staged))[(in ? d : 0u) * stride];
    if (!in) v = *reinterpret_cast<const V *>(x + xoff);
    return v;
}

// VPL adjacent values as one vector: one wide load or store.
template <class T, int VPL>
struct VecOf;
template <class T>
struct VecOf<T, 1> { typedef T type; };
template <>
struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <>
struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <>
struct VecOf<double, 4> { typedef double type __attribute__((ext_vector_type(4))); };
template <>
struct VecOf<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };

// The hardware hands workgroup b to XCD b % 8, each XCD with its own L2.  Staged products hand
// their row tiles out in runs of kXcdGroup consecutive tiles per XCD: neighbouring tiles, whose
// staged ranges overlap by the halo, then share one L2, while all eight XCDs still stream
// nearby parts of the matrix (whole contiguous ranges per XCD spread the streams too far
// apart).  The blocks of an incomplete last round keep their own number.  A bijection on
// [0, grid).
constexpr uint32_t kXcds = 8;
constexpr uint32_t kXcdGroup = 16;

__device__ __forceinline__ uint32_t xcd_group(uint32_t b, uint32_t grid) {
    const uint32_t x = b % kXcds, k = b / kXcds;
    if (k / kXcdGroup >= grid / (kXcds * kXcdGroup)) return b;
    return (k / kXcdGroup) * (kXcds * kXcdGroup) + x * kXcdGroup + k % kXcdGroup;
}

}  // namespace pjds
