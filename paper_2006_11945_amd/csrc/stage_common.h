// Device pieces shared by the stage kernel and the adjoint stage kernel:
// SSP-RK3 coefficients, the upwind-ordered WENO5 helpers, raw buffer
// access, XCD-aware block numbering and the LDS word layout.
#pragma once
#include <hip/hip_runtime.h>

#include "egb_device.h"

namespace egb {

template <int STAGE>
struct RK;
template <>
struct RK<0> {
    static constexpr double ca = 0.0, cb = 1.0;
};
template <>
struct RK<1> {
    static constexpr double ca = 0.75, cb = 0.25;
};
template <>
struct RK<2> {
    static constexpr double ca = 1.0 / 3.0, cb = 2.0 / 3.0;
};

constexpr int TZ = 64;  // z cells per tile (one wavefront row)

// WENO5 of six values u0..u5 read in upwind order (u3 is the cell itself,
// u0..u2 lie on the upwind side): differences u_k - u_{k-1}, formed in T,
// derivative in R.  Reading the stencil mirrored when the velocity component
// is negative turns D+ into minus D- of the mirrored values, so
// V * D(U) = |V| * weno_up(mirrored values) for either sign.
template <typename R, typename T>
__device__ __forceinline__ R weno_up(T u0, T u1, T u2, T u3, T u4, T u5) {
    return weno5<R>((R)(u1 - u0), (R)(u2 - u1), (R)(u3 - u2), (R)(u4 - u3), (R)(u5 - u4));
}

// The fifth-order linear upwind derivative of the same six values: the three
// WENO5 candidate stencils combined with their linear weights (0.1, 0.6,
// 0.3), which in the differences d_k = u_k - u_(k-1) is
//   (2 d1 - 13 d2 + 47 d3 + 27 d4 - 3 d5) / 60.
template <typename R, typename T>
__device__ __forceinline__ R upwind5_up(T u0, T u1, T u2, T u3, T u4, T u5) {
    const R d1 = (R)(u1 - u0), d2 = (R)(u2 - u1), d3 = (R)(u3 - u2), d4 = (R)(u4 - u3), d5 = (R)(u5 - u4);
    return ((R)2 * d1 - (R)13 * d2 + (R)47 * d3 + (R)27 * d4 - (R)3 * d5) * (R)(1.0 / 60.0);
}

// Value m of the upwind-ordered x stencil from the column queue q (q[3] is
// the cell): DIR 0 = every lane upwinds from -x, 1 = every lane from +x,
// 2 = per lane (`minus`).
template <int DIR, typename T>
__device__ __forceinline__ T upw(const T (&q)[7], int m, bool minus) {
    if constexpr (DIR == 0) return q[m];
    else if constexpr (DIR == 1) return q[6 - m];
    else return minus ? q[m] : q[6 - m];
}

// Raw buffer access: one descriptor per array (base, size < 4 GiB), a 32-bit
// per-lane byte offset and the plane offset in the scalar offset register.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          (int)voff, (int)soff, 0);
}

// XCD-aware numbering: hardware block b runs on XCD b % 8; give each XCD a
// contiguous range of logical tiles (a bijection of [0, n)).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q8 = n >> 3, r8 = n & 7, xcd = b & 7;
    return xcd * q8 + min(xcd, r8) + (b >> 3);
}

// LDS slice layout: NP planes of R (as raw words), then psi as two 32-bit
// planes (F32) or one 64-bit plane (F64), so that one cell has the same word
// index in every plane and one per-lane address serves them all (the plane
// is an immediate offset).
template <typename R>
struct LdsWord;
template <>
struct LdsWord<float> {
    using T = unsigned;
    static constexpr int PSI_WORDS = 2;
};
template <>
struct LdsWord<double> {
    using T = unsigned long long;
    static constexpr int PSI_WORDS = 1;
};

// Plane f (or psi) of the cell at byte address `byte` of the slice buffers.
template <typename R, typename S>
__device__ __forceinline__ R lds_r(const S& sm, int byte, int f) {
    const char* c = reinterpret_cast<const char*>(sm.w) + byte + f * S::PB;
    return __builtin_bit_cast(R, *reinterpret_cast<const typename S::W*>(c));
}
template <int NP, typename S>
__device__ __forceinline__ double lds_psi(const S& sm, int byte) {
    const char* c = reinterpret_cast<const char*>(sm.w) + byte + NP * S::PB;
    if constexpr (sizeof(typename S::W) == 4) {
        const unsigned lo = *reinterpret_cast<const unsigned*>(c);
        const unsigned hi = *reinterpret_cast<const unsigned*>(c + S::PB);
        return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(double, *reinterpret_cast<const unsigned long long*>(c));
    }
}

}  // namespace egb
