// Device helpers shared by the gfx950 kernels (wave64, MFMA 16x16).
#pragma once

#include <cfloat>
#include <cmath>

#include "internal.h"

namespace svdphat {

template <typename T>
struct Vec;
template <>
struct Vec<float> {
    typedef float t;   // one operand element per lane (16x16x4 f32)
    typedef float2 pair;
};
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 bh2 __attribute__((ext_vector_type(2)));
template <>
struct Vec<_Float16> {
    typedef h8 t;      // eight operand elements per lane (16x16x32 f16)
    typedef h2 pair;
};
template <>
struct Vec<__bf16> {
    typedef b8 t;      // eight operand elements per lane (16x16x32 bf16)
    typedef bh2 pair;
};

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(h8 a, h8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(b8 a, b8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ T cvt(float v) {
    return (T)v;
}
template <typename T>
__device__ __forceinline__ typename Vec<T>::pair mkpair(T a, T b) {
    typename Vec<T>::pair r;
    r.x = a;
    r.y = b;
    return r;
}

// Unit-modulus normalisation of one STFT coefficient (the per-microphone
// factor of eq. (3): |X_i X_j^*| = |X_i| |X_j|).  Bins whose |X|^2 is not a
// finite normal float (silent, or non-finite input) are treated as silent and
// give 0, so every product they enter is 0.
__device__ __forceinline__ void unit(float& re, float& im) {
    const float m2 = re * re + im * im;
    const bool ok = m2 >= FLT_MIN && m2 <= FLT_MAX;
    const float s = ok ? rsqrtf(m2) : 0.f;
    re = ok ? re * s : 0.f;
    im = ok ? im * s : 0.f;
}

// Orders one wave's LDS traffic (LDS serves a wave's operations in issue
// order; the fences keep the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// (value desc, index asc) order used for every argmax: ties go to the
// lowest index.
__device__ __forceinline__ bool better(float a, int ia, float b, int ib) {
    return a > b || (a == b && ia < ib);
}

}  // namespace svdphat
