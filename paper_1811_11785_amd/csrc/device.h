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


// Algorithm 1, online step 4: the power of one direction from its row of W,
// Y = Re sum_{p,k} exp(2 pi i k tau_p / N) x_{p,k}, for one frame (xf =
// [M][B] STFT values, tq = tau_p / N of the direction's pairs).  One wave;
// returns this lane's partial sum (the caller reduces over the wave).
template <int MAXM>
__device__ __forceinline__ float direction_power(const float2* __restrict__ xf, int M, int B,
                                                 const float* __restrict__ tq, int lane) {
    float acc = 0.f;
    if (MAXM <= 8) {
        // each lane takes bins b0 + lane + 64 j, j < NJ; the phase of bin
        // b + 64 follows from that of bin b by one complex multiplication
        constexpr int NJ = 5;
        for (int b0 = 0; b0 < B; b0 += 64 * NJ) {
            float nr[NJ][MAXM], ni[NJ][MAXM];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int m = 0; m < MAXM; ++m) {
                    const int bin = b0 + lane + 64 * j;
                    float2 v = (bin < B && m < M) ? xf[(int64_t)m * B + bin] : float2{0.f, 0.f};
                    nr[j][m] = v.x;
                    ni[j][m] = v.y;
                    unit(nr[j][m], ni[j][m]);
                }
            int p = 0;
#pragma unroll
            for (int i = 0; i < MAXM; ++i)
#pragma unroll
                for (int k = i + 1; k < MAXM; ++k)
                    if (k < M) {
                        const float tn = tq[p];
                        float t0 = (float)(b0 + lane) * tn;
                        t0 -= rintf(t0);
                        float t1 = 64.f * tn;
                        t1 -= rintf(t1);
                        float wr = __builtin_amdgcn_cosf(t0), wi = __builtin_amdgcn_sinf(t0);
                        const float sr = __builtin_amdgcn_cosf(t1), si = __builtin_amdgcn_sinf(t1);
#pragma unroll
                        for (int j = 0; j < NJ; ++j) {
                            const float xr = nr[j][i] * nr[j][k] + ni[j][i] * ni[j][k];
                            const float xi = ni[j][i] * nr[j][k] - nr[j][i] * ni[j][k];
                            acc = fmaf(wr, xr, fmaf(-wi, xi, acc));
                            const float nwr = wr * sr - wi * si;
                            wi = wr * si + wi * sr;
                            wr = nwr;
                        }
                        ++p;
                    }
        }
    } else {
        for (int bin = lane; bin < B; bin += 64) {
            float re[MAXM], im[MAXM];
#pragma unroll
            for (int m = 0; m < MAXM; ++m) {
                const float2 v = m < M ? xf[(int64_t)m * B + bin] : float2{0.f, 0.f};
                re[m] = v.x;
                im[m] = v.y;
                unit(re[m], im[m]);
            }
            int p = 0;
#pragma unroll
            for (int i = 0; i < MAXM; ++i)
#pragma unroll
                for (int k = i + 1; k < MAXM; ++k)
                    if (k < M) {
                        const float xr = re[i] * re[k] + im[i] * im[k];
                        const float xi = im[i] * re[k] - re[i] * im[k];
                        float t = (float)bin * tq[p];
                        t -= rintf(t);
                        acc = fmaf(__builtin_amdgcn_cosf(t), xr, fmaf(-__builtin_amdgcn_sinf(t), xi, acc));
                        ++p;
                    }
        }
    }
    return acc;
}


// The STFT values one lane needs for direction_power, loaded early (before
// the direction is known) so that their latency overlaps other work; used
// when the frame has at most 5 x 64 bins and at most 8 microphones.
template <int MAXM>
struct PowerPrefetch {
    static constexpr bool kRegs = MAXM <= 8;
    static constexpr int NJ = 5;
    float2 v[kRegs ? NJ : 1][kRegs ? MAXM : 1];
    bool ok = false;
    __device__ __forceinline__ void load(const float2* __restrict__ xf, int M, int B, int lane) {
        if constexpr (kRegs) {
            ok = B <= 64 * NJ;
            if (!ok) return;
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int m = 0; m < MAXM; ++m) {
                    const int bin = lane + 64 * j;
                    v[j][m] = (bin < B && m < M) ? xf[(int64_t)m * B + bin] : float2{0.f, 0.f};
                }
        }
    }
    __device__ __forceinline__ float power(const float2* __restrict__ xf, int M, int B,
                                           const float* __restrict__ tq, int lane) {
        if constexpr (kRegs) {
            if (ok) {
                float nr[NJ][MAXM], ni[NJ][MAXM];
#pragma unroll
                for (int j = 0; j < NJ; ++j)
#pragma unroll
                    for (int m = 0; m < MAXM; ++m) {
                        nr[j][m] = v[j][m].x;
                        ni[j][m] = v[j][m].y;
                        unit(nr[j][m], ni[j][m]);
                    }
                float acc = 0.f;
                int p = 0;
#pragma unroll
                for (int i = 0; i < MAXM; ++i)
#pragma unroll
                    for (int k = i + 1; k < MAXM; ++k)
                        if (k < M) {
                            const float tn = tq[p];
                            float t0 = (float)lane * tn;
                            t0 -= rintf(t0);
                            float t1 = 64.f * tn;
                            t1 -= rintf(t1);
                            float wr = __builtin_amdgcn_cosf(t0), wi = __builtin_amdgcn_sinf(t0);
                            const float sr = __builtin_amdgcn_cosf(t1), si = __builtin_amdgcn_sinf(t1);
#pragma unroll
                            for (int j = 0; j < NJ; ++j) {
                                const float xr = nr[j][i] * nr[j][k] + ni[j][i] * ni[j][k];
                                const float xi = ni[j][i] * nr[j][k] - nr[j][i] * ni[j][k];
                                acc = fmaf(wr, xr, fmaf(-wi, xi, acc));
                                const float nwr = wr * sr - wi * si;
                                wi = wr * si + wi * sr;
                                wr = nwr;
                            }
                            ++p;
                        }
                return acc;
            }
        }
        return direction_power<MAXM>(xf, M, B, tq, lane);
    }
};

}  // namespace svdphat
