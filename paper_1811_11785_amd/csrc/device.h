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
    const float m2 = fmaf(re, re, im * im);
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

// Wave-wide reduction of N 32-bit words per lane with a commutative
// combiner comb(v, o) (v := v combined with o), in registers: inside rows of
// 16 lanes the partner comes by DPP (quad permutations xor 1 and xor 2, then
// the half-row and row mirrors, which pair the already combined quads and
// halves); across rows v_permlane16_swap and v_permlane32_swap hand every
// lane both rows' (halves') values.  Every lane ends with the combination
// of all 64 lanes.
// m ? b : a on all 32 bits, by masks (a select between two arrays' words
// can be folded into a select of the arrays' addresses, which puts them in
// scratch memory; the bitwise blend keeps them in registers)
__device__ __forceinline__ uint32_t blend(uint32_t a, uint32_t b, bool m) {
    const uint32_t k = m ? ~0u : 0u;
    return (a & ~k) | (b & k);
}

template <int CTRL, int N>
__device__ __forceinline__ void dpp_words(const uint32_t (&v)[N], uint32_t (&o)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = (uint32_t)__builtin_amdgcn_mov_dpp((int)v[i], CTRL, 0xF, 0xF, false);
}

// the same inside each row of 16 lanes only
template <int N, typename Comb>
__device__ __forceinline__ void row_reduce(uint32_t (&v)[N], Comb comb) {
    uint32_t o[N];
    dpp_words<0xB1>(v, o);  // quad_perm [1, 0, 3, 2]
    comb(v, o);
    dpp_words<0x4E>(v, o);  // quad_perm [2, 3, 0, 1]
    comb(v, o);
    dpp_words<0x141>(v, o);  // row_half_mirror
    comb(v, o);
    dpp_words<0x140>(v, o);  // row_mirror
    comb(v, o);
}

template <int N, typename Comb>
__device__ __forceinline__ void wave_reduce(uint32_t (&v)[N], Comb comb) {
    uint32_t o[N];
    row_reduce(v, comb);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(v[i], v[i], false, false);
        v[i] = r[0];
        o[i] = r[1];
    }
    comb(v, o);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(v[i], v[i], false, false);
        v[i] = r[0];
        o[i] = r[1];
    }
    comb(v, o);
}

__device__ __forceinline__ float wave_max(float v) {
    uint32_t w[1] = {__float_as_uint(v)};
    wave_reduce(w, [](uint32_t (&a)[1], const uint32_t (&b)[1]) {
        a[0] = __float_as_uint(fmaxf(__uint_as_float(a[0]), __uint_as_float(b[0])));
    });
    return __uint_as_float(w[0]);
}
__device__ __forceinline__ float wave_sum(float v) {
    uint32_t w[1] = {__float_as_uint(v)};
    wave_reduce(w, [](uint32_t (&a)[1], const uint32_t (&b)[1]) {
        a[0] = __float_as_uint(__uint_as_float(a[0]) + __uint_as_float(b[0]));
    });
    return __uint_as_float(w[0]);
}

// (value desc, index asc) order used for every argmax: ties go to the
// lowest index.
__device__ __forceinline__ bool better(float a, int ia, float b, int ib) {
    return a > b || (a == b && ia < ib);
}


// Algorithm 1, online step 4: the power of direction q from its row of W,
// Y_q = Re sum_{p,k} exp(2 pi i k tau_p / N) x_{p,k}, for one frame.  With
// far-field delays (eq. (2)) the delay of pair p = (i, j) is tau_j - tau_i,
// so each term is Re(V_i conj(V_j)) with V_m = exp(-2 pi i k tau_m / N)
// X_m / |X_m| (0 for a silent bin: |X_m|^2 not a finite normal float), and
// the sum over the pairs i < j at a bin is (|sum_m V_m|^2 - sum_m |V_m|^2)
// / 2 (the delay-and-sum form of the same sum).  One wave: xf = [M][B] STFT
// values, t[m] = tau_m / N; lanes take bins lane + 64 j of the first
// Bmain = B - tail bins (all STFT loads of a block of 4 x 64 bins issued
// before any is used), and the last `tail` bins (B mod 64 when tail x M <=
// 64, typically the Nyquist bin) one (bin, microphone) per lane.  Returns
// the wave's total.  MK: mk = the frame's mask bytes [B]; a bin it drops
// contributes nothing (as a silent bin).
__device__ __forceinline__ float ds_term(float2 x, bool live, float cr, float ci, float& sre, float& sim) {
    const float m2 = fmaf(x.x, x.x, x.y * x.y);
    const bool ok = live && __builtin_amdgcn_classf(m2, 0x100);
    const float s = __builtin_amdgcn_rsqf(m2);
    const float ur = ok ? x.x * s : 0.f, ui = ok ? x.y * s : 0.f;
    sre = fmaf(ur, cr, fmaf(-ui, ci, sre));
    sim = fmaf(ur, ci, fmaf(ui, cr, sim));
    return ok ? 1.f : 0.f;
}

template <int MAXM, bool MK = false>
__device__ __forceinline__ float power_ds(const float2* __restrict__ xf, int M, int B, const float (&t)[MAXM],
                                          int lane, const uint8_t* __restrict__ mk = nullptr) {
    constexpr int NJ = MAXM <= 8 ? 4 : 1;
    const int tail = ((B % 64) * M <= 64) ? B % 64 : 0;
    const int Bm = B - tail;
    float acc = 0.f;
    for (int b0 = 0; b0 < Bm; b0 += 64 * NJ) {
        float2 v[NJ][MAXM];
        bool kp[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int bin = b0 + lane + 64 * j;
#pragma unroll
            for (int m = 0; m < MAXM; ++m) v[j][m] = xf[(bin < Bm && m < M) ? (int64_t)m * B + bin : 0];
            kp[j] = !MK || mk[bin < Bm ? bin : 0] != 0;
        }
        // phase of the lane's first bin and its step over 64 bins, per mic
        float cr[MAXM], ci[MAXM], sr[MAXM], si[MAXM];
#pragma unroll
        for (int m = 0; m < MAXM; ++m) {
            float p0 = (float)(b0 + lane) * t[m];
            p0 -= rintf(p0);
            float p1 = 64.f * t[m];
            p1 -= rintf(p1);
            cr[m] = __builtin_amdgcn_cosf(p0);  // argument in revolutions
            ci[m] = -__builtin_amdgcn_sinf(p0);
            sr[m] = __builtin_amdgcn_cosf(p1);
            si[m] = -__builtin_amdgcn_sinf(p1);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const bool live = b0 + lane + 64 * j < Bm && kp[j];
            float sre = 0.f, sim = 0.f, cnt = 0.f;
#pragma unroll
            for (int m = 0; m < MAXM; ++m)
                if (m < M) {
                    cnt += ds_term(v[j][m], live, cr[m], ci[m], sre, sim);
                    const float nr = cr[m] * sr[m] - ci[m] * si[m];
                    ci[m] = cr[m] * si[m] + ci[m] * sr[m];
                    cr[m] = nr;
                }
            acc += 0.5f * (fmaf(sre, sre, sim * sim) - cnt);
        }
    }
    float tot = wave_sum(acc);
    // tail bins: lane = (bin - Bm) * M + m
    for (int tb = 0; tb < tail; ++tb) {
        const int bin = Bm + tb;
        const bool mine = lane >= tb * M && lane < (tb + 1) * M;
        const int m = lane - tb * M;
        const float2 x = xf[mine ? (int64_t)m * B + bin : 0];
        const bool kb = !MK || mk[bin] != 0;
        float tm = 0.f;
#pragma unroll
        for (int k = 0; k < MAXM; ++k)
            if (k == m) tm = t[k];
        float p0 = (float)bin * tm;
        p0 -= rintf(p0);
        float sre = 0.f, sim = 0.f;
        const float cnt = ds_term(x, mine && kb, __builtin_amdgcn_cosf(p0), -__builtin_amdgcn_sinf(p0), sre, sim);
        const float sr = wave_sum(sre), sm = wave_sum(sim), c = wave_sum(cnt);
        tot += 0.5f * (fmaf(sr, sr, sm * sm) - c);
    }
    return tot;
}

}  // namespace svdphat
