// Online kernels of SVD-PHAT for gfx950 (Algorithm 1, online steps 1-4,
// Section 3) and of plain SRP-PHAT (eqs. (3), (9), (6), Section 2).
//
// SVD-PHAT, per batch of frames:
//   k_gemm1   PHAT cross-spectra (eq. (3)) formed in LDS from the STFT and
//             projected with MFMA: Z = S V^H X (eq. (12), S folded into V^H),
//             stacked real, split over the reduction axis -> partial Z.
//   k_zprep   sums the partial Z, keeps an FP32 copy and its norm, and packs a
//             (scaled) copy in the GEMM2 operand type and fragment order.
//   k_gemm2   Y = Re(U Z) (eqs. (13)-(14)) with MFMA and a max-only epilogue:
//             one maximum per (frame, tile of 64 directions).
//   k_final   per frame: candidate tiles within the rounding bound of the
//             maximum are rescored in FP32, the best class and the margin to
//             the runner-up are taken, and the power of the chosen direction is
//             evaluated from its row of W (Algorithm 1, online step 4).
//   (HILO)    frames with a small margin get Z recomputed with a split hi/lo
//             product and are rescored again.
// SRP-PHAT: k_phat_frag materialises the PHAT vector in FP32, k_srp_gemm
// multiplies by the stored W with FP32 MFMA and an argmax epilogue,
// k_srp_reduce reduces across direction tiles.
#include "internal.h"

#include <cfloat>
#include <cmath>

namespace svdphat {

namespace {

template <typename T>
struct Vec;
template <>
struct Vec<float> {
    typedef float t;
};
template <>
struct Vec<_Float16> {
    typedef h8 t;
};
template <>
struct Vec<__bf16> {
    typedef b8 t;
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

// Unit-modulus normalisation of one STFT coefficient; a silent bin (|X|^2
// below the smallest normal float) gives 0, so its PHAT products are 0.
// Bins whose |X|^2 is not a finite normal float (silent, or non-finite input)
// are treated as silent.
__device__ __forceinline__ void unit(float& re, float& im) {
    const float m2 = re * re + im * im;
    const bool ok = m2 >= FLT_MIN && m2 <= FLT_MAX;
    const float s = ok ? rsqrtf(m2) : 0.f;
    re = ok ? re * s : 0.f;
    im = ok ? im * s : 0.f;
}

// Orders the LDS traffic of one wave (LDS executes a wave's operations in
// issue order; this keeps the compiler from moving them across).
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

// ------------------------------------------------------------------ GEMM1
// One workgroup: NF frames (16 per wave) x up to NRB row blocks of Z, over
// the chunks [split * cps, (split + 1) * cps) of the reduction axis.  For
// each chunk the PHAT vector of BB bins is formed in LDS (eq. (3); per-mic
// unit normalisation, then X_i conj(X_j) for the pairs i < j in order),
// rounded to T, then multiplied by the packed A fragments.
constexpr int NRB_MAX = 12;
constexpr int XPAD = 8;

template <typename T, int NF, int MAXM, bool HILO>
__global__ __launch_bounds__(NF * 4) void k_gemm1(
    const float2* __restrict__ X, int64_t nfr, int M, int P, int B, const int8_t* __restrict__ pi,
    const int8_t* __restrict__ pj, const T* __restrict__ A, const T* __restrict__ Alo, int nRB, int BB, int CW,
    int nch, int cps, float* __restrict__ zpart, int64_t zstride, int Rp, const int* __restrict__ flist,
    const int* __restrict__ fcount) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL;
    typedef typename Vec<T>::t VT;
    constexpr int NT = NF * 4;
    extern __shared__ __align__(16) char smem[];
    T* xs = reinterpret_cast<T*>(smem);
    const int ldx = CW + XPAD;
    T* xl = xs + NF * ldx;

    const int64_t n = flist ? (int64_t)*fcount : nfr;
    const int64_t f0 = (int64_t)blockIdx.x * NF;
    if (f0 >= n) return;
    const int split = blockIdx.y;
    const int c0 = split * cps, c1 = min(nch, c0 + cps);
    const int rbs = blockIdx.z * NRB_MAX;
    const int nrb = min(NRB_MAX, nRB - rbs);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ks_chunk = CW / KS;

    // padding columns of the tile stay zero
    for (int i = threadIdx.x; i < NF * ldx; i += NT) {
        int col = i % ldx;
        if (col >= BB * 2 * P) {
            xs[i] = cvt<T>(0.f);
            if (HILO) xl[i] = cvt<T>(0.f);
        }
    }

    f4 acc[NRB_MAX];
#pragma unroll
    for (int r = 0; r < NRB_MAX; ++r) acc[r] = f4{0.f, 0.f, 0.f, 0.f};

    for (int ch = c0; ch < c1; ++ch) {
        __syncthreads();
        for (int it = threadIdx.x; it < NF * BB; it += NT) {
            const int fl = it / BB, bl = it % BB;
            const int64_t fpos = f0 + fl;
            const int bin = ch * BB + bl;
            T* dst = xs + fl * ldx + bl * 2 * P;
            T* dlo = xl + fl * ldx + bl * 2 * P;
            if (fpos < n && bin < B) {
                const int64_t f = flist ? (int64_t)flist[fpos] : fpos;
                const float2* xf = X + f * M * B + bin;
                float re[MAXM], im[MAXM];
#pragma unroll
                for (int m = 0; m < MAXM; ++m) {
                    float2 v = m < M ? xf[(int64_t)m * B] : float2{0.f, 0.f};
                    re[m] = v.x;
                    im[m] = v.y;
                    unit(re[m], im[m]);
                }
                int p = 0;
#pragma unroll
                for (int i = 0; i < MAXM; ++i)
#pragma unroll
                    for (int j = i + 1; j < MAXM; ++j)
                        if (j < M) {
                            float xr = re[i] * re[j] + im[i] * im[j];
                            float xi = im[i] * re[j] - re[i] * im[j];
                            T hr = cvt<T>(xr), hi = cvt<T>(xi);
                            dst[2 * p] = hr;
                            dst[2 * p + 1] = hi;
                            if (HILO) {
                                dlo[2 * p] = cvt<T>(xr - (float)hr);
                                dlo[2 * p + 1] = cvt<T>(xi - (float)hi);
                            }
                            ++p;
                        }
            } else {
                for (int k = 0; k < 2 * P; ++k) {
                    dst[k] = cvt<T>(0.f);
                    if (HILO) dlo[k] = cvt<T>(0.f);
                }
            }
        }
        __syncthreads();
        const T* Ach = A + (int64_t)ch * ks_chunk * nRB * 64 * EPL;
        const T* Alch = HILO ? Alo + (int64_t)ch * ks_chunk * nRB * 64 * EPL : nullptr;
        const T* brow = xs + (wave * 16 + (lane & 15)) * ldx + EPL * (lane >> 4);
        const T* blrow = xl + (wave * 16 + (lane & 15)) * ldx + EPL * (lane >> 4);
        for (int ks = 0; ks < ks_chunk; ++ks) {
            VT b = *reinterpret_cast<const VT*>(brow + ks * KS);
            VT bl;
            if (HILO) bl = *reinterpret_cast<const VT*>(blrow + ks * KS);
#pragma unroll
            for (int r = 0; r < NRB_MAX; ++r)
                if (r < nrb) {
                    const int64_t off = (((int64_t)ks * nRB + rbs + r) * 64 + lane) * EPL;
                    VT a = *reinterpret_cast<const VT*>(Ach + off);
                    acc[r] = mfma(a, b, acc[r]);
                    if (HILO) {
                        VT al = *reinterpret_cast<const VT*>(Alch + off);
                        acc[r] = mfma(a, bl, acc[r]);
                        acc[r] = mfma(al, b, acc[r]);
                    }
                }
        }
    }
    // D layout: lane holds rows 4*(lane/16) + j of column lane%16
    const int64_t fpos = f0 + wave * 16 + (lane & 15);
    if (fpos < n) {
        float* zp = zpart + (int64_t)split * zstride + fpos * Rp;
#pragma unroll
        for (int r = 0; r < NRB_MAX; ++r)
            if (r < nrb) {
                const int row = (rbs + r) * 16 + 4 * (lane >> 4);
                *reinterpret_cast<f4*>(zp + row) = acc[r];
            }
    }
}

// ------------------------------------------------------------------ Z prep
// One wave per frame: z = sum of the split partials (FP32), ||z||, and the
// GEMM2 operand copy in T, scaled by a power of two for FP16 so that
// max |z| * scale lies in [2^13, 2^14).
template <typename T>
__global__ __launch_bounds__(256) void k_zprep(const float* __restrict__ zpart, int nsplit, int64_t zstride,
                                               int64_t nfr, const int* __restrict__ fcount, int Rp, float* __restrict__ z32,
                                               T* __restrict__ zfrag, float* __restrict__ zscale,
                                               float* __restrict__ znorm, int scale16) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL;
    const int64_t n = fcount ? (int64_t)*fcount : nfr;
    const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= n) return;
    float mx = 0.f, ss = 0.f;
    for (int r = lane; r < Rp; r += 64) {
        float v = 0.f;
        for (int s = 0; s < nsplit; ++s) v += zpart[(int64_t)s * zstride + f * Rp + r];
        z32[f * Rp + r] = v;
        mx = fmaxf(mx, fabsf(v));
        ss += v * v;
    }
    mx = wave_max(mx);
    ss = wave_sum(ss);
    float sc = 1.f;
    if (scale16 && mx > 0.f) {
        int e;
        frexpf(mx, &e);  // mx in [2^(e-1), 2^e)
        sc = ldexpf(1.f, 14 - e);
    }
    if (lane == 0) {
        zscale[f] = sc;
        znorm[f] = sqrtf(ss);
    }
    if (zfrag) {
        const int64_t fb = f >> 4;
        const int nn = (int)(f & 15);
        const int KSn = Rp / KS;
        for (int r = lane; r < Rp; r += 64) {
            float v = z32[f * Rp + r] * sc;
            const int ks = r / KS, kin = r % KS;
            const int l = nn + 16 * (kin / EPL), e = kin % EPL;
            zfrag[((fb * KSn + ks) * 64 + l) * EPL + e] = cvt<T>(v);
        }
    }
}

// ------------------------------------------------------------------ GEMM2
// Workgroup: 4 waves x 64 directions (one tile each) x 64 frames.  The
// epilogue keeps only the maximum of each frame over the wave's 64 rows.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm2(const T* __restrict__ U, int KSn, const T* __restrict__ zfrag,
                                               int64_t nfr, int ncls, const float* __restrict__ zscale,
                                               float uinv, float* __restrict__ pmax, int64_t pstride,
                                               float* __restrict__ ycls, int64_t yld) {
    constexpr int EPL = Mf<T>::EPL;
    typedef typename Vec<T>::t VT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + wave;
    const int rb0 = tile * 4;
    const int64_t fb0 = (int64_t)blockIdx.y * 4;
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < KSn; ++ks) {
        VT a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *reinterpret_cast<const VT*>(U + (((int64_t)(rb0 + i) * KSn + ks) * 64 + lane) * EPL);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[j] = *reinterpret_cast<const VT*>(zfrag + (((fb0 + j) * KSn + ks) * 64 + lane) * EPL);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t f = (fb0 + j) * 16 + (lane & 15);
        const float inv = f < nfr ? uinv / zscale[f] : 0.f;
        float m = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + e;
                float v = acc[i][j][e];
                if (row < ncls) m = fmaxf(m, v);
                if (ycls && f < nfr && row < ncls) ycls[f * yld + row] = v * inv;
            }
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        if (lane < 16 && f < nfr) pmax[(int64_t)tile * pstride + f] = m * inv;
    }
}

// ------------------------------------------------------------------ final
// One wave per frame.  eps bounds |y_lowprec - y_fp32| for every direction
// of the frame (eps = ecoef * ||z||, ecoef from the operand rounding and the
// FP32 accumulation, Cauchy-Schwarz with max_q ||U_q||); every tile whose
// maximum is within 2 eps of the frame maximum is rescored in FP32.
template <int MAXM>
__global__ __launch_bounds__(256) void k_final(
    const float2* __restrict__ X, int M, int P, int B, const float* __restrict__ pmax, int64_t pstride, int ntile,
    int ncls, const float* __restrict__ z32, int Rp, const float* __restrict__ znorm, float ecoef, float kappa,
    int rescore, const float* __restrict__ U32T, const int32_t* __restrict__ rows, const int32_t* __restrict__ rep,
    const float* __restrict__ tauN, int64_t nfr, const int* __restrict__ flist, const int* __restrict__ fcount,
    const float* __restrict__ z32_first, int32_t* __restrict__ doa, float* __restrict__ power,
    float* __restrict__ yhat, float* __restrict__ margin, float hilo_thr, int* __restrict__ hlist,
    int* __restrict__ hcount) {
    __shared__ float zs[4][1024];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t n = flist ? (int64_t)*fcount : nfr;
    const int64_t pos = (int64_t)blockIdx.x * 4 + wave;
    if (pos >= n) return;
    const int64_t f = flist ? (int64_t)flist[pos] : pos;  // frame
    const float* z = z32 + pos * Rp;
    float* zw = zs[wave];
    for (int r = lane; r < Rp; r += 64) zw[r] = z[r];
    float eps = ecoef * znorm[pos];
    if (flist) {
        // second pass: z was recomputed; widen by kappa * ||z - z_first||
        float d2 = 0.f;
        for (int r = lane; r < Rp; r += 64) {
            float d = z[r] - z32_first[f * Rp + r];
            d2 += d * d;
        }
        eps += kappa * sqrtf(wave_sum(d2)) * 1.01f;
    }
    wave_sync();

    // frame maximum over tiles
    float ym = -INFINITY;
    for (int t = lane; t < ntile; t += 64) ym = fmaxf(ym, pmax[(int64_t)t * pstride + f]);
    ym = wave_max(ym);
    const float thr = rescore ? ym - 2.f * eps : ym;

    // pass 1: best over the rescored candidate tiles (value desc, index asc)
    float by = -INFINITY;
    int bq = 0x7fffffff;
    float ncmax = -INFINITY;  // max over tiles not rescored
    for (int t0 = 0; t0 < ntile; t0 += 64) {
        const int t = t0 + lane;
        float pv = t < ntile ? pmax[(int64_t)t * pstride + f] : -INFINITY;
        const bool cand = pv >= thr;
        if (!cand) ncmax = fmaxf(ncmax, pv);
        uint64_t mask = __ballot(cand);
        while (mask) {
            const int tt = t0 + __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int row = tt * QTILE + lane;
            const float* ut = U32T + (int64_t)tt * Rp * QTILE + lane;
            float y = 0.f;
            for (int r = 0; r < Rp; ++r) y = fmaf(ut[(int64_t)r * QTILE], zw[r], y);
            if (row < ncls) {
                const int q = rows[row];
                if (y > by || (y == by && q < bq)) {
                    by = y;
                    bq = q;
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        float oy = __shfl_xor(by, o);
        int oq = __shfl_xor(bq, o);
        if (oy > by || (oy == by && oq < bq)) {
            by = oy;
            bq = oq;
        }
    }
    if (bq < 0 || bq >= 0x7fffffff) bq = rows[0];  // no finite candidate
    const int cls = rep[bq];
    // pass 2: runner-up over other classes among the candidates
    float sy = -INFINITY;
    for (int t0 = 0; t0 < ntile; t0 += 64) {
        const int t = t0 + lane;
        float pv = t < ntile ? pmax[(int64_t)t * pstride + f] : -INFINITY;
        uint64_t mask = __ballot(pv >= thr);
        while (mask) {
            const int tt = t0 + __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int row = tt * QTILE + lane;
            if (row < ncls && rep[rows[row]] != cls) {
                const float* ut = U32T + (int64_t)tt * Rp * QTILE + lane;
                float y = 0.f;
                for (int r = 0; r < Rp; ++r) y = fmaf(ut[(int64_t)r * QTILE], zw[r], y);
                sy = fmaxf(sy, y);
            }
        }
    }
    sy = wave_max(sy);
    ncmax = wave_max(ncmax);
    if (ncmax > -INFINITY) sy = fmaxf(sy, ncmax + eps);
    const float mg = (by - sy) / fmaxf(fabsf(by), FLT_MIN);

    // Algorithm 1 online step 4: Y of the chosen direction from its row of W
    const float* tq = tauN + (int64_t)cls * P;
    float acc = 0.f;
    for (int bin = lane; bin < B; bin += 64) {
        const float2* xf = X + f * M * B + bin;
        float re[MAXM], im[MAXM];
#pragma unroll
        for (int m = 0; m < MAXM; ++m) {
            float2 v = m < M ? xf[(int64_t)m * B] : float2{0.f, 0.f};
            re[m] = v.x;
            im[m] = v.y;
            unit(re[m], im[m]);
        }
        int p = 0;
#pragma unroll
        for (int i = 0; i < MAXM; ++i)
#pragma unroll
            for (int j = i + 1; j < MAXM; ++j)
                if (j < M) {
                    float xr = re[i] * re[j] + im[i] * im[j];
                    float xi = im[i] * re[j] - re[i] * im[j];
                    float t = (float)bin * tq[p];
                    t -= rintf(t);
                    float c = __builtin_amdgcn_cosf(t), s = __builtin_amdgcn_sinf(t);
                    acc = fmaf(c, xr, fmaf(-s, xi, acc));
                    ++p;
                }
    }
    acc = wave_sum(acc);
    if (lane == 0) {
        doa[f] = cls;
        power[f] = acc;
        if (yhat) yhat[f] = by;
        if (margin) margin[f] = mg;
        if (!flist && hlist && mg < hilo_thr) {
            int k = atomicAdd(hcount, 1);
            hlist[k] = (int)f;
        }
    }
}

// y_opt: every direction takes the value of its scored row
__global__ void k_scatter_y(const float* __restrict__ ycls, int64_t yld, const int32_t* __restrict__ rowof,
                            int Q, int64_t nfr, float* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nfr * Q) return;
    const int64_t f = i / Q;
    const int q = (int)(i % Q);
    y[i] = ycls[f * yld + rowof[q]];
}

// ------------------------------------------------------------------ SRP
// PHAT vector in FP32, written as MFMA B-operand fragments of the 16x16x4
// instruction: element (k, frame) -> [frame/16][k/4][lane = frame%16 +
// 16 (k%4)], k = (bin P + p) 2 + {0: Re, 1: Im}.
// Frames from nfr up to fpad and the columns past 2L are written as zeros.
template <int MAXM>
__global__ void k_phat_frag(const float2* __restrict__ X, int64_t nfr, int64_t fpad, int M, int P, int B, int Wks,
                            float* __restrict__ xfr) {
    const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= fpad * B) return;
    const int64_t f = it / B;
    const int bin = (int)(it % B);
    const bool live = f < nfr;
    const float2* xf = X + (live ? f : 0) * M * B + bin;
    float re[MAXM], im[MAXM];
#pragma unroll
    for (int m = 0; m < MAXM; ++m) {
        float2 v = (live && m < M) ? xf[(int64_t)m * B] : float2{0.f, 0.f};
        re[m] = v.x;
        im[m] = v.y;
        unit(re[m], im[m]);
    }
    const int64_t base = (f >> 4) * Wks * 64;
    const int nn = (int)(f & 15);
    if (bin == B - 1)
        for (int k = 2 * P * B; k < 4 * Wks; ++k) xfr[base + (k >> 2) * 64 + nn + 16 * (k & 3)] = 0.f;
    int p = 0;
#pragma unroll
    for (int i = 0; i < MAXM; ++i)
#pragma unroll
        for (int j = i + 1; j < MAXM; ++j)
            if (j < M) {
                const float xr = re[i] * re[j] + im[i] * im[j];
                const float xi = im[i] * re[j] - re[i] * im[j];
                const int k = (bin * P + p) * 2;
                xfr[base + (k >> 2) * 64 + nn + 16 * (k & 3)] = xr;
                xfr[base + ((k + 1) >> 2) * 64 + nn + 16 * ((k + 1) & 3)] = xi;
                ++p;
            }
}

// W in FP32 as A-operand fragments of the 16x16x4 instruction: element
// (row q, k) -> [q/16][k/4][lane = q%16 + 16 (k%4)]; Re part cos, Im part
// -sin of 2 pi bin tau / N (phase reduced in FP64).
__global__ void k_w_frag(const double* __restrict__ tau, int Q, int P, int N, int L, int Wks, int rows_pad,
                         float* __restrict__ wfr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)rows_pad * Wks * 4;
    if (i >= total) return;
    const int lane = (int)(i % 64);
    const int64_t rest = i / 64;
    const int ks = (int)(rest % Wks);
    const int rb = (int)(rest / Wks);
    const int q = rb * 16 + (lane & 15);
    const int k = ks * 4 + (lane >> 4);
    const int c = k >> 1;
    float v = 0.f;
    if (q < Q && c < L) {
        const int bin = c / P, p = c % P;
        double t = (double)bin * tau[(int64_t)q * P + p] / (double)N;
        t -= rint(t);
        double s, co;
        sincospi(2.0 * t, &s, &co);
        v = (k & 1) ? (float)(-s) : (float)co;
    }
    wfr[i] = v;
}

// Plain SRP-PHAT GEMM, FP32 MFMA.  Workgroup 2 x 2 waves, tile 128
// directions x 128 frames; each wave 64 x 64.  Epilogue: per frame the
// maximum over the workgroup's 128 directions and its lowest index.
__global__ __launch_bounds__(256) void k_srp_gemm(const float* __restrict__ W, const float* __restrict__ xfr,
                                                  int Wks, int Q, int64_t nfr, float* __restrict__ pv,
                                                  int* __restrict__ pidx, int64_t pstride, float* __restrict__ y,
                                                  int64_t yld) {
    __shared__ float sv[2][128];
    __shared__ int si[2][128];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave >> 1, wc = wave & 1;
    const int rb0 = blockIdx.x * 8 + wr * 4;
    const int64_t fb0 = (int64_t)blockIdx.y * 8 + wc * 4;
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const float* wp[4];
    const float* xp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) wp[i] = W + ((int64_t)(rb0 + i) * Wks) * 64 + lane;
#pragma unroll
    for (int j = 0; j < 4; ++j) xp[j] = xfr + ((fb0 + j) * Wks) * 64 + lane;
    float a[4], b[4], an[4], bn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a[i] = wp[i][0];
        b[i] = xp[i][0];
    }
    for (int ks = 0; ks < Wks; ++ks) {
        const int kn = ks + 1 < Wks ? ks + 1 : ks;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            an[i] = wp[i][(int64_t)kn * 64];
            bn[i] = xp[i][(int64_t)kn * 64];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = an[i];
            b[i] = bn[i];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t f = (fb0 + j) * 16 + (lane & 15);
        float m = -INFINITY;
        int mi = 0x7fffffff;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + e;
                const float v = acc[i][j][e];
                if (row < Q) {
                    if (v > m) {  // rows visited in increasing order within a lane
                        m = v;
                        mi = row;
                    }
                    if (y && f < nfr) y[f * yld + row] = v;
                }
            }
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float om = __shfl_xor(m, o);
            const int oi = __shfl_xor(mi, o);
            if (om > m || (om == m && oi < mi)) {
                m = om;
                mi = oi;
            }
        }
        if (lane < 16) {
            sv[wr][wc * 64 + j * 16 + lane] = m;
            si[wr][wc * 64 + j * 16 + lane] = mi;
        }
    }
    __syncthreads();
    if (threadIdx.x < 128) {
        const int c = threadIdx.x;
        float m = sv[0][c];
        int mi = si[0][c];
        const float m1 = sv[1][c];
        const int i1 = si[1][c];
        if (m1 > m || (m1 == m && i1 < mi)) {
            m = m1;
            mi = i1;
        }
        const int64_t f = (int64_t)blockIdx.y * 128 + c;
        if (f < nfr) {
            pv[(int64_t)blockIdx.x * pstride + f] = m;
            pidx[(int64_t)blockIdx.x * pstride + f] = mi;
        }
    }
}

__global__ void k_srp_reduce(const float* __restrict__ pv, const int* __restrict__ pidx, int64_t pstride,
                             int ntile, int64_t nfr, const int32_t* __restrict__ rep, int32_t* __restrict__ doa,
                             float* __restrict__ power) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nfr) return;
    float m = -INFINITY;
    int mi = 0x7fffffff;
    for (int t = 0; t < ntile; ++t) {
        const float v = pv[(int64_t)t * pstride + f];
        const int i = pidx[(int64_t)t * pstride + f];
        if (v > m || (v == m && i < mi)) {
            m = v;
            mi = i;
        }
    }
    if (mi < 0 || mi >= 0x7fffffff) mi = 0;  // no finite power
    doa[f] = rep[mi];
    power[f] = m;
}

// unit roundoff of each operand type
inline double unit_roundoff(int prec) {
    return prec == P_FP32 ? std::ldexp(1.0, -24) : prec == P_FP16 ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
}

template <typename T>
void run_locate(svdphat_plan* p, const float2* X, int64_t F, int prec, uint32_t mode, int32_t* doa, float* power,
                float* yhat, float* margin, float* y_opt, hipStream_t s) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL;
    const G1Layout& g = p->g1[prec];
    const int Rp = p->Rp, nRB = Rp / 16, KSn = Rp / KS;
    const int ntile = p->ncls_pad / QTILE;
    const int64_t Fc = round_up64(F, 64);
    const int nrg = cdiv(nRB, NRB_MAX);
    const int ftiles = (int)(Fc / 64);
    int nsplit = std::max(1, std::min(std::min(g.nch, 8), cdiv(1024, ftiles * nrg)));
    const int cps = cdiv(g.nch, nsplit);
    nsplit = cdiv(g.nch, cps);
    const bool hilo = (mode & SVDPHAT_HILO) && prec != P_FP32;

    // workspace carve-up
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += round_up64((int64_t)bytes, 256);
        return o;
    };
    const size_t o_zpart = take(sizeof(float) * nsplit * Fc * Rp);
    const size_t o_z32 = take(sizeof(float) * Fc * Rp);
    const size_t o_z32h = hilo ? take(sizeof(float) * Fc * Rp) : 0;
    const size_t o_zfrag = take(sizeof(T) * Fc * Rp);
    const size_t o_zsc = take(sizeof(float) * Fc);
    const size_t o_zn = take(sizeof(float) * Fc);
    const size_t o_znh = hilo ? take(sizeof(float) * Fc) : 0;
    const size_t o_pmax = take(sizeof(float) * ntile * Fc);
    const size_t o_hl = hilo ? take(sizeof(int) * Fc) : 0;
    const size_t o_hc = hilo ? take(sizeof(int) * 64) : 0;
    const size_t o_y = y_opt ? take(sizeof(float) * Fc * p->ncls_pad) : 0;
    char* w = (char*)ws_get(p, s, off);
    float* zpart = (float*)(w + o_zpart);
    float* z32 = (float*)(w + o_z32);
    T* zfrag = (T*)(w + o_zfrag);
    float* zsc = (float*)(w + o_zsc);
    float* zn = (float*)(w + o_zn);
    float* pmax = (float*)(w + o_pmax);
    float* ycls = y_opt ? (float*)(w + o_y) : nullptr;
    int* hl = hilo ? (int*)(w + o_hl) : nullptr;
    int* hc = hilo ? (int*)(w + o_hc) : nullptr;
    // zero the padding frames of the GEMM2 operand
    SP_HIP(hipMemsetAsync(zfrag, 0, sizeof(T) * Fc * Rp, s));
    if (hilo) SP_HIP(hipMemsetAsync(hc, 0, sizeof(int), s));

    const int M = p->M;
    const int64_t zstride = Fc * Rp;
    KernelTimer kt(s);
    const size_t lds = (size_t)64 * (g.CW + XPAD) * sizeof(T);
    kt.begin("gemm1");
    dim3 g1grid(ftiles, nsplit, nrg);
    if (M <= 8)
        k_gemm1<T, 64, 8, false><<<g1grid, 256, lds, s>>>(X, F, M, p->P, p->B, p->d_pi, p->d_pj, (const T*)p->A[prec],
                                                          nullptr, nRB, g.BB, g.CW, g.nch, cps, zpart, zstride, Rp,
                                                          nullptr, nullptr);
    else
        k_gemm1<T, 64, 16, false><<<g1grid, 256, lds, s>>>(X, F, M, p->P, p->B, p->d_pi, p->d_pj, (const T*)p->A[prec],
                                                           nullptr, nRB, g.BB, g.CW, g.nch, cps, zpart, zstride, Rp,
                                                           nullptr, nullptr);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("zprep");
    k_zprep<T><<<dim3((unsigned)(Fc / 4)), 256, 0, s>>>(zpart, nsplit, zstride, F, nullptr, Rp, z32, zfrag, zsc, zn,
                                                        prec == P_FP16 ? 1 : 0);
    SP_HIP(hipGetLastError());
    kt.end();
    const float uinv = 1.f / p->uscale[prec];
    kt.begin("gemm2");
    k_gemm2<T><<<dim3(p->ncls_pad / 256, (unsigned)(Fc / 64)), 256, 0, s>>>(
        (const T*)p->Ufr[prec], KSn, zfrag, F, p->ncls, zsc, uinv, pmax, Fc, ycls, p->ncls_pad);
    SP_HIP(hipGetLastError());
    kt.end();
    if (y_opt) {
        kt.begin("scatter_y");
        const int64_t tot = F * p->Q;
        // row of every direction: its class representative's row
        k_scatter_y<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>(ycls, p->ncls_pad, p->d_rowof, p->Q, F, y_opt);
        SP_HIP(hipGetLastError());
        kt.end();
    }
    const double u = unit_roundoff(prec);
    const double acc_err = 2.0 * Rp * std::ldexp(1.0, -24);
    const double lin = prec == P_FP32 ? acc_err : (2.0 * u + u * u + acc_err);
    const float ecoef = (float)(lin * p->kappa * 1.01);
    const int rescore = (mode & SVDPHAT_RESCORE) ? 1 : 0;
    const float hthr = prec == P_FP16 ? 1e-4f : 1e-3f;
    auto finalize = [&](const char* name, const float* zz, const float* znn, const int* fl, const int* fc,
                        const float* zfirst) {
        kt.begin(name);
        dim3 grid((unsigned)(Fc / 4));
        if (M <= 8)
            k_final<8><<<grid, 256, 0, s>>>(X, M, p->P, p->B, pmax, Fc, ntile, p->ncls, zz, Rp, znn, ecoef,
                                            (float)p->kappa, rescore, p->U32T, p->d_rows, p->d_rep, p->d_tauN_all, F,
                                            fl, fc, zfirst, doa, power, yhat, margin, hthr, fl ? nullptr : hl, hc);
        else
            k_final<16><<<grid, 256, 0, s>>>(X, M, p->P, p->B, pmax, Fc, ntile, p->ncls, zz, Rp, znn, ecoef,
                                             (float)p->kappa, rescore, p->U32T, p->d_rows, p->d_rep, p->d_tauN_all, F,
                                             fl, fc, zfirst, doa, power, yhat, margin, hthr, fl ? nullptr : hl, hc);
        SP_HIP(hipGetLastError());
        kt.end();
    };
    finalize("final", z32, zn, nullptr, nullptr, nullptr);
    if (hilo) {
        float* z32h = (float*)(w + o_z32h);
        float* znh = (float*)(w + o_znh);
        const size_t lds2 = (size_t)2 * 32 * (g.CW + XPAD) * sizeof(T);
        kt.begin("gemm1_hilo");
        dim3 hg((unsigned)(Fc / 32), nsplit, nrg);
        if (M <= 8)
            k_gemm1<T, 32, 8, true><<<hg, 128, lds2, s>>>(X, F, M, p->P, p->B, p->d_pi, p->d_pj, (const T*)p->A[prec],
                                                          (const T*)p->Alo[prec], nRB, g.BB, g.CW, g.nch, cps, zpart,
                                                          zstride, Rp, hl, hc);
        else
            k_gemm1<T, 32, 16, true><<<hg, 128, lds2, s>>>(X, F, M, p->P, p->B, p->d_pi, p->d_pj,
                                                           (const T*)p->A[prec], (const T*)p->Alo[prec], nRB, g.BB,
                                                           g.CW, g.nch, cps, zpart, zstride, Rp, hl, hc);
        SP_HIP(hipGetLastError());
        kt.end();
        kt.begin("zprep_hilo");
        k_zprep<T><<<dim3((unsigned)(Fc / 4)), 256, 0, s>>>(zpart, nsplit, zstride, F, hc, Rp, z32h, nullptr, zsc,
                                                            znh, 0);
        SP_HIP(hipGetLastError());
        kt.end();
        finalize("final_hilo", z32h, znh, hl, hc, z32);
    }
    kt.flush();
    (void)EPL;
}

}  // namespace

void launch_locate(svdphat_plan* p, const void* X, int64_t F, int prec, uint32_t mode, int32_t* doa, float* power,
                   float* yhat, float* margin, float* y_opt, hipStream_t s) {
    const float2* x = (const float2*)X;
    if (prec == P_FP32) run_locate<float>(p, x, F, prec, mode, doa, power, yhat, margin, y_opt, s);
    else if (prec == P_FP16) run_locate<_Float16>(p, x, F, prec, mode, doa, power, yhat, margin, y_opt, s);
    else run_locate<__bf16>(p, x, F, prec, mode, doa, power, yhat, margin, y_opt, s);
}

void build_w_fp32_frags(svdphat_plan* p) {
    const int Wk = round_up(2 * p->L, 4) / 4;
    p->Wks = Wk;
    p->Wrows_pad = round_up(p->Q, 128);
    const int64_t total = (int64_t)p->Wrows_pad * Wk * 4;
    if (hipMalloc((void**)&p->Wfr, total * sizeof(float)) != hipSuccess) {
        p->Wfr = nullptr;
        fail(SVDPHAT_E_NOMEM, "device allocation of W (" + std::to_string(total * 4) + " bytes) failed");
    }
    p->device_bytes += total * (int64_t)sizeof(float);
    double* dtau = nullptr;
    SP_HIP(hipMalloc((void**)&dtau, p->tau.size() * sizeof(double)));
    SP_HIP(hipMemcpy(dtau, p->tau.data(), p->tau.size() * sizeof(double), hipMemcpyHostToDevice));
    k_w_frag<<<dim3((unsigned)((total + 255) / 256)), 256>>>(dtau, p->Q, p->P, p->N, p->L, Wk, p->Wrows_pad, p->Wfr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(dtau);
    if (e != hipSuccess) fail(SVDPHAT_E_DEVICE, std::string("k_w_frag: ") + hipGetErrorString(e));
}

void launch_srp(svdphat_plan* p, const void* Xv, int64_t F, int32_t* doa, float* power, float* y_opt,
                hipStream_t s) {
    const float2* X = (const float2*)Xv;
    const int64_t Fp = round_up64(F, 128);
    const int Wks = p->Wks;
    const int ntile = p->Wrows_pad / 128;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += round_up64((int64_t)bytes, 256);
        return o;
    };
    const size_t o_x = take(sizeof(float) * Fp * Wks * 4);
    const size_t o_v = take(sizeof(float) * ntile * Fp);
    const size_t o_i = take(sizeof(int) * ntile * Fp);
    char* w = (char*)ws_get(p, s, off);
    KernelTimer kt(s);
    float* xfr = (float*)(w + o_x);
    float* pv = (float*)(w + o_v);
    int* pidx = (int*)(w + o_i);
    kt.begin("srp_phat");
    const int64_t items = Fp * p->B;
    if (p->M <= 8)
        k_phat_frag<8><<<dim3((unsigned)((items + 255) / 256)), 256, 0, s>>>(X, F, Fp, p->M, p->P, p->B, Wks, xfr);
    else
        k_phat_frag<16><<<dim3((unsigned)((items + 255) / 256)), 256, 0, s>>>(X, F, Fp, p->M, p->P, p->B, Wks, xfr);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("srp_gemm");
    k_srp_gemm<<<dim3(ntile, (unsigned)(Fp / 128)), 256, 0, s>>>(p->Wfr, xfr, Wks, p->Q, F, pv, pidx, Fp, y_opt,
                                                                 p->Q);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("srp_reduce");
    k_srp_reduce<<<dim3((unsigned)((F + 255) / 256)), 256, 0, s>>>(pv, pidx, Fp, ntile, F, p->d_rep, doa, power);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.flush();
}

}  // namespace svdphat
