// Online SVD-PHAT on gfx950 (Algorithm 1, online steps 1-4, Section 3) with
// the exhaustive search of eq. (14).
//
//   k_gemm1   PHAT cross-spectra (eq. (3)) formed in LDS from the STFT and
//             projected with MFMA: Z = S V^H X (eq. (12) with S folded into
//             V^H), stacked real.  The reduction axis is split over the grid
//             (partial Z per split) and, inside a workgroup, interleaved over
//             the four waves, so each A fragment is read once per workgroup.
//   k_zprep   sums the partial Z, keeps an FP32 copy and ||z||, and packs a
//             copy in the GEMM2 operand type and fragment order (FP16 scaled
//             by a power of two per frame).
//   k_gemm2   Y = Re(U Z) (eqs. (13)-(14)) with MFMA.  Each wave holds the U
//             fragments of one tile of 64 scored directions in registers and
//             streams frames; its epilogue keeps one maximum per (frame, tile).
//   k_final   (k_final_np without the power) per frame: every tile whose
//             maximum is within the rounding bound
//             of the frame maximum is rescored in FP32; best class, runner-up
//             and margin; frames whose margin is within the modelled GEMM1
//             rounding are queued for a hi/lo recomputation, which
//             k_gemm1_list and k_final_list (summing the list's partial Z
//             itself) redo over the device-counted list.
//   k_power   the power of the chosen direction from its row of W (Algorithm
//             1, online step 4), once the directions are final.
#include "device.h"

#include <type_traits>

namespace svdphat {

namespace {

constexpr int XPAD = 8;  // LDS row padding (elements) of the x tile
constexpr int G1_IPT8 = 3;   // chunk items per thread, arrays of up to 8 microphones
constexpr int G1_IPT16 = 1;  // and of up to 16

// ------------------------------------------------------------------ GEMM1
// Workgroup: 4 waves, NF frames, NRB row blocks of Z (row group blockIdx.z),
// the chunks [blockIdx.y * cps, ...) of the reduction axis.  Per chunk, the
// PHAT vector of BB bins x NF frames is formed in LDS (per-mic unit
// normalisation, then X_i conj(X_j) for pairs i < j in order, rounded to T
// and stored as (Re, Im) pairs), then the chunk's k-steps are shared out
// round-robin to the waves; each wave accumulates all NRB x NF/16 output
// blocks.  The four partial sums are added through LDS at the end.
template <typename T, int NF, int NRB, int MAXM, int IPT, bool HILO, bool RED3 = false>
__device__ __forceinline__ void gemm1_body(int bx, int by, int bz, const float2* __restrict__ X, int64_t nfr,
                                           int M, int P, int B, const T* __restrict__ A, const T* __restrict__ Alo,
                                           int nRB, int BB, int CW, int nch, int cps, float* __restrict__ zpart,
                                           int64_t zstride, int Rp, const int* __restrict__ flist,
                                           const int* __restrict__ fcount) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL, FB = NF / 16;
    typedef typename Vec<T>::t VT;
    typedef typename Vec<T>::pair VP;
    extern __shared__ __align__(16) char smem[];
    T* xs = reinterpret_cast<T*>(smem);
    const int ldx = CW + XPAD;
    T* xl = xs + NF * ldx;

    const int64_t n = flist ? (int64_t)*fcount : nfr;
    const int64_t f0 = (int64_t)bx * NF;
    if (f0 >= n) return;
    const int c0 = by * cps, c1 = min(nch, c0 + cps);
    const int rbs = bz * NRB;
    const int nrb = min(NRB, nRB - rbs);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ks_chunk = CW / KS;
    const int twoP = 2 * P;

    // the first chunk's A fragments depend on nothing: they go out first
    VT an[NRB], aln[NRB];
    auto loadA = [&](int ch, int ks) {
        const int64_t cbase = (int64_t)ch * ks_chunk * nRB;
#pragma unroll
        for (int r = 0; r < NRB; ++r)
            if (r < nrb) {
                const int64_t off = ((cbase + (int64_t)ks * nRB + rbs + r) * 64 + lane) * EPL;
                an[r] = *reinterpret_cast<const VT*>(A + off);
                if (HILO) aln[r] = *reinterpret_cast<const VT*>(Alo + off);
            }
    };
    if (wave < ks_chunk) loadA(c0, wave);
    f4 acc[NRB][FB];
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
        for (int j = 0; j < FB; ++j) acc[r][j] = f4{0.f, 0.f, 0.f, 0.f};

    // STFT values of the next chunk are loaded into registers before the
    // current chunk's MFMA phase, so their latency hides behind it.  Item
    // it = (frame it / BB, bin it % BB); at most IPT items per thread; the
    // item's frame and base address do not change from chunk to chunk.
    float2 xv[IPT][MAXM];
    const float2* xbase[IPT];
    int bofs[IPT];
    bool ilive[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int it = threadIdx.x + 256 * k;
        const int fl = it / BB, bl = it - (it / BB) * BB;
        const int64_t fpos = f0 + fl;
        ilive[k] = it < NF * BB && fpos < n;
        const int64_t f = ilive[k] ? (flist ? (int64_t)flist[fpos] : fpos) : 0;
        xbase[k] = X + f * M * B + bl;
        bofs[k] = bl;
    }
    auto fetch = [&](int ch) {
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const bool live = ilive[k] && ch * BB + bofs[k] < B;
            const float2* xf = xbase[k] + ch * BB;
#pragma unroll
            for (int m = 0; m < MAXM; ++m) xv[k][m] = (live && m < M) ? xf[(int64_t)m * B] : float2{0.f, 0.f};
        }
    };
    fetch(c0);
    // zero the pad columns past the chunk's pair products (read by the last
    // k-step) while the loads are in flight
    {
        const int c0w = BB * twoP, pw = ldx - c0w;
        for (int i = threadIdx.x; i < NF * pw; i += 256) {
            const int fl = i / pw;
            const int idx = fl * ldx + c0w + (i - fl * pw);
            xs[idx] = cvt<T>(0.f);
            if (HILO) xl[idx] = cvt<T>(0.f);
        }
    }
    for (int ch = c0; ch < c1; ++ch) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const int it = threadIdx.x + 256 * k;
            if (it >= NF * BB) break;
            const int fl = it / BB, bl = bofs[k];
            VP* dst = reinterpret_cast<VP*>(xs + fl * ldx + bl * twoP);
            VP* dlo = reinterpret_cast<VP*>(xl + fl * ldx + bl * twoP);
            // pair (i, j), i < j < M, goes to slot i M - i (i + 1) / 2 + j - i - 1
            // of the bin's run; pairs with j >= M go to the row's padding past
            // the tile (columns CW .. ldx - 1, never read), so the unrolled
            // loops below carry no branch per pair
            VP* pad = reinterpret_cast<VP*>(xs + fl * ldx + CW);
            VP* padl = reinterpret_cast<VP*>(xl + fl * ldx + CW);
            auto slot = [&](VP* base, VP* sink, int i, int j) {
                return j < M ? base + (i * M - i * (i + 1) / 2 + j - i - 1) : sink;
            };
            float re[MAXM], im[MAXM];
#pragma unroll
            for (int m = 0; m < MAXM; ++m) {
                re[m] = xv[k][m].x;
                im[m] = xv[k][m].y;
                unit(re[m], im[m]);
            }
            if constexpr (std::is_same<T, _Float16>::value && !HILO) {
                // FP16 operands: the pair products are formed in packed f16,
                // (Re, Im) = (re_i, im_i) re_j + (im_i, -re_i) im_j
                h2 a[MAXM], c[MAXM];
#pragma unroll
                for (int m = 0; m < MAXM; ++m) {
                    a[m] = h2{(_Float16)re[m], (_Float16)im[m]};
                    c[m] = h2{(_Float16)im[m], (_Float16)(-re[m])};
                }
#pragma unroll
                for (int i = 0; i < MAXM; ++i)
#pragma unroll
                    for (int j = i + 1; j < MAXM; ++j) {
                        const h2 rj = h2{a[j].x, a[j].x}, ij = h2{a[j].y, a[j].y};
                        *slot(dst, pad, i, j) = a[i] * rj + c[i] * ij;
                    }
            } else {
#pragma unroll
                for (int i = 0; i < MAXM; ++i)
#pragma unroll
                    for (int j = i + 1; j < MAXM; ++j) {
                        const float xr = re[i] * re[j] + im[i] * im[j];
                        const float xi = im[i] * re[j] - re[i] * im[j];
                        const T hr = cvt<T>(xr), hi = cvt<T>(xi);
                        *slot(dst, pad, i, j) = mkpair<T>(hr, hi);
                        if (HILO) *slot(dlo, padl, i, j) = mkpair<T>(cvt<T>(xr - (float)hr), cvt<T>(xi - (float)hi));
                    }
            }
        }
        __syncthreads();
        if (ch + 1 < c1) fetch(ch + 1);
        if (ch > c0 && wave < ks_chunk) loadA(ch, wave);
        for (int ks = wave; ks < ks_chunk; ks += 4) {
            VT a[NRB], al[NRB];
#pragma unroll
            for (int r = 0; r < NRB; ++r) {
                a[r] = an[r];
                if (HILO) al[r] = aln[r];
            }
            if (ks + 4 < ks_chunk) loadA(ch, ks + 4);
            VT b[FB], bl[FB];
#pragma unroll
            for (int j = 0; j < FB; ++j) {
                const T* bp = xs + (j * 16 + (lane & 15)) * ldx + ks * KS + EPL * (lane >> 4);
                b[j] = *reinterpret_cast<const VT*>(bp);
                if (HILO) bl[j] = *reinterpret_cast<const VT*>(bp + NF * ldx);
            }
#pragma unroll
            for (int r = 0; r < NRB; ++r)
                if (r < nrb)
#pragma unroll
                    for (int j = 0; j < FB; ++j) {
                        acc[r][j] = mfma(a[r], b[j], acc[r][j]);
                        if (HILO) {
                            acc[r][j] = mfma(a[r], bl[j], acc[r][j]);
                            acc[r][j] = mfma(al[r], b[j], acc[r][j]);
                        }
                    }
        }
    }
    // add the four waves' partial sums through LDS (RED3: waves 1-3 at once,
    // in three regions)
    __syncthreads();
    f4* red = reinterpret_cast<f4*>(smem);
    if constexpr (RED3) {
        if (wave > 0)
#pragma unroll
            for (int r = 0; r < NRB; ++r)
#pragma unroll
                for (int j = 0; j < FB; ++j) red[(((wave - 1) * NRB + r) * FB + j) * 64 + lane] = acc[r][j];
        __syncthreads();
        if (wave == 0)
#pragma unroll
            for (int w = 0; w < 3; ++w)
#pragma unroll
                for (int r = 0; r < NRB; ++r)
#pragma unroll
                    for (int j = 0; j < FB; ++j) acc[r][j] += red[((w * NRB + r) * FB + j) * 64 + lane];
        __syncthreads();  // LDS free for the next item
    }
    for (int w = 1; w < (RED3 ? 1 : 4); ++w) {
        if (wave == w)
#pragma unroll
            for (int r = 0; r < NRB; ++r)
#pragma unroll
                for (int j = 0; j < FB; ++j) red[(r * FB + j) * 64 + lane] = acc[r][j];
        __syncthreads();
        if (wave == 0)
#pragma unroll
            for (int r = 0; r < NRB; ++r)
#pragma unroll
                for (int j = 0; j < FB; ++j) acc[r][j] += red[(r * FB + j) * 64 + lane];
        __syncthreads();
    }
    if (wave != 0) return;
    // D layout: lane holds rows 4*(lane/16) + e of column lane%16
#pragma unroll
    for (int j = 0; j < FB; ++j) {
        const int64_t fpos = f0 + j * 16 + (lane & 15);
        if (fpos >= n) continue;
        float* zp = zpart + (int64_t)by * zstride + fpos * Rp;
#pragma unroll
        for (int r = 0; r < NRB; ++r)
            if (r < nrb) *reinterpret_cast<f4*>(zp + (rbs + r) * 16 + 4 * (lane >> 4)) = acc[r][j];
    }
}

// the same over a device-counted frame list, grid-stride over (frame tile,
// split) items
template <typename T, int NF, int NRB, int MAXM, int IPT, bool HILO>
__global__ __launch_bounds__(256) void k_gemm1_list(const float2* __restrict__ X, int M, int P, int B,
                                                    const T* __restrict__ A, const T* __restrict__ Alo, int nRB,
                                                    int BB, int CW, int nch, int cps, int nsplit,
                                                    float* __restrict__ zpart, int64_t zstride, int Rp,
                                                    const int* __restrict__ flist, const int* __restrict__ fcount) {
    const int64_t n = *fcount;
    const int64_t items = (n + NF - 1) / NF * nsplit;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x)
        gemm1_body<T, NF, NRB, MAXM, IPT, HILO, true>((int)(it / nsplit), (int)(it % nsplit), blockIdx.z, X, n, M, P, B, A,
                                                Alo, nRB, BB, CW, nch, cps, zpart, zstride, Rp, flist, fcount);
}

template <typename T, int NF, int NRB, int MAXM, int IPT, bool HILO>
__global__ __launch_bounds__(256) void k_gemm1(const float2* __restrict__ X, int64_t nfr, int M, int P, int B,
                                               const T* __restrict__ A, const T* __restrict__ Alo, int nRB, int BB,
                                               int CW, int nch, int cps, float* __restrict__ zpart, int64_t zstride,
                                               int Rp, const int* __restrict__ flist, const int* __restrict__ fcount) {
    gemm1_body<T, NF, NRB, MAXM, IPT, HILO>(blockIdx.x, blockIdx.y, blockIdx.z, X, nfr, M, P, B, A, Alo, nRB, BB, CW,
                                            nch, cps, zpart, zstride, Rp, flist, fcount);
}

// ------------------------------------------------------------------ Z prep
// One wave per frame: z = sum of the split partials (FP32), ||z||, and the
// GEMM2 operand copy in T (FP16: scaled by 2^e so that max |z| lies in
// [2^13, 2^14)), in B-operand fragment order [frame/16][k-step][lane][EPL].
// Partial sums of GEMM1 to add for frame f: nsplit, or with the streamed
// GEMM1 (sG > 0 workgroups over sU units of snch chunks per 64-frame tile)
// one per workgroup whose unit range meets the frame's tile.
__device__ __forceinline__ int zpart_count(int64_t f, int nsplit, int sG, int64_t sU, int snch) {
    if (sG <= 0) return nsplit;
    const int64_t t = f >> 6;
    const int64_t u0 = t * snch, u1 = u0 + snch - 1;
    const int w0 = (int)(((u0 + 1) * sG - 1) / sU), w1 = (int)(((u1 + 1) * sG - 1) / sU);
    return w1 - w0 + 1;
}

template <typename T>
__device__ __forceinline__ void zprep_body(int bx, const float* __restrict__ zpart, int nsplit0, int64_t zstride,
                                           int64_t nfr, const int* __restrict__ fcount, int Rp,
                                           float* __restrict__ z32, T* __restrict__ zfrag,
                                           float* __restrict__ zscale, float* __restrict__ znorm, int scale16,
                                           int sG = 0, int64_t sU = 0, int snch = 0) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL;
    const int64_t n = fcount ? (int64_t)*fcount : nfr;
    const int64_t f = (int64_t)bx * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= n) return;
    const int nsplit = zpart_count(f, nsplit0, sG, sU, snch);
    float mx = 0.f, ss = 0.f;
    for (int r = lane; r < Rp; r += 64) {
        // the split partials are loaded eight at a time, all in flight together
        float v = 0.f;
        for (int s0 = 0; s0 < nsplit; s0 += 8) {
            float part[8];
#pragma unroll
            for (int s = 0; s < 8; ++s)
                part[s] = s0 + s < nsplit ? zpart[(int64_t)(s0 + s) * zstride + f * Rp + r] : 0.f;
#pragma unroll
            for (int s = 0; s < 8; ++s) v += part[s];
        }
        z32[f * Rp + r] = v;
        mx = fmaxf(mx, fabsf(v));
        ss += v * v;
    }
    mx = wave_max(mx);
    ss = wave_sum(ss);
    float sc = 1.f;
    if (scale16 && mx > 0.f) {
        int e;
        frexpf(mx, &e);
        sc = ldexpf(1.f, 14 - e);
    }
    if (lane == 0) {
        if (zscale) zscale[f] = sc;
        znorm[f] = sqrtf(ss);
    }
    if (zfrag) {
        const int64_t fb = f >> 4;
        const int nn = (int)(f & 15);
        const int KSn = Rp / KS;
        for (int r = lane; r < Rp; r += 64) {
            const float v = z32[f * Rp + r] * sc;
            const int ks = r / KS, kin = r % KS;
            zfrag[((fb * KSn + ks) * 64 + nn + 16 * (kin / EPL)) * EPL + kin % EPL] = cvt<T>(v);
        }
    }
}

// The same for 16-bit operands and Rp <= 128, sixteen lanes per frame: lane
// j < Rp / 8 of a frame's group sums rows 8j .. 8j+7 over the partials
// (16-byte loads, all in flight together), the group reduces max |z| and
// ||z||^2 within its 16 lanes, and each lane writes its 8 rows of the GEMM2
// operand as one 16-byte piece of the fragment.
template <typename T>
__global__ __launch_bounds__(256) void k_zprep16(const float* __restrict__ zpart, int nsplit0, int64_t zstride,
                                                 int64_t nfr, int Rp, float* __restrict__ z32, T* __restrict__ zfrag,
                                                 float* __restrict__ zscale, float* __restrict__ znorm, int scale16,
                                                 int sG, int64_t sU, int snch, int* __restrict__ clear = nullptr) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL;
    static_assert(EPL == 8, "16-bit fragment layout");
    // a word the later kernels of the call count into (the hi/lo list
    // count), cleared here instead of by a launch of its own
    if (clear && blockIdx.x == 0 && threadIdx.x == 0) *clear = 0;
    typedef typename Vec<T>::t VT;
    const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    const int64_t f = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 6) * 4 + g;
    const bool fl = f < nfr;
    const int64_t fc = fl ? f : 0;
    const bool act = fl && j < Rp / 8;
    const int ns = zpart_count(fc, nsplit0, sG, sU, snch);
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float* src = zpart + fc * Rp + 8 * (act ? j : 0);
    // slots two at a time: most frames have one or two (a frame tile that
    // one or two workgroups cover), so no clamped copies are loaded
    for (int s0 = 0; s0 < ns; s0 += 2) {
        float4 a[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float* p = src + (int64_t)min(s0 + s, ns - 1) * zstride;
            a[s][0] = *reinterpret_cast<const float4*>(p);
            a[s][1] = *reinterpret_cast<const float4*>(p + 4);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
            if (s0 + s < ns) {
                v[0] += a[s][0].x; v[1] += a[s][0].y; v[2] += a[s][0].z; v[3] += a[s][0].w;
                v[4] += a[s][1].x; v[5] += a[s][1].y; v[6] += a[s][1].z; v[7] += a[s][1].w;
            }
    }
    float mx = 0.f, ss = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if (!act) v[e] = 0.f;
        mx = fmaxf(mx, fabsf(v[e]));
        ss = fmaf(v[e], v[e], ss);
    }
    {
        // over the frame's 16 lanes (one row), in registers
        uint32_t v[2] = {__float_as_uint(mx), __float_as_uint(ss)};
        row_reduce(v, [](uint32_t (&x)[2], const uint32_t (&o)[2]) {
            x[0] = __float_as_uint(fmaxf(__uint_as_float(x[0]), __uint_as_float(o[0])));
            x[1] = __float_as_uint(__uint_as_float(x[1]) + __uint_as_float(o[1]));
        });
        mx = __uint_as_float(v[0]);
        ss = __uint_as_float(v[1]);
    }
    float sc = 1.f;
    if (scale16 && mx > 0.f) {
        int e;
        frexpf(mx, &e);
        sc = ldexpf(1.f, 14 - e);
    }
    if (!act) return;
    *reinterpret_cast<float4*>(z32 + f * Rp + 8 * j) = float4{v[0], v[1], v[2], v[3]};
    *reinterpret_cast<float4*>(z32 + f * Rp + 8 * j + 4) = float4{v[4], v[5], v[6], v[7]};
    if (j == 0) {
        zscale[f] = sc;
        znorm[f] = sqrtf(ss);
    }
    // rows 8j .. 8j+7: k-step 8j / KS, lane (f & 15) + 16 ((8j % KS) / 8) of the fragment
    const int KSn = Rp / KS;
    const int64_t fb = f >> 4;
    VT h;
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = cvt<T>(v[e] * sc);
    *reinterpret_cast<VT*>(zfrag + ((fb * KSn + (8 * j) / KS) * 64 + (f & 15) + 16 * ((8 * j % KS) / 8)) * EPL) = h;
}

template <typename T>
__global__ __launch_bounds__(256) void k_zprep(const float* __restrict__ zpart, int nsplit, int64_t zstride,
                                               int64_t nfr, const int* __restrict__ fcount, int Rp,
                                               float* __restrict__ z32, T* __restrict__ zfrag,
                                               float* __restrict__ zscale, float* __restrict__ znorm, int scale16,
                                               int sG, int64_t sU, int snch, int* __restrict__ clear = nullptr) {
    if (clear && blockIdx.x == 0 && threadIdx.x == 0) *clear = 0;  // as in k_zprep16
    zprep_body<T>(blockIdx.x, zpart, nsplit, zstride, nfr, fcount, Rp, z32, zfrag, zscale, znorm, scale16, sG, sU,
                  snch);
}

// ------------------------------------------------------------------ GEMM2
// Wave = one tile of 64 scored directions (4 row blocks); workgroup = 4 tiles
// x a range of FCH frames, streamed 16 at a time.  With KSN > 0 (exactly
// KSn k-steps) the wave keeps the tile's U fragments in registers and a
// ring of two Z-fragment sets in flight (the loads of block b+2 are issued
// after the MFMAs of block b, outside every branch, so the wait counts stay
// exact; the ring's first values pass through an empty asm statement so the
// compiler cannot merge the two load sites).  KSN = 0 is the general form
// (U fragments read per k-step).  The epilogue keeps one maximum per (frame,
// tile), frame-major: pmax[f * pstride + tile], scaled back by the power-of-
// two scales of U and of the frame's Z.

// maximum over lanes l, l ^ 16, l ^ 32, l ^ 48 (the four row groups of a
// 16 x 16 MFMA result)
__device__ __forceinline__ float max_rowgroups(float m) {
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(m), __float_as_uint(m), false, false);
    m = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(m), __float_as_uint(m), false, false);
    return fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

template <typename T, int KSN, bool YOUT = false>
__device__ __forceinline__ void gemm2_body(int bx, int by, const T* __restrict__ U, int KSn,
                                           const T* __restrict__ zfrag, int64_t nfr, int fch, int ncls, int ntile,
                                           const float* __restrict__ zscale, float uinv, float* __restrict__ pmax,
                                           int64_t pstride, float* __restrict__ ycls, int64_t yld,
                                           const int* __restrict__ fmap = nullptr,
                                           const int* __restrict__ fcount = nullptr) {
    constexpr int EPL = Mf<T>::EPL;
    constexpr int NK = KSN > 0 ? KSN : 1;
    typedef typename Vec<T>::t VT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = bx * 4 + wave;
    if (tile >= ntile) return;
    const int rb0 = tile * 4;
    const int64_t fbeg = (int64_t)by * fch;
    const int64_t fend = min<int64_t>(fcount ? (int64_t)*fcount : nfr, fbeg + fch);
    if (fbeg >= fend) return;
    const int64_t fb0 = fbeg >> 4, fbl = (fend - 1) >> 4;  // first and last frame block
    const int nb = (int)(fbl - fb0 + 1);
    // the last tile may hold padding rows, which must not take part
    const bool masked = (tile + 1) * QTILE > ncls;

    VT a[4][NK];
    if constexpr (KSN > 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks)
                a[i][ks] = *reinterpret_cast<const VT*>(U + (((int64_t)(rb0 + i) * KSN + ks) * 64 + lane) * EPL);
    }
    VT bz[2][NK];
    float sc[2];
    auto loadB = [&](int slot, int64_t fb) {
        if constexpr (KSN > 0) {
            const T* zb = zfrag + (fb * KSN * 64 + lane) * EPL;
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks) bz[slot][ks] = *reinterpret_cast<const VT*>(zb + (int64_t)ks * 64 * EPL);
        }
        sc[slot] = zscale[min(fb * 16 + (lane & 15), fend - 1)];
    };
    loadB(0, fb0);
    loadB(1, min(fb0 + 1, fbl));
    if constexpr (KSN > 0) {
#pragma unroll
        for (int sl = 0; sl < 2; ++sl)
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks) asm volatile("" : "+v"(bz[sl][ks]));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks) asm volatile("" : "+v"(a[i][ks]));
    }
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) asm volatile("" : "+v"(sc[sl]));

    for (int i0 = 0; i0 < nb; i0 += 2) {
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
            const int64_t fb = fb0 + i0 + sl;
            if (i0 + sl < nb) {
                f4 acc[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
                if constexpr (KSN > 0) {
#pragma unroll
                    for (int ks = 0; ks < KSN; ++ks)
#pragma unroll
                        for (int i = 0; i < 4; ++i) acc[i] = mfma(a[i][ks], bz[sl][ks], acc[i]);
                } else {
                    const T* zb = zfrag + (fb * KSn * 64 + lane) * EPL;
                    for (int ks = 0; ks < KSn; ++ks) {
                        const VT b = *reinterpret_cast<const VT*>(zb + (int64_t)ks * 64 * EPL);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const VT ai =
                                *reinterpret_cast<const VT*>(U + (((int64_t)(rb0 + i) * KSn + ks) * 64 + lane) * EPL);
                            acc[i] = mfma(ai, b, acc[i]);
                        }
                    }
                }
                // D layout: lane holds rows 4 (lane / 16) + e of column (frame) lane % 16
                const int64_t f = fb * 16 + (lane & 15);
                const float inv = uinv * __builtin_amdgcn_rcpf(sc[sl]);  // both powers of two: exact
                float m = -INFINITY;
                if (!masked) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int e = 0; e < 4; ++e) m = fmaxf(m, acc[i][e]);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if ((rb0 + i) * 16 + 4 * (lane >> 4) + e < ncls) m = fmaxf(m, acc[i][e]);
                }
                m = max_rowgroups(m);
                if (lane < 16 && f < fend) pmax[(fmap ? (int64_t)fmap[f] : f) * pstride + tile] = m * inv;
                if (YOUT && f < fend) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int row = (rb0 + i) * 16 + 4 * (lane >> 4) + e;
                            if (row < ncls) ycls[f * yld + row] = acc[i][e] * inv;
                        }
                }
            }
            loadB(sl, min(fb + 2, fbl));
        }
    }
}

template <typename T, int KSN, bool YOUT = false>
__global__ __launch_bounds__(256) void k_gemm2(const T* __restrict__ U, int KSn, const T* __restrict__ zfrag,
                                               int64_t nfr, int fch, int ncls, int ntile,
                                               const float* __restrict__ zscale, float uinv,
                                               float* __restrict__ pmax, int64_t pstride, float* __restrict__ ycls,
                                               int64_t yld) {
    gemm2_body<T, KSN, YOUT>(blockIdx.x, blockIdx.y, U, KSn, zfrag, nfr, fch, ncls, ntile, zscale, uinv, pmax,
                             pstride, ycls, yld);
}

// GEMM2 over a list of frames: position f of zfrag holds frame fmap[f];
// the count is read on the device.
template <int KSN>
__global__ __launch_bounds__(256) void k_gemm2_list(const _Float16* __restrict__ U, int KSn,
                                                    const _Float16* __restrict__ zfrag, int64_t nmax, int fch,
                                                    int ncls, int ntile, const float* __restrict__ zscale, float uinv,
                                                    float* __restrict__ pmax, int64_t pstride,
                                                    const int* __restrict__ fmap, const int* __restrict__ fcount) {
    gemm2_body<_Float16, KSN>(blockIdx.x, blockIdx.y, U, KSn, zfrag, nmax, fch, ncls, ntile, zscale, uinv, pmax,
                              pstride, nullptr, 0, fmap, fcount);
}

// ------------------------------------------------------------------ final



// y = sum_r U[row, r] zw[r] for one lane's row of a tile of the FP32
// rescoring copy, laid out [tile][Rp/4][QTILE][4] (four consecutive r of a
// row in one 16-byte piece, a wave's pieces for one r/4 in 1 KiB); ut points
// at the lane's first piece.  Batches of NB pieces are issued before their
// FMAs; a small NB keeps the registers of a many-wave kernel down, a larger
// NB puts a whole row in flight where few waves run.  The products go into
// four partial sums by r mod 4, each in increasing r, whatever NB is.
// (Rp is a multiple of 32.)
template <int NB>
__device__ __forceinline__ float row_dot(const float* __restrict__ ut, const float* zw, int Rp) {
    constexpr int SB = NB < 8 ? NB : 8;  // nq is a multiple of 8, so of SB
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const int nq = Rp / 4;
    for (int q0 = 0; q0 < nq; q0 += NB) {
        f4 v[NB];
#pragma unroll
        for (int b = 0; b < NB; b += SB)
            if (q0 + b < nq)
#pragma unroll
                for (int i = b; i < b + SB; ++i) v[i] = *reinterpret_cast<const f4*>(ut + (int64_t)(q0 + i) * (QTILE * 4));
#pragma unroll
        for (int b = 0; b < NB; b += SB)
            if (q0 + b < nq)
#pragma unroll
                for (int i = b; i < b + SB; ++i) {
                    const f4 zv = *reinterpret_cast<const f4*>(zw + 4 * (q0 + i));
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[e] = fmaf(v[i][e], zv[e], acc[e]);
                }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// One wave per frame.  The memory traffic comes in three dependent rounds:
// (1) the frame's tile maxima with their bounds, z and ||z||; (2) for each
// candidate tile, its rows of the FP32 copy of U with their directions and
// classes; (3) the per-microphone delays of the chosen class and the
// frame's STFT values (the power).  Each round's loads are issued together.
// HILO: the hi/lo pass over its frame list, with z the sum of the list
// GEMM1's zp_n partials (zpart) and the first pass's z in z32_first; it runs
// few waves, so every round trip is exposed and the loads are issued as
// early as their addresses are known.
template <int MAXM, bool DEDUP, bool HILO = false>
__device__ __forceinline__ void final_body(int bx, const FinalArgs& a) {
    __shared__ float zs[4][1024];
    // the frame position is wave-uniform: list entries and per-frame scalars
    // come in on scalar loads, apart from the vector loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t n = a.flist ? (int64_t)*a.fcount : a.nfr;
    const int64_t pos = (int64_t)bx * 4 + wave;
    if (pos >= n) return;
    const int Rp = a.Rp, T = a.ntile;
    const bool r128 = Rp <= 128;
    // HILO: the partial slots of this list position (run k = Rp floats at
    // zpart + k * zp_stride + pos * Rp) depend on the position only, so they
    // are issued before the frame index arrives: up to 16 16-byte pieces per
    // lane, later staged in LDS and summed per row in slot order
    constexpr int ZQ = HILO ? 16 : 1;
    __shared__ float zpl[HILO ? 4 : 1][HILO ? 64 * 4 * ZQ : 1];
    const int nq = Rp / 4, nitem = a.zp_n * nq;
    const bool zlist = HILO && r128 && nitem <= 64 * ZQ;
    f4 zq[ZQ];
    int zit[ZQ];
    if constexpr (HILO) {
        const float rnq = __builtin_amdgcn_rcpf((float)nq);
#pragma unroll
        for (int i = 0; i < ZQ; ++i) {
            // piece it = (run k, 16-byte column j), clamped into range (the
            // clamped copies are loaded but not used); the +0.5 keeps the
            // float quotient at least 1/64 clear of integers, so truncating
            // it is exact
            const int it = min(lane + 64 * i, nitem - 1);
            const int k = (int)(((float)it + 0.5f) * rnq), j = it - k * nq;
            zit[i] = it;
            zq[i] = *reinterpret_cast<const f4*>(a.zpart + (int64_t)k * a.zp_stride + pos * Rp + 4 * j);
        }
    }
    const int64_t f = a.flist ? (int64_t)a.flist[pos] : pos;
    const float* pm = a.pmax + f * a.pstride;

    // ---- stage 1: frame maximum over tiles, the tile holding it and that
    // tile's bound (carried through the reduction), z into LDS
    float ym = -INFINITY, km = 0.f;
    int tm = 0x7fffffff;
    // z of up to 128 rows is loaded with the tile maxima, so both arrive
    // in one round trip
    const float* z = a.z32 + pos * Rp;
    const bool zfast = !HILO && r128;
    float zpre[2] = {0.f, 0.f}, zf[2] = {0.f, 0.f};
    if (zfast) {
        zpre[0] = z[min(lane, Rp - 1)];
        zpre[1] = z[min(lane + 64, Rp - 1)];
    }
    if (HILO && r128 && a.z32_first) {
        zf[0] = a.z32_first[f * Rp + min(lane, Rp - 1)];
        zf[1] = a.z32_first[f * Rp + min(lane + 64, Rp - 1)];
    }
    for (int t0 = 0; t0 < T; t0 += 256) {
        float pv[4], kv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = t0 + lane + 64 * j;
            pv[j] = pm[t < T ? t : 0];
            kv[j] = a.tkappa[t < T ? t : 0];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = t0 + lane + 64 * j;
            if (t < T && better(pv[j], t, ym, tm)) {
                ym = pv[j];
                tm = t;
                km = kv[j];
            }
        }
    }
    // the partial slots through LDS, each row summed in slot order
    if constexpr (HILO) {
        if (zlist) {
            float* zl = zpl[wave];
#pragma unroll
            for (int i = 0; i < ZQ; ++i) *reinterpret_cast<f4*>(zl + 4 * zit[i]) = zq[i];  // copies: same value
            wave_sync();
            const int l0 = min(lane, Rp - 1), l1 = min(lane + 64, Rp - 1);
            for (int k = 0; k < a.zp_n; ++k) {
                zpre[0] += zl[k * Rp + l0];
                zpre[1] += zl[k * Rp + l1];
            }
        }
    }
    float* zw = zs[wave];
    float dz2 = 0.f;
    for (int r = lane; r < Rp; r += 64) {
        float v = 0.f;
        if (zfast || zlist) {
            v = r == lane ? zpre[0] : zpre[1];
        } else if (HILO) {
            // the GEMM1 partial sums of this list position, eight in flight
            for (int s0 = 0; s0 < a.zp_n; s0 += 8) {
                float part[8];
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    part[s] = s0 + s < a.zp_n ? a.zpart[(int64_t)(s0 + s) * a.zp_stride + pos * Rp + r] : 0.f;
#pragma unroll
                for (int s = 0; s < 8; ++s) v += part[s];
            }
        } else {
            v = z[r];
        }
        zw[r] = v;
        if (HILO && a.z32_first) {
            const float d = v - (r128 ? (r == lane ? zf[0] : zf[1]) : a.z32_first[f * Rp + r]);
            dz2 += d * d;
        }
    }
    const float ef = a.ecoef * a.znorm1[f] + (HILO && a.z32_first ? 1.01f * sqrtf(wave_sum(dz2)) : 0.f);
    {
        // (maximum, its tile, the tile's bound) over the wave
        uint32_t v[3] = {__float_as_uint(ym), (uint32_t)tm, __float_as_uint(km)};
        wave_reduce(v, [](uint32_t (&x)[3], const uint32_t (&o)[3]) {
            const bool ob = better(__uint_as_float(o[0]), (int)o[1], __uint_as_float(x[0]), (int)x[1]);
#pragma unroll
            for (int i = 0; i < 3; ++i) x[i] = blend(x[i], o[i], ob);
        });
        ym = __uint_as_float(v[0]);
        tm = (int)v[1];
        km = __uint_as_float(v[2]);
    }
    wave_sync();
    const float thr = a.rescore ? ym - km * ef : ym;

    // ---- stage 2: rescore the candidate tiles in FP32: best (y1, q1, r1,
    // class c1) and runner-up (y2, q2, r2)
    float y1 = -INFINITY, y2 = -INFINITY, ncmax = -INFINITY;
    int q1 = 0x7fffffff, q2 = 0x7fffffff, r1 = -1, r2 = -1, c1 = 0;
    int ncand = 0;
    for (int t0 = 0; t0 < T; t0 += 64) {
        const int t = t0 + lane;
        const float et = t < T ? (a.rescore ? a.tkappa[t] * ef : 0.f) : 0.f;
        const float pv = t < T ? pm[t] : -INFINITY;
        const bool cand = pv + et >= thr;
        if (!cand) ncmax = fmaxf(ncmax, pv + et);
        uint64_t mask = __ballot(cand);
        ncand += __popcll(mask);
        while (mask) {
            const int tt = t0 + __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int row = tt * QTILE + lane;
            const int q = a.rows[row < a.ncls ? row : 0];
            const int c = a.rowcls[row];
            const float* ut = a.U32T + (int64_t)tt * Rp * QTILE + 4 * lane;
            const float y = HILO && r128 ? row_dot<32>(ut, zw, Rp) : row_dot<4>(ut, zw, Rp);
            if (row < a.ncls) {
                if (better(y, q, y1, q1)) {
                    if (DEDUP) {
                        y2 = y1;
                        q2 = q1;
                        r2 = r1;
                    }
                    y1 = y;
                    q1 = q;
                    r1 = row;
                    c1 = c;
                } else if (DEDUP && better(y, q, y2, q2)) {
                    y2 = y;
                    q2 = q;
                    r2 = row;
                }
            }
        }
    }
    // wave-wide best and (scored rows being distinct classes) runner-up:
    // merging two (best, runner-up) pairs is commutative, as the butterfly
    // of wave_reduce needs
    {
        uint32_t v[7] = {__float_as_uint(y1), (uint32_t)q1, (uint32_t)r1, (uint32_t)c1,
                         __float_as_uint(y2), (uint32_t)q2, (uint32_t)r2};
        wave_reduce(v, [](uint32_t (&x)[7], const uint32_t (&o)[7]) {
            // selects only (no branches), so the words stay in registers
            const float xy1 = __uint_as_float(x[0]), oy1 = __uint_as_float(o[0]);
            const float xy2 = __uint_as_float(x[4]), oy2 = __uint_as_float(o[4]);
            const bool ob = better(oy1, (int)o[1], xy1, (int)x[1]);  // the other best wins
            // runner-up: if the other best wins, the better of this best and
            // the other runner-up; else the better of this runner-up and the
            // other best
            const bool s_x1 = DEDUP && better(xy1, (int)x[1], oy2, (int)o[5]);
            const bool s_o1 = DEDUP && better(oy1, (int)o[1], xy2, (int)x[5]);
            uint32_t n[7];
#pragma unroll
            for (int i = 0; i < 4; ++i) n[i] = blend(x[i], o[i], ob);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                n[4 + i] = !DEDUP ? x[4 + i]
                                  : blend(blend(x[4 + i], o[i], s_o1), blend(o[4 + i], x[i], s_x1), ob);
#pragma unroll
            for (int i = 0; i < 7; ++i) x[i] = n[i];
        });
        y1 = __uint_as_float(v[0]);
        q1 = (int)v[1];
        r1 = (int)v[2];
        c1 = (int)v[3];
        y2 = __uint_as_float(v[4]);
        q2 = (int)v[5];
        r2 = (int)v[6];
    }
    if (q1 < 0 || q1 == 0x7fffffff) {  // no finite candidate
        q1 = a.rows[0];
        r1 = 0;
        c1 = a.rowcls[0];
    }
    const int cls = c1;
    if (!DEDUP) {
        // runner-up over directions of other classes among the candidates
        float sy = -INFINITY;
        int sr = -1;
        for (int t0 = 0; t0 < T; t0 += 64) {
            const int t = t0 + lane;
            const float et = t < T ? (a.rescore ? a.tkappa[t] * ef : 0.f) : 0.f;
            const float pv = t < T ? pm[t] : -INFINITY;
            uint64_t mask = __ballot(pv + et >= thr);
            while (mask) {
                const int tt = t0 + __ffsll((unsigned long long)mask) - 1;
                mask &= mask - 1;
                const int row = tt * QTILE + lane;
                if (row < a.ncls && a.rowcls[row] != cls) {
                    const float* ut = a.U32T + (int64_t)tt * Rp * QTILE + 4 * lane;
                    const float y = HILO && r128 ? row_dot<32>(ut, zw, Rp) : row_dot<4>(ut, zw, Rp);
                    if (y > sy) {
                        sy = y;
                        sr = row;
                    }
                }
            }
        }
        {
            uint32_t v[2] = {__float_as_uint(sy), (uint32_t)sr};
            wave_reduce(v, [](uint32_t (&x)[2], const uint32_t (&o)[2]) {
                const float xy = __uint_as_float(x[0]), oy = __uint_as_float(o[0]);
                const bool ob = oy > xy || (oy == xy && (int)o[1] < (int)x[1]);
#pragma unroll
                for (int i = 0; i < 2; ++i) x[i] = blend(x[i], o[i], ob);
            });
            sy = __uint_as_float(v[0]);
            sr = (int)v[1];
        }
        y2 = sy;
        r2 = sr;
    }
    ncmax = wave_max(ncmax);
    const float yr = fmaxf(y2, ncmax);
    const float mg = (y1 - yr) / fmaxf(fabsf(y1), FLT_MIN);

    // hi/lo trigger (first pass): GEMM1 rounding perturbs z_r by about u
    // sigma_r (random signs), so y1 - y2 moves by about u ||(U_q1 - U_q2)
    // sigma||; frames whose rescored gap is within hilo_k times that are
    // redone.  ||(U_q1 - U_q2) sigma|| <= 2 max_q ||U_q sigma|| decides most
    // frames without loading the two rows.
    bool redo = false;
    if (!HILO && a.hlist && !a.flist && (y1 - yr) < a.hilo_k * a.u * 2.f * a.usig_max) {
        float d2 = 0.f;
        if (r2 >= 0 && y2 >= ncmax) {
            const float* u1 = a.U32T + (int64_t)(r1 / QTILE) * Rp * QTILE + 4 * (r1 % QTILE);
            const float* u2 = a.U32T + (int64_t)(r2 / QTILE) * Rp * QTILE + 4 * (r2 % QTILE);
            for (int r = lane; r < Rp; r += 64) {
                const int64_t o = (int64_t)(r / 4) * (QTILE * 4) + r % 4;
                const float d = (u1[o] - u2[o]) * a.sig[r];
                d2 += d * d;
            }
            d2 = wave_sum(d2);
        } else {
            // runner-up not rescored: bound with the largest row difference
            d2 = 4.f * a.usig_max * a.usig_max;
        }
        redo = (y1 - yr) < a.hilo_k * a.u * sqrtf(d2);
    }
    if (!HILO && a.hlist && !a.flist && a.hilo_all) redo = true;

    // ---- stage 3 (when the power is not left to k_power): Algorithm 1
    // online step 4, the power of the chosen direction from its row of W
    // (delay-and-sum form)
    // (MAXM = 0: no power here, which keeps the register count and so the
    // number of frames in flight up)
    float acc = 0.f;
    if constexpr (MAXM > 0) {
        if (a.power) {
            float t[MAXM];
#pragma unroll
            for (int m = 0; m < MAXM; ++m) t[m] = m < a.M ? a.tauM[(int64_t)cls * a.M + m] : 0.f;
            acc = power_ds<MAXM>(a.X + f * a.M * a.B, a.M, a.B, t, lane);
        }
    }
    if (lane == 0) {
        a.doa[f] = cls;
        if (a.power) a.power[f] = acc;
        if (a.yhat) a.yhat[f] = y1;
        if (a.margin) a.margin[f] = mg;
        if (redo) {
            const int k = atomicAdd(a.hcount, 1);
            a.hlist[k] = (int)f;
        }
        if (a.stats) {
            atomicAdd(a.stats, (unsigned long long)ncand);
            if (redo) atomicAdd(a.stats + 1, 1ull);
        }
    }
}

template <int MAXM, bool DEDUP>
__global__ __launch_bounds__(256) void k_final(FinalArgs a) {
    final_body<MAXM, DEDUP>(blockIdx.x, a);
}


// the same without the power (k_power computes it afterwards): few enough
// registers (rows rescored four pieces at a time) for eight waves per SIMD,
// so more frames' dependent loads overlap; that beats fewer, larger load
// rounds per candidate tile at fewer waves
template <bool DEDUP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_final_np(FinalArgs a) {
    final_body<0, DEDUP>(blockIdx.x, a);
}

// the hi/lo pass over its device-counted frame list, grid-stride (few
// frames)
template <int MAXM, bool DEDUP>
__global__ __launch_bounds__(256) void k_final_list(FinalArgs a) {
    const int64_t n = *a.fcount;
    for (int64_t bx = blockIdx.x; bx * 4 < n; bx += gridDim.x) final_body<MAXM, DEDUP, true>((int)bx, a);
}


// Algorithm 1 online step 4 for every frame once the search is final: the
// power of direction doa[f] from its row of W (delay-and-sum form).  One
// wave per frame; the frame, its direction and the direction's delays are
// wave-uniform (scalar loads), so the STFT loads are the only vector loads.
// (With flist, the frames flist[0 .. *fcount), grid-stride.  MK: mask
// [nfr][B], a dropped bin contributes nothing.)
template <int MAXM, bool MK>
__global__ __launch_bounds__(256) void k_power(const float2* __restrict__ X, int M, int B,
                                               const int32_t* __restrict__ doa, const float* __restrict__ tauM,
                                               int64_t nfr, float* __restrict__ power,
                                               const int* __restrict__ flist, const int* __restrict__ fcount,
                                               const uint8_t* __restrict__ mask) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t n = fcount ? (int64_t)*fcount : nfr;
    for (int64_t pos = (int64_t)blockIdx.x * 4 + wave; pos < n; pos += (int64_t)gridDim.x * 4) {
        const int64_t f = flist ? (int64_t)__builtin_amdgcn_readfirstlane(flist[pos]) : pos;
        const int q = __builtin_amdgcn_readfirstlane(doa[f]);
        float t[MAXM];
#pragma unroll
        for (int m = 0; m < MAXM; ++m) t[m] = m < M ? tauM[(int64_t)q * M + m] : 0.f;
        const float acc = power_ds<MAXM, MK>(X + f * M * B, M, B, t, lane, MK ? mask + f * B : nullptr);
        if (lane == 0) power[f] = acc;
    }
}

template <bool MK>
void launch_power_t(const svdphat_plan* p, const float2* X, const int32_t* doa, int64_t F, float* power,
                    const int* flist, const int* fcount, const uint8_t* mask, hipStream_t s) {
    const dim3 grid(flist ? 512u : (unsigned)((F + 3) / 4));
    const int M = p->M, B = p->B;
    const float* tau = p->d_tauM_all;
    // the exact microphone count where it is common (no padded microphone's
    // loads, fewer registers)
    if (M == 6) k_power<6, MK><<<grid, 256, 0, s>>>(X, M, B, doa, tau, F, power, flist, fcount, mask);
    else if (M == 7) k_power<7, MK><<<grid, 256, 0, s>>>(X, M, B, doa, tau, F, power, flist, fcount, mask);
    else if (M <= 8) k_power<8, MK><<<grid, 256, 0, s>>>(X, M, B, doa, tau, F, power, flist, fcount, mask);
    else k_power<16, MK><<<grid, 256, 0, s>>>(X, M, B, doa, tau, F, power, flist, fcount, mask);
}

void launch_power(const svdphat_plan* p, const float2* X, const int32_t* doa, int64_t F, float* power,
                  const int* flist, const int* fcount, hipStream_t s, const uint8_t* mask) {
    if (mask) launch_power_t<true>(p, X, doa, F, power, flist, fcount, mask, s);
    else launch_power_t<false>(p, X, doa, F, power, flist, fcount, nullptr, s);
}

// ------------------------------------------------------------------ grouped
// Ragged batches: one launch per stage and template class walks a device
// work list of (array, x, y, z) items; each item runs the same body as the
// single-plan kernel with that array's descriptor (FP16 operands).
template <int NRB, int MAXM, int IPT>
__global__ __launch_bounds__(256) void k_gemm1_grouped(const RDesc* __restrict__ d, const int4* __restrict__ work) {
    const int4 w = work[blockIdx.x];
    if (w.x < 0) return;  // padding of the XCD queues
    const RDesc& a = d[w.x];
    gemm1_body<_Float16, 64, NRB, MAXM, IPT, false>(w.y, w.z, w.w, a.X, a.F, a.M, a.P, a.B,
                                                    (const _Float16*)a.A, nullptr, a.nRB, a.BB, a.CW, a.nch, a.cps,
                                                    a.zpart, a.zstride, a.Rp, nullptr, nullptr);
}

__global__ __launch_bounds__(256) void k_zprep_grouped(const RDesc* __restrict__ d, const int4* __restrict__ work) {
    const int4 w = work[blockIdx.x];
    const RDesc& a = d[w.x];
    zprep_body<_Float16>(w.y, a.zpart, a.nsplit, a.zstride, a.F, nullptr, a.Rp, a.z32, (_Float16*)a.zfrag, a.zsc,
                         a.zn, 1);
}

template <int KSN>
__global__ __launch_bounds__(256) void k_gemm2_grouped(const RDesc* __restrict__ d, const int4* __restrict__ work) {
    const int4 w = work[blockIdx.x];
    const RDesc& a = d[w.x];
    gemm2_body<_Float16, KSN>(w.y, w.z, (const _Float16*)a.U, a.KSn, (const _Float16*)a.zfrag, a.F, a.fch,
                                    a.ncls, a.ntile, a.zsc, a.uinv, a.pmax, a.pstride, nullptr, 0);
}

template <int MAXM>
__global__ __launch_bounds__(256) void k_final_grouped(const RDesc* __restrict__ d, const int4* __restrict__ work) {
    const int4 w = work[blockIdx.x];
    const RDesc& a = d[w.x];
    final_body<MAXM, true>(w.y, a.fin);
}

// synthetic STFT values for the tuner (any finite values do)
__global__ void k_fill_synth(float2* X, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)(i * 2654435761u) ^ 0x9e3779b9u;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    X[i] = float2{(float)(h & 0xffff) / 32768.f - 1.f, (float)(h >> 16) / 32768.f - 1.f};
}

// y_opt: every direction takes the value of its scored row
__global__ void k_scatter_y(const float* __restrict__ ycls, int64_t yld, const int32_t* __restrict__ rowof, int Q,
                            int64_t nfr, float* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nfr * Q) return;
    const int64_t f = i / Q;
    const int q = (int)(i % Q);
    y[i] = ycls[f * yld + rowof[q]];
}

inline double unit_roundoff(int prec) {
    return prec == P_FP32 ? std::ldexp(1.0, -24) : prec == P_FP16 ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
}

// ------------------------------------------------------------------ launch

// Split of GEMM1's reduction axis: `want` splits (0: enough workgroups for
// about four per CU), rounded so that every split gets the same chunk count.
void g1_split_layout(const G1Layout& g, int Rp, int64_t F, int want, int* nsplit, int* cps) {
    const int ftiles = (int)(round_up64(F, 64) / 64);
    const int nrg = cdiv(Rp / 16, 12);
    int ns = want > 0 ? want : std::max(1, std::min(8, cdiv(1024, ftiles * nrg)));
    ns = std::max(1, std::min(ns, g.nch));
    const int c = cdiv(g.nch, ns);
    *cps = c;
    *nsplit = cdiv(g.nch, c);
}

template <typename T, int NF, bool HILO, int NRB>
void launch_g1_nrb(dim3 grid, size_t lds, hipStream_t s, int M, const float2* X, int64_t F, svdphat_plan* p,
                   int prec, const G1Layout& g, int cps, float* zpart, int64_t zstride, const int* fl,
                   const int* fc) {
    const int nRB = p->Rp / 16;
    const T* A = (const T*)p->A[prec];
    const T* Alo = (const T*)p->Alo[prec];
    if (NF * g.BB > 256 * (M <= 8 ? G1_IPT8 : G1_IPT16))
        fail(SVDPHAT_E_UNSUPPORTED, "GEMM1 chunk larger than the workgroup's item budget");
    if (M <= 8)
        k_gemm1<T, NF, NRB, 8, G1_IPT8, HILO><<<grid, 256, lds, s>>>(X, F, M, p->P, p->B, A, Alo, nRB, g.BB, g.CW,
                                                                     g.nch, cps, zpart, zstride, p->Rp, fl, fc);
    else
        k_gemm1<T, NF, NRB, 16, G1_IPT16, HILO><<<grid, 256, lds, s>>>(X, F, M, p->P, p->B, A, Alo, nRB, g.BB, g.CW,
                                                                       g.nch, cps, zpart, zstride, p->Rp, fl, fc);
}

template <typename T, int NF, bool HILO>
int launch_g1(int ftiles, int nsplit, hipStream_t s, const float2* X, int64_t F, svdphat_plan* p, int prec,
              const G1Layout& g, int cps, float* zpart, int64_t zstride, const int* fl, const int* fc) {
    const int nRB = p->Rp / 16;
    const int nrbw = nRB <= 12 ? nRB : 12;
    const int NRB = nrbw <= 2 ? 2 : nrbw <= 4 ? 4 : nrbw <= 6 ? 6 : nrbw <= 8 ? 8 : nrbw <= 10 ? 10 : 12;
    dim3 grid(ftiles, nsplit, cdiv(nRB, NRB));
    const size_t xbytes = (size_t)(HILO ? 2 : 1) * NF * (g.CW + XPAD) * sizeof(T);
    const size_t rbytes = (size_t)NRB * (NF / 16) * 64 * sizeof(f4);
    const size_t lds = std::max(xbytes, rbytes);
    switch (NRB) {
        case 2: launch_g1_nrb<T, NF, HILO, 2>(grid, lds, s, p->M, X, F, p, prec, g, cps, zpart, zstride, fl, fc); break;
        case 4: launch_g1_nrb<T, NF, HILO, 4>(grid, lds, s, p->M, X, F, p, prec, g, cps, zpart, zstride, fl, fc); break;
        case 6: launch_g1_nrb<T, NF, HILO, 6>(grid, lds, s, p->M, X, F, p, prec, g, cps, zpart, zstride, fl, fc); break;
        case 8: launch_g1_nrb<T, NF, HILO, 8>(grid, lds, s, p->M, X, F, p, prec, g, cps, zpart, zstride, fl, fc); break;
        case 10: launch_g1_nrb<T, NF, HILO, 10>(grid, lds, s, p->M, X, F, p, prec, g, cps, zpart, zstride, fl, fc); break;
        default: launch_g1_nrb<T, NF, HILO, 12>(grid, lds, s, p->M, X, F, p, prec, g, cps, zpart, zstride, fl, fc); break;
    }
    return NRB;
}

// frames per GEMM2 workgroup: about one wave per 4096 (tile, 16-frame
// block) pairs, so the grid is about one round of four waves per SIMD
int g2_frames(int ntile, int64_t F) {
    const int64_t blocks = (int64_t)ntile * ((F + 15) / 16);
    const int64_t per = std::max<int64_t>(1, (blocks + 4095) / 4096);
    return (int)std::min<int64_t>(16 * per, 4096);
}

template <typename T>
void launch_g2(svdphat_plan* p, const ScoreRows& sr, int prec, const T* zfrag, int64_t F, const float* zsc,
               float* pmax, int64_t pstride, float* ycls, hipStream_t s) {
    constexpr int KS = Mf<T>::KSTEP;
    const int KSn = p->Rp / KS;
    const int ntile = p->ncls_pad / QTILE;
    const int fch = g2_frames(ntile, F);
    dim3 grid(cdiv(ntile, 4), (unsigned)((F + fch - 1) / fch));
    const float uinv = 1.f / sr.uscale[prec];
    const T* U = (const T*)sr.Ufr[prec];
    if (ycls) {
        // every reduced power as well (debugging output): general form
        k_gemm2<T, 0, true><<<grid, 256, 0, s>>>(U, KSn, zfrag, F, fch, p->ncls, ntile, zsc, uinv, pmax, pstride, ycls,
                                                 p->ncls_pad);
        return;
    }
#define SP_G2(N) k_gemm2<T, N><<<grid, 256, 0, s>>>(U, KSn, zfrag, F, fch, p->ncls, ntile, zsc, uinv, pmax, pstride, \
                                                    nullptr, p->ncls_pad)
    // U fragments of the tile stay in registers when they fit (<= 96 VGPRs)
    if constexpr (sizeof(T) == 2) {
        switch (KSn) {
            case 1: SP_G2(1); return;
            case 2: SP_G2(2); return;
            case 3: SP_G2(3); return;
            case 4: SP_G2(4); return;
            case 5: SP_G2(5); return;
            case 6: SP_G2(6); return;
        }
    } else {
        switch (KSn) {
            case 8: SP_G2(8); return;
            case 16: SP_G2(16); return;
            case 24: SP_G2(24); return;
        }
    }
    SP_G2(0);
#undef SP_G2
}

void launch_final(const FinalArgs& fa, int M, bool dedup, int64_t nwaves, hipStream_t s) {
    dim3 grid((unsigned)((nwaves + 3) / 4));
    if (!fa.power) {
        if (dedup) k_final_np<true><<<grid, 256, 0, s>>>(fa);
        else k_final_np<false><<<grid, 256, 0, s>>>(fa);
    } else if (M <= 8) {
        if (dedup) k_final<8, true><<<grid, 256, 0, s>>>(fa);
        else k_final<8, false><<<grid, 256, 0, s>>>(fa);
    } else {
        if (dedup) k_final<16, true><<<grid, 256, 0, s>>>(fa);
        else k_final<16, false><<<grid, 256, 0, s>>>(fa);
    }
}


// hi/lo pass over the device-counted frame list (32 frames per workgroup)
template <typename T>
void launch_g1_list(hipStream_t s, const float2* X, svdphat_plan* p, int prec, const G1Layout& g, int nsplit, int cps,
                    float* zpart, int64_t zstride, const int* fl, const int* fc) {
    const int nRB = p->Rp / 16;
    const int NRB = nRB <= 2 ? 2 : nRB <= 4 ? 4 : nRB <= 6 ? 6 : nRB <= 8 ? 8 : nRB <= 10 ? 10 : 12;
    // grid-stride over (frame tile, split) items of the short device-counted
    // list: one workgroup per CU
    dim3 grid(cu_count(p->device), 1, cdiv(nRB, NRB));
    const size_t xbytes = (size_t)2 * 32 * (g.CW + XPAD) * sizeof(T);
    const size_t lds = std::max(xbytes, (size_t)3 * NRB * 2 * 64 * sizeof(f4));  // three waves' partial sums
    const T* A = (const T*)p->A[prec];
    const T* Alo = (const T*)p->Alo[prec];
    const int M = p->M;
#define SP_G1L(N)                                                                                                   \
    if (NRB == N) {                                                                                                 \
        if (M <= 8)                                                                                                 \
            k_gemm1_list<T, 32, N, 8, G1_IPT8, true><<<grid, 256, lds, s>>>(X, M, p->P, p->B, A, Alo, nRB, g.BB,    \
                                                                            g.CW, g.nch, cps, nsplit, zpart,       \
                                                                            zstride, p->Rp, fl, fc);               \
        else                                                                                                        \
            k_gemm1_list<T, 32, N, 16, G1_IPT16, true><<<grid, 256, lds, s>>>(X, M, p->P, p->B, A, Alo, nRB, g.BB,  \
                                                                              g.CW, g.nch, cps, nsplit, zpart,     \
                                                                              zstride, p->Rp, fl, fc);             \
        return;                                                                                                     \
    }
    SP_G1L(2) SP_G1L(4) SP_G1L(6) SP_G1L(8) SP_G1L(10) SP_G1L(12)
#undef SP_G1L
}

void launch_final_list(const FinalArgs& fa, int M, bool dedup, hipStream_t s) {
    // grid-stride over the device-counted list, which is short
    dim3 grid(64);
    if (!fa.power) {
        if (dedup) k_final_list<0, true><<<grid, 256, 0, s>>>(fa);
        else k_final_list<0, false><<<grid, 256, 0, s>>>(fa);
    } else if (M <= 8) {
        if (dedup) k_final_list<8, true><<<grid, 256, 0, s>>>(fa);
        else k_final_list<8, false><<<grid, 256, 0, s>>>(fa);
    } else {
        if (dedup) k_final_list<16, true><<<grid, 256, 0, s>>>(fa);
        else k_final_list<16, false><<<grid, 256, 0, s>>>(fa);
    }
}

template <typename T>
void run_locate(svdphat_plan* p, const float2* X, int64_t F, int prec, uint32_t mode, int32_t* doa, float* power,
                float* yhat, float* margin, float* y_opt, hipStream_t s, void* scratch, size_t scratch_bytes,
                const uint8_t* mask, float2* xm) {
    const G1Layout& g = p->g1[prec];
    const int Rp = p->Rp;
    const int ntile = p->ncls_pad / QTILE;
    const int64_t Fc = round_up64(F, 64);
    const int ftiles = (int)(Fc / 64);
    int nsplit, cps;
    g1_split_layout(g, Rp, F, 0, &nsplit, &cps);
    G1Sched sc;
    const bool streamed = g1s_sched(prec, p, F, &sc);
    const int zslots = streamed ? sc.slots : nsplit;
    const bool hilo = (mode & (SVDPHAT_HILO | SVDPHAT_HILO_ALL)) && prec != P_FP32;
    // a mask is applied by the streamed GEMM1's producers, the hi/lo pass
    // (on masked copies of its listed frames, in xm) and the power
    SP_REQUIRE(!mask || (streamed && (!hilo || xm)), SVDPHAT_E_UNSUPPORTED, "masked search without its streamed form");
    // the hi/lo pass covers few frames: more splits keep the grid busy
    int hsplit = g.nch, hcps = 1;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += round_up64((int64_t)bytes, 256);
        return o;
    };
    const int maxsplit = std::max(zslots, hilo ? hsplit : 1);
    const size_t o_zpart = take(sizeof(float) * maxsplit * Fc * Rp);
    const size_t o_z32 = take(sizeof(float) * Fc * Rp);
    const size_t o_zfrag = take(sizeof(T) * Fc * Rp);
    const size_t o_zsc = take(sizeof(float) * Fc);
    const size_t o_zn = take(sizeof(float) * Fc);
    const int ntp = pmax_stride(p);
    const size_t o_pmax = take(sizeof(float) * ntp * Fc);
    const size_t o_hl = hilo ? take(sizeof(int) * Fc) : 0;
    const size_t o_hc = hilo ? take(sizeof(int) * 64) : 0;
    const size_t o_y = y_opt ? take(sizeof(float) * Fc * p->ncls_pad) : 0;
    const size_t o_st = take(sizeof(unsigned long long) * 4);
    // the caller's scratch buffer (checked before anything is enqueued), or
    // the plan's workspace of this stream
    if (scratch)
        SP_REQUIRE(off <= scratch_bytes, SVDPHAT_E_INVAL,
                   "this call needs " + std::to_string(off) + " bytes of scratch memory, more than the " +
                       std::to_string(scratch_bytes) + " available: split the frames into smaller calls");
    char* w = scratch ? (char*)scratch : (char*)ws_get(p, s, off);
    unsigned long long* stats = counting_on() ? (unsigned long long*)(w + o_st) : nullptr;
    if (stats) zero_async(stats, sizeof(unsigned long long) * 4, s);
    float* zpart = (float*)(w + o_zpart);
    float* z32 = (float*)(w + o_z32);
    T* zfrag = (T*)(w + o_zfrag);
    float* zsc = (float*)(w + o_zsc);
    float* zn = (float*)(w + o_zn);
    float* pmax = (float*)(w + o_pmax);
    float* ycls = y_opt ? (float*)(w + o_y) : nullptr;
    int* hl = hilo ? (int*)(w + o_hl) : nullptr;
    int* hc = hilo ? (int*)(w + o_hc) : nullptr;
    // (the GEMM2 operand's padding frames feed only padding columns, whose
    // results are never written)
    // (hc, the hi/lo list count, is cleared by the Z preparation kernel)

    const int64_t zstride = Fc * Rp;
    KernelTimer kt(s);
    kt.begin("gemm1");
    if (streamed) launch_g1_streamed(prec, p, sc, X, F, zpart, zstride, s, mask);
    else launch_g1<T, 64, false>(ftiles, nsplit, s, X, F, p, prec, g, cps, zpart, zstride, nullptr, nullptr);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("zprep");
    if constexpr (sizeof(T) == 2) {
        if (Rp <= 128)
            k_zprep16<T><<<dim3((unsigned)((F + 15) / 16)), 256, 0, s>>>(zpart, zslots, zstride, F, Rp, z32, zfrag, zsc,
                                                                    zn, prec == P_FP16 ? 1 : 0,
                                                                    streamed ? sc.G : 0, sc.U, sc.nch, hc);
        else
            k_zprep<T><<<dim3((unsigned)(Fc / 4)), 256, 0, s>>>(zpart, zslots, zstride, F, nullptr, Rp, z32, zfrag,
                                                                zsc, zn, prec == P_FP16 ? 1 : 0,
                                                                streamed ? sc.G : 0, sc.U, sc.nch, hc);
    } else {
        k_zprep<T><<<dim3((unsigned)(Fc / 4)), 256, 0, s>>>(zpart, zslots, zstride, F, nullptr, Rp, z32, zfrag, zsc,
                                                            zn, 0, streamed ? sc.G : 0, sc.U, sc.nch, hc);
    }
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("gemm2");
    // eq. (14) searches the rows of U, eq. (15) the rows of U / ||U sigma||
    const ScoreRows& sr = p->sr[(mode & SVDPHAT_NORMALIZED) ? 1 : 0];
    launch_g2<T>(p, sr, prec, zfrag, F, zsc, pmax, ntp, ycls, s);
    SP_HIP(hipGetLastError());
    kt.end();
    if (y_opt) {
        kt.begin("scatter_y");
        const int64_t tot = F * p->Q;
        k_scatter_y<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>(ycls, p->ncls_pad, p->d_rowof, p->Q, F, y_opt);
        SP_HIP(hipGetLastError());
        kt.end();
    }
    // eps of a tile = kappa_t (2u + u^2 + 2 Rp 2^-24) ||z|| bounds |y_lowprec -
    // y_fp32| for its rows (operand rounding of U and z, FP32 accumulation of
    // both products; Cauchy-Schwarz with the tile's largest ||U_q||)
    const double u = unit_roundoff(prec);
    const double accum = 2.0 * Rp * std::ldexp(1.0, -24);
    const double lin = prec == P_FP32 ? accum : (2.0 * u + u * u + accum);
    FinalArgs fa{};
    fa.X = X;
    fa.M = p->M;
    fa.P = p->P;
    fa.B = p->B;
    fa.pmax = pmax;
    fa.pstride = ntp;
    fa.ntile = ntile;
    fa.ncls = p->ncls;
    fa.z32 = z32;
    fa.z32_first = nullptr;
    fa.znorm1 = zn;
    fa.Rp = Rp;
    fa.ecoef = (float)(lin * 1.01);
    fa.rescore = (mode & SVDPHAT_RESCORE) ? 1 : 0;
    fa.U32T = sr.U32T;
    fa.tkappa = sr.tkappa;
    fa.sig = p->d_sig;
    fa.rows = p->d_rows;
    fa.rep = p->d_rep;
    fa.tauN = p->d_tauN_all;
    fa.tauM = p->d_tauM_all;
    fa.rowcls = p->d_rowcls;
    fa.usig_max = sr.usig_max;
    fa.nfr = F;
    fa.doa = doa;
    fa.power = nullptr;  // k_power below, after the hi/lo pass
    fa.yhat = yhat;
    fa.margin = margin;
    fa.hilo_k = 4.f;
    fa.hilo_all = (mode & SVDPHAT_HILO_ALL) ? 1 : 0;
    fa.u = (float)u;
    fa.hlist = hl;
    fa.hcount = hc;
    fa.stats = stats;
    const bool dedup = !(p->flags & SVDPHAT_NO_DEDUP);
    kt.begin("final");
    launch_final(fa, p->M, dedup, F, s);
    SP_HIP(hipGetLastError());
    kt.end();
    if (hilo) {
        kt.begin("gemm1_hilo");
        if (mask) launch_mask_list(p, X, mask, hl, hc, xm, s);
        launch_g1_list<T>(s, mask ? xm : X, p, prec, g, hsplit, hcps, zpart, zstride, hl, hc);
        SP_HIP(hipGetLastError());
        kt.end();
        FinalArgs fb = fa;
        fb.z32 = nullptr;
        fb.zpart = zpart;  // z of the list positions summed in the rescoring kernel
        fb.zp_n = hsplit;
        fb.zp_stride = zstride;
        fb.z32_first = z32;
        fb.flist = hl;
        fb.fcount = hc;
        fb.hlist = nullptr;
        fb.stats = nullptr;
        kt.begin("final_hilo");
        launch_final_list(fb, p->M, dedup, s);
        SP_HIP(hipGetLastError());
        kt.end();
    }
    // Algorithm 1 online step 4 for every frame, once the directions are final
    kt.begin("power");
    launch_power(p, X, doa, F, power, nullptr, nullptr, s, mask);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.flush();
    if (stats) {
        unsigned long long h[4] = {0, 0, 0, 0};
        SP_HIP(hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        timing_count("count:final_tiles_rescored", (double)h[0], F);
        timing_count("count:frames_hilo", (double)h[1], F);
    }
}

}  // namespace



// GEMM1 + Z prep in FP16 into caller buffers (zpart holds zpart_floats()).
int64_t front_zpart_floats(const svdphat_plan* p, int64_t F) {
    int nsplit, cps;
    g1_split_layout(p->g1[P_FP16], p->Rp, F, 0, &nsplit, &cps);
    G1Sched sc;
    if (g1s_sched(P_FP16, p, F, &sc)) nsplit = sc.slots;
    return (int64_t)nsplit * round_up64(F, 64) * p->Rp;
}

void front_fp16(svdphat_plan* p, const float2* X, int64_t F, float* zpart, float* z32, _Float16* zfrag, float* zsc,
                float* zn, hipStream_t s) {
    const G1Layout& g = p->g1[P_FP16];
    const int64_t Fc = round_up64(F, 64);
    int nsplit, cps;
    g1_split_layout(g, p->Rp, F, 0, &nsplit, &cps);
    G1Sched sc;
    const bool streamed = g1s_sched(P_FP16, p, F, &sc);
    if (streamed) launch_g1_streamed(P_FP16, p, sc, X, F, zpart, Fc * p->Rp, s);
    else launch_g1<_Float16, 64, false>((int)(Fc / 64), nsplit, s, X, F, p, P_FP16, g, cps, zpart, Fc * p->Rp,
                                        nullptr, nullptr);
    SP_HIP(hipGetLastError());
    k_zprep<_Float16><<<dim3((unsigned)(Fc / 4)), 256, 0, s>>>(zpart, streamed ? sc.slots : nsplit, Fc * p->Rp, F,
                                                               nullptr, p->Rp, z32, zfrag, zsc, zn, 1,
                                                               streamed ? sc.G : 0, sc.U, sc.nch);
    SP_HIP(hipGetLastError());
}

// GEMM2 (FP16) over the frames listed in flist (positions of zfrag hold
// those frames) and the FP32-rescored search for them (pmax frame-indexed,
// z32 position-indexed, znorm frame-indexed).
void back_list_fp16(svdphat_plan* p, const float2* X, int64_t Fmax, const int* flist, const int* fcount,
                    const _Float16* zfrag, const float* zsc, const float* z32pos, const float* zn_frame,
                    float* pmax, int32_t* doa, float* power, float* margin, hipStream_t s) {
    const int64_t pstride = pmax_stride(p);
    const int KSn = p->Rp / Mf<_Float16>::KSTEP;
    const int ntile = p->ncls_pad / QTILE;
    const int fch = 256;
    dim3 grid(cdiv(ntile, 4), (unsigned)((Fmax + fch - 1) / fch));
    const float uinv = 1.f / p->sr[0].uscale[P_FP16];
#define SP_G2L(N)                                                                                             \
    k_gemm2_list<N><<<grid, 256, 0, s>>>((const _Float16*)p->sr[0].Ufr[P_FP16], KSn, zfrag, Fmax, fch, p->ncls, ntile, zsc, \
                                         uinv, pmax, pstride, flist, fcount)
    switch (KSn) {
        case 1: SP_G2L(1); break;
        case 2: SP_G2L(2); break;
        case 3: SP_G2L(3); break;
        case 4: SP_G2L(4); break;
        case 5: SP_G2L(5); break;
        case 6: SP_G2L(6); break;
        default: SP_G2L(0); break;
    }
#undef SP_G2L
    SP_HIP(hipGetLastError());
    FinalArgs fa{};
    fa.X = X;
    fa.M = p->M;
    fa.P = p->P;
    fa.B = p->B;
    fa.pmax = pmax;
    fa.pstride = pstride;
    fa.ntile = ntile;
    fa.ncls = p->ncls;
    fa.z32 = z32pos;
    fa.znorm1 = zn_frame;
    fa.Rp = p->Rp;
    const double u = std::ldexp(1.0, -11);
    fa.ecoef = (float)((2.0 * u + u * u + 2.0 * p->Rp * std::ldexp(1.0, -24)) * 1.01);
    fa.rescore = 1;
    fa.U32T = p->sr[0].U32T;
    fa.tkappa = p->sr[0].tkappa;
    fa.sig = p->d_sig;
    fa.rows = p->d_rows;
    fa.rep = p->d_rep;
    fa.tauN = p->d_tauN_all;
    fa.tauM = p->d_tauM_all;
    fa.rowcls = p->d_rowcls;
    fa.usig_max = p->sr[0].usig_max;
    fa.nfr = Fmax;
    fa.flist = flist;
    fa.fcount = fcount;
    fa.doa = doa;
    fa.power = power;
    fa.margin = margin;
    fa.hilo_k = 4.f;
    fa.u = (float)u;
    launch_final(fa, p->M, !(p->flags & SVDPHAT_NO_DEDUP), Fmax, s);
    SP_HIP(hipGetLastError());
}

int g1_nrb_class(int nRB) {
    const int w = nRB <= 12 ? nRB : 12;
    return w <= 2 ? 2 : w <= 4 ? 4 : w <= 6 ? 6 : w <= 8 ? 8 : w <= 10 ? 10 : 12;
}

size_t g1_lds_bytes(int NRB, int CW) {
    return std::max((size_t)64 * (CW + XPAD) * sizeof(_Float16), (size_t)NRB * 4 * 64 * sizeof(f4));
}

void g1_split(const svdphat_plan* p, int64_t F, int want, int* nsplit, int* cps) {
    g1_split_layout(p->g1[P_FP16], p->Rp, F, want, nsplit, cps);
}

// Grouped launch classes: GEMM1 cls = NRB class * 2 + (M > 8); GEMM2 cls =
// the k-step count when the tile's U fragments stay in registers (1-6), else
// 0; search cls = (M > 8).
void launch_grouped(const GroupLaunch& g, const RDesc* d, hipStream_t s) {
    if (g.nwork <= 0) return;
    dim3 grid((unsigned)g.nwork);
    if (g.stage == 0) {
        const int nrb = g.cls / 2;
        const bool big = g.cls % 2;
#define SP_G1(N)                                                                                       \
    if (nrb == N) {                                                                                    \
        if (big) k_gemm1_grouped<N, 16, G1_IPT16><<<grid, 256, g.lds, s>>>(d, g.work);                 \
        else k_gemm1_grouped<N, 8, G1_IPT8><<<grid, 256, g.lds, s>>>(d, g.work);                       \
        return;                                                                                        \
    }
        SP_G1(2) SP_G1(4) SP_G1(6) SP_G1(8) SP_G1(10) SP_G1(12)
#undef SP_G1
        fail(SVDPHAT_E_UNSUPPORTED, "grouped GEMM1 class");
    } else if (g.stage == 1) {
        k_zprep_grouped<<<grid, 256, 0, s>>>(d, g.work);
    } else if (g.stage == 2) {
        switch (g.cls) {
            case 1: k_gemm2_grouped<1><<<grid, 256, 0, s>>>(d, g.work); break;
            case 2: k_gemm2_grouped<2><<<grid, 256, 0, s>>>(d, g.work); break;
            case 3: k_gemm2_grouped<3><<<grid, 256, 0, s>>>(d, g.work); break;
            case 4: k_gemm2_grouped<4><<<grid, 256, 0, s>>>(d, g.work); break;
            case 5: k_gemm2_grouped<5><<<grid, 256, 0, s>>>(d, g.work); break;
            case 6: k_gemm2_grouped<6><<<grid, 256, 0, s>>>(d, g.work); break;
            default: k_gemm2_grouped<0><<<grid, 256, 0, s>>>(d, g.work); break;
        }
    } else {
        if (g.cls) k_final_grouped<16><<<grid, 256, 0, s>>>(d, g.work);
        else k_final_grouped<8><<<grid, 256, 0, s>>>(d, g.work);
    }
}

void tune_time(svdphat_plan* p, int64_t F, int nsplit_want, int fch, double* us_g1, double* us_g2, hipStream_t s) {
    const G1Layout& g = p->g1[P_FP16];
    const int Rp = p->Rp;
    const int64_t Fc = round_up64(F, 64);
    int nsplit, cps;
    g1_split_layout(g, Rp, F, nsplit_want, &nsplit, &cps);
    const int ntile = p->ncls_pad / QTILE;
    const size_t nx = (size_t)F * p->M * p->B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += round_up64((int64_t)bytes, 256);
        return o;
    };
    const size_t o_x = take(nx * sizeof(float2));
    const size_t o_zp = take(sizeof(float) * nsplit * Fc * Rp);
    const size_t o_z = take(sizeof(float) * Fc * Rp);
    const size_t o_zf = take(sizeof(_Float16) * Fc * Rp);
    const size_t o_sc = take(sizeof(float) * Fc);
    const size_t o_zn = take(sizeof(float) * Fc);
    const size_t o_pm = take(sizeof(float) * pmax_stride(p) * Fc);
    char* w = (char*)ws_get(p, s, off);
    float2* X = (float2*)(w + o_x);
    k_fill_synth<<<dim3((unsigned)((nx + 255) / 256)), 256, 0, s>>>(X, (int64_t)nx);
    float* zpart = (float*)(w + o_zp);
    hipEvent_t e[3];
    for (auto& ev : e) SP_HIP(hipEventCreate(&ev));
    const int reps = 3;
    for (int it = 0; it <= reps; ++it) {
        if (it == 1) SP_HIP(hipEventRecord(e[0], s));
        launch_g1<_Float16, 64, false>((int)(Fc / 64), nsplit, s, X, F, p, P_FP16, g, cps, zpart, Fc * Rp, nullptr,
                                       nullptr);
        k_zprep<_Float16><<<dim3((unsigned)(Fc / 4)), 256, 0, s>>>(zpart, nsplit, Fc * Rp, F, nullptr, Rp,
                                                                   (float*)(w + o_z), (_Float16*)(w + o_zf),
                                                                   (float*)(w + o_sc), (float*)(w + o_zn), 1, 0, 0,
                                                                   0);
    }
    SP_HIP(hipEventRecord(e[1], s));
    const int KSn = Rp / Mf<_Float16>::KSTEP;
    dim3 grid(cdiv(ntile, 4), (unsigned)((F + fch - 1) / fch));
    for (int it = 0; it < reps; ++it) {
#define SP_G2T(N)                                                                                            \
    k_gemm2<_Float16, N><<<grid, 256, 0, s>>>((const _Float16*)p->sr[0].Ufr[P_FP16], KSn, (const _Float16*)(w + o_zf), F, \
                                              fch, p->ncls, ntile, (const float*)(w + o_sc), 1.f,                   \
                                              (float*)(w + o_pm), pmax_stride(p), nullptr, 0)
        switch (KSn) {
            case 1: SP_G2T(1); break;
            case 2: SP_G2T(2); break;
            case 3: SP_G2T(3); break;
            case 4: SP_G2T(4); break;
            case 5: SP_G2T(5); break;
            case 6: SP_G2T(6); break;
            default: SP_G2T(0); break;
        }
#undef SP_G2T
    }
    SP_HIP(hipEventRecord(e[2], s));
    SP_HIP(hipGetLastError());
    SP_HIP(hipEventSynchronize(e[2]));
    float a = 0.f, b = 0.f;
    SP_HIP(hipEventElapsedTime(&a, e[0], e[1]));
    SP_HIP(hipEventElapsedTime(&b, e[1], e[2]));
    for (auto& ev : e) (void)hipEventDestroy(ev);
    *us_g1 = 1e3 * a / reps;
    *us_g2 = 1e3 * b / reps;
}

bool mask_fused(const svdphat_plan* p, int64_t F, int prec, bool y_opt) {
    G1Sched sc;
    return (y_opt || !gv_applicable(p, F)) && g1s_sched(prec, p, F, &sc);
}

void launch_locate(svdphat_plan* p, const void* X, int64_t F, int prec, uint32_t mode, int32_t* doa, float* power,
                   float* yhat, float* margin, float* y_opt, hipStream_t s, void* scratch, size_t scratch_bytes,
                   const uint8_t* mask, float2* xm) {
    const float2* x = (const float2*)X;
    SP_REQUIRE(!mask || mask_fused(p, F, prec, y_opt != nullptr), SVDPHAT_E_UNSUPPORTED,
               "masked search without its streamed form");
    if (!y_opt && gv_applicable(p, F)) {
        // a few frames: GEMV form in FP32 (frame1.hip), on the caller's
        // scratch buffer or the plan's workspace of this stream
        const size_t need = gv_scratch_bytes(p, F);
        if (scratch)
            SP_REQUIRE(need <= scratch_bytes, SVDPHAT_E_INVAL, "scratch memory too small for this call");
        void* w = scratch ? scratch : ws_get(p, s, need);
        launch_gv(p, p->sr[(mode & SVDPHAT_NORMALIZED) ? 1 : 0], x, F, doa, power, yhat, margin, w, s);
        return;
    }
    if (prec == P_FP32)
        run_locate<float>(p, x, F, prec, mode, doa, power, yhat, margin, y_opt, s, scratch, scratch_bytes, mask, xm);
    else if (prec == P_FP16)
        run_locate<_Float16>(p, x, F, prec, mode, doa, power, yhat, margin, y_opt, s, scratch, scratch_bytes, mask,
                             xm);
    else run_locate<__bf16>(p, x, F, prec, mode, doa, power, yhat, margin, y_opt, s, scratch, scratch_bytes, mask, xm);
}

}  // namespace svdphat
