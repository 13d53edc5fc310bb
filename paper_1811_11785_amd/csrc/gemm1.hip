// GEMM1, streamed form: Z = S V^H x (eq. (12) with S folded into V^H) with
// the PHAT cross-spectra (eq. (3)) formed on chip, for 16-bit operands, 6 to
// 8 microphones and all row blocks of Z in one workgroup.
//
// Work units are (frame tile of 64 frames, chunk of BB bins) pairs in tile-
// major order; a persistent grid of G workgroups (one per CU) takes equal
// contiguous ranges of units, so every workgroup streams its STFT values
// without a break from its first unit to its last.  A workgroup has 8
// waves in two roles, one of each on every SIMD:
//   producers (waves 4-7) load the STFT values of the units ahead into a
//     register ring of XD units (each thread one frame and a pair of bins,
//     one 16-byte load per microphone; 64 frames x 4 pairs fill the 256
//     threads) and form each unit's PHAT tile (per-mic unit normalisation,
//     then X_i conj(X_j) for pairs i < j in order, rounded to T, stored as
//     (Re, Im)) in one of two LDS buffers;
//   consumers (waves 0-3) take the k-steps wave, wave + 4, ... of the
//     unit's KSC = ceil(8 MM (MM - 1) / 32) k-steps, keep a ring of A
//     fragments in flight and run the MFMAs, each accumulating every (row
//     block, frame block) of the tile's Z; at the end of a frame tile (or
//     of the range) the four consumers' partial sums are added through LDS
//     (three rounds, with the producers taking part in the barriers) and
//     written to slot w - w0, w0 the first workgroup whose range meets the
//     tile.
// One barrier per unit hands a PHAT tile from the producers to the
// consumers.  The Z preparation sums the w1 - w0 + 1 slots of a frame.
//
// Memory order.  Vector-memory loads complete in issue order for a wave's
// wait counter, so a wave that waits for one load also waits for every load
// it issued earlier.  Splitting the roles keeps the two streams apart: the
// producers' STFT loads run XD units ahead without the consumers' A loads
// queueing behind them, and each consumer issues the A fragments of unit
// u+2 as soon as the MFMAs of unit u that read those registers are issued.
// Loop-carried registers are first filled outside the loop; an empty asm
// statement on those first values keeps the compiler from merging the two
// load sites into one load at the top of the loop (which would turn every
// prefetch into a load right before its use).  Loads sit outside every
// branch so that the wait counts stay exact.
//
// Cache footprint.  A unit reads a short run of bins from each (frame,
// microphone) row of the STFT, so every row keeps one partly used cache
// line in L2 until its next unit; with one workgroup per CU (the LDS request
// guarantees it) the lines in flight on an XCD stay well inside its L2.
// The chunks of a frame tile are visited in a rotated order, so that the
// first workgroup starting inside the tile starts at chunk 0: the
// workgroups of an XCD then walk the chunks of A (the same for every frame
// tile) nearly in step and share them in L2 instead of each fetching all
// of A from memory.
#include "device.h"

namespace svdphat {

namespace {

constexpr int G1S_NF = 64;
constexpr int G1S_BB = 8;   // bins per chunk
constexpr int G1S_PAD = 8;  // LDS row padding (elements)
constexpr int G1S_XD = 4;   // units of STFT values in flight (even)

// k-steps of 32 per chunk for MM microphones (MM (MM - 1) stacked values
// per bin)
constexpr int g1s_ksc(int MM) { return (G1S_BB * MM * (MM - 1) + 31) / 32; }

// four floats read with one 16-byte load from an 8-byte aligned address
struct __attribute__((aligned(8))) f4u {
    float x, y, z, w;
};

// unit-modulus normalisation (the per-microphone factor of eq. (3)) of one
// STFT value, rounded to a half pair; values whose |X|^2 is not a finite
// normal float are silent and give 0
__device__ __forceinline__ h2 unit_h2(float re, float im) {
    const float m2 = fmaf(re, re, im * im);  // fused as written, so every instance rounds alike
    const float s = __builtin_amdgcn_rsqf(m2);
    const h2 u = h2{(_Float16)(re * s), (_Float16)(im * s)};
    return __builtin_amdgcn_classf(m2, 0x100) ? u : h2{(_Float16)0.f, (_Float16)0.f};
}

// workgroup whose unit range holds unit u (ranges [w U / G, (w+1) U / G))
__host__ __device__ inline int g1s_owner(int64_t u, int G, int64_t U) { return (int)(((u + 1) * G - 1) / U); }

// rotation of frame tile t's chunk order: position j of the tile holds chunk
// (j + phi) mod nch, phi chosen so that the first workgroup whose range
// starts inside the tile starts at chunk 0 (0 when none does)
__device__ inline int g1s_phi(int64_t t, int nch, int G, int64_t U) {
    const int64_t t0 = t * nch;
    const int wf = g1s_owner(t0, G, U);
    if ((int64_t)wf * U / G == t0 || wf + 1 >= G) return 0;
    const int64_t s2 = (int64_t)(wf + 1) * U / G;
    return s2 < t0 + nch ? (int)(nch - (s2 - t0)) : 0;
}

template <typename T, int MM, int NRB, int XD, bool MK>
__global__ __launch_bounds__(512) void k_gemm1s(const float2* __restrict__ X, int64_t nfr, int B,
                                                const T* __restrict__ A, int nch, int64_t U,
                                                float* __restrict__ zpart, int64_t zstride, int Rp,
                                                const uint8_t* __restrict__ mask) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL, NF = G1S_NF, FB = NF / 16;
    constexpr int P = MM * (MM - 1) / 2, TWOP = 2 * P;
    constexpr int BB = G1S_BB, BP = BB / 2;
    constexpr int KSC = g1s_ksc(MM), KPW = (KSC + 3) / 4;
    constexpr int AD = KPW <= 2 ? 2 : 1;  // units of A fragments in flight
    constexpr int CW = KSC * KS;          // stacked values per chunk (BB * TWOP used)
    constexpr int LDX = CW + G1S_PAD;
    constexpr int PADC = CW - BB * TWOP;
    constexpr int PL = NF * BP / 4;       // (frame, bin pair) items per producer wave
    static_assert(KS == 32 && PL == 64 && XD % 2 == 0, "chunk layout");
    typedef typename Vec<T>::t VT;
    typedef typename Vec<T>::pair VP;
    extern __shared__ __align__(16) char smem[];
    T* xsb = reinterpret_cast<T*>(smem);  // two tiles of NF x LDX
    // then the region where the consumers add their partial sums
    f4* red = reinterpret_cast<f4*>(smem + (size_t)2 * NF * LDX * sizeof(T));

    const int G = gridDim.x, w = blockIdx.x;
    const int64_t ub = (int64_t)w * U / G, ue = (int64_t)(w + 1) * U / G;  // this workgroup's units
    if (ub >= ue) return;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // chunk of unit u in frame tile t; only the first and the last tile of
    // the range can have a rotation (no other workgroup starts in between)
    const int64_t tf = ub / nch, tl = (ue - 1) / nch;
    const int phf = g1s_phi(tf, nch, G, U), phl = g1s_phi(tl, nch, G, U);
    // unit cursor: unit u = t nch + j, moved one unit at a time and held at
    // the range's last unit (no division inside the loops)
    struct Cur {
        int64_t u, t;
        int j;
    };
    auto cur_at = [&](int64_t u) {
        const int64_t t = u / nch;
        return Cur{u, t, (int)(u - t * nch)};
    };
    auto adv = [&](Cur& c) {
        if (c.u + 1 < ue) {
            ++c.u;
            if (++c.j == nch) {
                c.j = 0;
                ++c.t;
            }
        }
    };
    auto chunk = [&](const Cur& c) {
        const int v = c.j + (c.t == tf ? phf : c.t == tl ? phl : 0);
        return v >= nch ? v - nch : v;
    };

    // padding columns of both tiles are zero (the PHAT phase never writes them)
    if (PADC > 0)
        for (int i = tid; i < 2 * NF * PADC; i += 512) xsb[(i / PADC) * LDX + BB * TWOP + i % PADC] = cvt<T>(0.f);

    f4 acc[NRB][FB];
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
        for (int j = 0; j < FB; ++j) acc[r][j] = f4{0.f, 0.f, 0.f, 0.f};

    if (wave >= 4) {
        // ---------------------------------------------------------- producer
        // item (frame it / BP, bins 2 (it % BP) and 2 (it % BP) + 1), it =
        // 64 (wave - 4) + lane
        const int it = PL * (wave - 4) + lane;
        const int fl = it / BP, b0 = 2 * (it % BP);
        // Ring slot d holds the units ub + d (mod XD).  Loads are
        // unconditional: a pair whose second bin is past the last one reads
        // the pair one bin earlier, and a pair outside the data reads frame 0,
        // bins 0-1; the values are selected (or zeroed) where consumed.
        f4u xv[XD][MM];
        int xmode[XD];  // 2: both bins, 1: first bin only (shifted load), 0: none
        // MK: the mask bytes of the two loaded bins (bit 0: the load's first
        // bin, bit 8: its second), fetched with the values
        int xmk[XD];
        auto fetch = [&](int d, const Cur& cu) {
            const int64_t t = cu.t;
            const int c = chunk(cu);
            const int64_t f = t * NF + fl;
            const int s0 = c * BB + b0;
            const int mode = f >= nfr ? 0 : s0 + 1 < B ? 2 : s0 < B ? 1 : 0;
            xmode[d] = mode;
            const int64_t off = mode == 2 ? f * MM * B + s0 : mode == 1 ? f * MM * B + s0 - 1 : 0;
#pragma unroll
            for (int m = 0; m < MM; ++m) xv[d][m] = *reinterpret_cast<const f4u*>(X + off + (int64_t)m * B);
            if constexpr (MK) {
                const int64_t mo = mode == 2 ? f * B + s0 : mode == 1 ? f * B + s0 - 1 : 0;
                xmk[d] = (int)mask[mo] | ((int)mask[mo + 1] << 8);
            }
        };
        // PHAT tile of one chunk from ring slot d; FULL: every pair of the
        // chunk lies inside the data (no per-value selection)
        auto phat_impl = [&](auto full_tag, int d, T* xs) {
            constexpr bool FULL = decltype(full_tag)::value;
            const int mode = xmode[d];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                VP* dst = reinterpret_cast<VP*>(xs + fl * LDX + (b0 + q) * TWOP);
                // MK: whether the mask keeps this bin (bin q of the pair is the
                // load's bin q, or its second bin for the shifted load)
                bool keep = true;
                if constexpr (MK) keep = (xmk[d] >> (q == 1 || (!FULL && mode == 1) ? 8 : 0)) & 0xFF;
                float re[MM], im[MM];
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    const f4u v = xv[d][m];
                    if (FULL) {
                        re[m] = q == 0 ? v.x : v.z;
                        im[m] = q == 0 ? v.y : v.w;
                    } else if (q == 0) {
                        re[m] = mode == 2 ? v.x : mode == 1 ? v.z : 0.f;
                        im[m] = mode == 2 ? v.y : mode == 1 ? v.w : 0.f;
                    } else {
                        re[m] = mode == 2 ? v.z : 0.f;
                        im[m] = mode == 2 ? v.w : 0.f;
                    }
                }
                if constexpr (std::is_same<T, _Float16>::value) {
                    h2 u[MM];
#pragma unroll
                    for (int m = 0; m < MM; ++m) u[m] = unit_h2(re[m], im[m]);
                    if constexpr (MK)
#pragma unroll
                        for (int m = 0; m < MM; ++m) u[m] = keep ? u[m] : h2{(_Float16)0.f, (_Float16)0.f};
                    // (Re, Im) of X_i conj(X_j) = (a c + b d, b c - a d) for
                    // X_i = a + ib, X_j = c + id
                    int p = 0;
#pragma unroll
                    for (int i = 0; i < MM; ++i) {
                        const h2 sw = __builtin_shufflevector(u[i], u[i], 1, 0);
#pragma unroll
                        for (int j = i + 1; j < MM; ++j) {
                            const h2 cc = h2{u[j].x, u[j].x}, dd = h2{u[j].y, -u[j].y};
                            dst[p] = u[i] * cc + sw * dd;
                            ++p;
                        }
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < MM; ++m) unit(re[m], im[m]);
                    if constexpr (MK)
#pragma unroll
                        for (int m = 0; m < MM; ++m) {
                            re[m] = keep ? re[m] : 0.f;
                            im[m] = keep ? im[m] : 0.f;
                        }
                    int p = 0;
#pragma unroll
                    for (int i = 0; i < MM; ++i)
#pragma unroll
                        for (int j = i + 1; j < MM; ++j) {
                            // FMAs as written: every instance of the kernel
                            // (with or without the mask) rounds alike
                            dst[p] = mkpair<T>(cvt<T>(fmaf(re[i], re[j], im[i] * im[j])),
                                               cvt<T>(fmaf(im[i], re[j], -(re[i] * im[j]))));
                            ++p;
                        }
                }
            }
        };
        auto phat = [&](int d, const Cur& cu, T* xs) {
            const int64_t t = cu.t;
            const int c = chunk(cu);
            if ((t + 1) * NF <= nfr && (c + 1) * BB <= B) phat_impl(std::true_type{}, d, xs);
            else phat_impl(std::false_type{}, d, xs);
        };
        // cursors: cf the next unit to fetch, cp the next unit to form, cu
        // the unit whose MFMAs the consumers run (its tile end brings the
        // six barriers of their partial-sum rounds)
        Cur cf = cur_at(ub), cp = cur_at(ub), cu = cur_at(ub);
#pragma unroll
        for (int d = 0; d < XD; ++d) {
            fetch(d, cf);  // units ub + d (at most ue - 1)
            adv(cf);
        }
#pragma unroll
        for (int d = 0; d < XD; ++d)
#pragma unroll
            for (int m = 0; m < MM; ++m)
                asm volatile("" : "+v"(xv[d][m].x), "+v"(xv[d][m].y), "+v"(xv[d][m].z), "+v"(xv[d][m].w));
        phat(0, cp, xsb);
        adv(cp);
        fetch(0, cf);
        adv(cf);
        for (int64_t u0 = ub; u0 < ue; u0 += XD) {
#pragma unroll
            for (int d = 0; d < XD; ++d) {
                const int64_t u = u0 + d;
                if (u < ue) __syncthreads();  // tile of unit u complete; tile of u+1 free
                if (u + 1 < ue) {
                    phat((d + 1) % XD, cp, xsb + ((d + 1) & 1) * NF * LDX);  // unit u + 1
                    adv(cp);
                }
                fetch((d + 1) % XD, cf);  // unit u + 1 + XD (at most ue - 1)
                adv(cf);
                if (u < ue) {
                    if (cu.j == nch - 1 || u == ue - 1)
                        for (int k = 0; k < 6; ++k) __syncthreads();
                    adv(cu);
                }
            }
        }
    } else {
        // ---------------------------------------------------------- consumer
        // ring of AD units of A fragments: slot sl holds the units ub + sl
        // (mod AD); the fragments of unit u+AD are loaded into the registers
        // of unit u right after the MFMAs of u that read them.  This wave
        // takes k-steps wave + 4 kk, kk < nkk (the same for the whole wave).
        const int nkk = (KSC - __builtin_amdgcn_readfirstlane(wave) + 3) / 4;
        auto has = [&](int kk) { return KSC % 4 == 0 || kk < nkk; };
        VT a[AD][KPW][NRB];
        auto loadA = [&](int sl, const Cur& cu, int kk) {
            const int c = chunk(cu);
            const T* base = A + (((int64_t)c * KSC + wave + 4 * kk) * NRB * 64 + lane) * EPL;
#pragma unroll
            for (int r = 0; r < NRB; ++r) a[sl][kk][r] = *reinterpret_cast<const VT*>(base + r * 64 * EPL);
        };
        // cursors: cl the next unit whose fragments are loaded, cc the unit
        // whose MFMAs run
        Cur cl = cur_at(ub), cc = cur_at(ub);
#pragma unroll
        for (int sl = 0; sl < AD; ++sl) {
#pragma unroll
            for (int kk = 0; kk < KPW; ++kk)
                if (has(kk)) loadA(sl, cl, kk);  // unit ub + sl (at most ue - 1)
            adv(cl);
        }
#pragma unroll
        for (int sl = 0; sl < AD; ++sl)
#pragma unroll
            for (int kk = 0; kk < KPW; ++kk)
#pragma unroll
                for (int r = 0; r < NRB; ++r) asm volatile("" : "+v"(a[sl][kk][r]));
        for (int64_t u0 = ub; u0 < ue; u0 += AD) {
#pragma unroll
            for (int sl = 0; sl < AD; ++sl) {
                const int64_t u = u0 + sl;
                if (u < ue) {
                    __syncthreads();  // tile of unit u complete
                    const T* xs = xsb + ((u - ub) & 1) * NF * LDX;  // the producers' buffer of unit u
#pragma unroll
                    for (int kk = 0; kk < KPW; ++kk) {
                        if (!has(kk)) continue;
                        const T* bp = xs + (lane & 15) * LDX + (wave + 4 * kk) * KS + EPL * (lane >> 4);
                        VT b[FB];
#pragma unroll
                        for (int j = 0; j < FB; ++j) b[j] = *reinterpret_cast<const VT*>(bp + j * 16 * LDX);
#pragma unroll
                        for (int r = 0; r < NRB; ++r)
#pragma unroll
                            for (int j = 0; j < FB; ++j) acc[r][j] = mfma(a[sl][kk][r], b[j], acc[r][j]);
                        loadA(sl, cl, kk);  // unit u + AD (at most ue - 1)
                    }
                    const int64_t t = cc.t;
                    if (cc.j == nch - 1 || u == ue - 1) {
                        // end of this workgroup's part of frame tile t: the four
                        // consumers' sums are added in wave 0 (wave k writes,
                        // wave 0 adds, k = 3, 2, 1; every round between two
                        // barriers the producers also pass), which writes slot
                        // w - w0.  D layout: lane holds rows 4 (lane / 16) + e
                        // of column lane % 16.
                        for (int k = 3; k >= 1; --k) {
                            if (wave == k)
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
                        const int slot = w - g1s_owner(t * nch, G, U);
#pragma unroll
                        for (int j = 0; j < FB; ++j) {
                            const int64_t fpos = t * NF + j * 16 + (lane & 15);
                            float* zp = zpart + (int64_t)slot * zstride + fpos * Rp;
                            if (wave == 0 && fpos < nfr)
#pragma unroll
                                for (int r = 0; r < NRB; ++r)
                                    *reinterpret_cast<f4*>(zp + r * 16 + 4 * (lane >> 4)) = acc[r][j];
#pragma unroll
                            for (int r = 0; r < NRB; ++r) acc[r][j] = f4{0.f, 0.f, 0.f, 0.f};
                        }
                        // once per tile: let every memory operation finish, so
                        // that this path rejoins the loop with nothing pending
                        // and the loop's wait counts need not allow for the
                        // stores (vector stores count in vmcnt)
                        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
                    }
                    adv(cc);
                } else {
#pragma unroll
                    for (int kk = 0; kk < KPW; ++kk)
                        if (has(kk)) loadA(sl, cl, kk);
                }
                adv(cl);
            }
        }
    }
}

// whether the streamed form covers (microphones, row blocks)
constexpr bool g1s_ok(int M, int nRB) { return M >= 6 && M <= 8 && (nRB == 2 || nRB == 4 || nRB == 6); }

// LDS of the streamed kernel: two PHAT tiles, and at least 81 KiB so that
// one workgroup runs per CU
template <typename T, int MM, int NRB>
constexpr size_t g1s_lds() {
    constexpr size_t tiles = 2 * G1S_NF * (g1s_ksc(MM) * Mf<T>::KSTEP + G1S_PAD) * sizeof(T);
    constexpr size_t b = tiles + (size_t)NRB * (G1S_NF / 16) * 64 * sizeof(f4);  // + the reduction region
    return b > 81 * 1024 ? b : 81 * 1024;
}

template <typename T, int MM>
void launch_mm(int nRB, int G, hipStream_t s, const float2* X, int64_t F, int B, const void* A, int nch, int64_t U,
               float* zpart, int64_t zstride, int Rp, const uint8_t* mask) {
    const T* a = (const T*)A;
    switch (nRB) {
#define G1S_CASE(NRB_)                                                                                          \
    case NRB_:                                                                                                  \
        if constexpr (g1s_ok(MM, NRB_)) {                                                                       \
            constexpr size_t lds = g1s_lds<T, MM, NRB_>();                                                      \
            if (mask)                                                                                           \
                k_gemm1s<T, MM, NRB_, G1S_XD, true><<<G, 512, lds, s>>>(X, F, B, a, nch, U, zpart, zstride, Rp, mask); \
            else                                                                                                \
                k_gemm1s<T, MM, NRB_, G1S_XD, false><<<G, 512, lds, s>>>(X, F, B, a, nch, U, zpart, zstride, Rp,   \
                                                                      nullptr);                                 \
        }                                                                                                       \
        return;
        G1S_CASE(2)
        G1S_CASE(4)
        G1S_CASE(6)
#undef G1S_CASE
    }
}

}  // namespace

int cu_count(int device) {
    static int cached[64] = {0};
    if (device < 0 || device >= 64) return 256;
    if (!cached[device]) {
        int n = 0;
        SP_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device));
        cached[device] = n > 0 ? n : 256;
    }
    return cached[device];
}

bool g1s_layout(int M, int nRB, int kstep, int* CW, int* BB) {
    if (kstep != 32 || !g1s_ok(M, nRB)) return false;
    *CW = g1s_ksc(M) * kstep;
    *BB = G1S_BB;
    return true;
}

bool g1s_sched(int prec, const svdphat_plan* p, int64_t F, G1Sched* out) {
    const int nRB = p->Rp / 16;
    int cw = 0, bb = 0;
    const bool split = p->as_split > 0 && prec != P_FP32;  // two row-group passes
    const G1Layout& g = split ? p->g1s[prec] : p->g1[prec];
    if (prec == P_FP32 || p->B < 2 || F < 1) return false;
    if (!split && (!g1s_layout(p->M, nRB, 32, &cw, &bb) || g.CW != cw || g.BB != bb)) return false;
    G1Sched sc;
    const int64_t ftiles = (F + G1S_NF - 1) / G1S_NF;
    sc.nch = g.nch;
    sc.U = ftiles * g.nch;
    // two passes pay the pipeline's start twice: only with at least 8 units
    // per workgroup of a full grid (at 4096 frames of the 3-D plan, K = 71:
    // 67 us against 75 for the general kernel; at 256 frames 54 against 36)
    if (split && sc.U < 8 * (int64_t)cu_count(p->device)) return false;
    // one workgroup per CU, at least 8 units each
    sc.G = (int)std::max<int64_t>(1, std::min<int64_t>(cu_count(p->device), sc.U / 8));
    int runs = 1;
    for (int64_t t = 0; t < ftiles; ++t)
        runs = std::max(runs, g1s_owner((t + 1) * sc.nch - 1, sc.G, sc.U) - g1s_owner(t * sc.nch, sc.G, sc.U) + 1);
    sc.slots = runs;
    *out = sc;
    return true;
}

// one launch of the streamed kernel over nRB row blocks whose A fragments
// start at A, writing rows 0 .. 16 nRB - 1 of the Z slots at zpart
static void launch_g1_pass(int prec, const svdphat_plan* p, const G1Sched& sc, const float2* X, int64_t F,
                           const void* A, int nRB, float* zpart, int64_t zstride, const uint8_t* mask,
                           hipStream_t s) {
    const int B = p->B, Rp = p->Rp;
    SP_REQUIRE(nRB == 2 || nRB == 4 || nRB == 6, SVDPHAT_E_UNSUPPORTED, "streamed GEMM1: 2, 4 or 6 row blocks");
    if (prec == P_FP16) {
        switch (p->M) {
            case 6: launch_mm<_Float16, 6>(nRB, sc.G, s, X, F, B, A, sc.nch, sc.U, zpart, zstride, Rp, mask); return;
            case 7: launch_mm<_Float16, 7>(nRB, sc.G, s, X, F, B, A, sc.nch, sc.U, zpart, zstride, Rp, mask); return;
            case 8: launch_mm<_Float16, 8>(nRB, sc.G, s, X, F, B, A, sc.nch, sc.U, zpart, zstride, Rp, mask); return;
        }
    } else {
        switch (p->M) {
            case 6: launch_mm<__bf16, 6>(nRB, sc.G, s, X, F, B, A, sc.nch, sc.U, zpart, zstride, Rp, mask); return;
            case 7: launch_mm<__bf16, 7>(nRB, sc.G, s, X, F, B, A, sc.nch, sc.U, zpart, zstride, Rp, mask); return;
            case 8: launch_mm<__bf16, 8>(nRB, sc.G, s, X, F, B, A, sc.nch, sc.U, zpart, zstride, Rp, mask); return;
        }
    }
    fail(SVDPHAT_E_UNSUPPORTED, "streamed GEMM1 launched for an unsupported plan");
}

void launch_g1_streamed(int prec, const svdphat_plan* p, const G1Sched& sc, const float2* X, int64_t F, float* zpart,
                        int64_t zstride, hipStream_t s, const uint8_t* mask) {
    if (p->as_split > 0) {
        // two passes over the frames, each with its row group's A; the second
        // writes Z's rows from 16 as_split on, in the same slots (the two
        // passes share the schedule)
        const int nRB = p->Rp / 16, n0 = p->as_split;
        launch_g1_pass(prec, p, sc, X, F, p->As[prec][0], n0, zpart, zstride, mask, s);
        SP_HIP(hipGetLastError());
        launch_g1_pass(prec, p, sc, X, F, p->As[prec][1], nRB - n0, zpart + 16 * n0, zstride, mask, s);
        return;
    }
    launch_g1_pass(prec, p, sc, X, F, p->A[prec], p->Rp / 16, zpart, zstride, mask, s);
}

}  // namespace svdphat
