// Plain SRP-PHAT in FP32 on gfx950 (Section 2: PHAT eq. (3), powers
// eq. (9), argmax eq. (6)), the comparison form of the reduced search.
//   k_phat_frag   PHAT vector in FP32, written as MFMA B-operand fragments.
//   k_srp_gemm    Y = [Re W, -Im W] [Re X; Im X] with FP32 MFMA and an argmax
//                 epilogue per (frame, tile of 128 directions).
//   k_srp_reduce  argmax across tiles; the power is the winning row's Y.
#include "device.h"

namespace svdphat {

namespace {

// ------------------------------------------------------------------ SRP
// PHAT vector in FP32, written as MFMA B-operand fragments of the 16x16x4
// instruction: element (k, frame) -> [frame/16][k/4][lane = frame%16 +
// 16 (k%4)], k = (bin P + p) 2 + {0: Re, 1: Im}.  Frames from nfr up to the
// padded count and the columns past 2L are written as zeros.
// One workgroup per (block of 16 frames, run of SB bins): thread (bin b,
// frame nn) forms the P pair products of its (frame, bin) into LDS in the
// fragment order, and the block's fragments of those bins, one contiguous
// run of the output ([k0/4, kend/4) x 64 floats), go out in 16-byte stores
// (the last run takes the zero columns up to 4 Wks as well).
template <int MAXM, int SB>
__global__ __launch_bounds__(SB * 16) void k_phat_frag(const float2* __restrict__ X, int64_t nfr, int M, int P, int B,
                                                       int Wks, int nchunk, float* __restrict__ xfr) {
    extern __shared__ __align__(16) float st[];  // SB 2P x 16 staged values
    const int64_t fb = blockIdx.x / nchunk;
    const int c = (int)(blockIdx.x - fb * nchunk);
    const int t = threadIdx.x, nn = t & 15, b = t >> 4;
    const int64_t f = fb * 16 + nn;
    const int bin = c * SB + b;
    const bool live = f < nfr && bin < B;
    const float2* xf = X + (live ? f * M * B + bin : 0);
    float re[MAXM], im[MAXM];
#pragma unroll
    for (int m = 0; m < MAXM; ++m) {
        const float2 v = (live && m < M) ? xf[(int64_t)m * B] : float2{0.f, 0.f};
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
                const int k = (b * P + p) * 2;  // column within the run
                st[(k >> 2) * 64 + nn + 16 * (k & 3)] = fmaf(re[i], re[j], im[i] * im[j]);
                st[((k + 1) >> 2) * 64 + nn + 16 * ((k + 1) & 3)] = fmaf(im[i], re[j], -(re[i] * im[j]));
                ++p;
            }
    __syncthreads();
    const int kw = SB * 2 * P;  // staged columns (a multiple of 4)
    const int k0 = c * kw;
    const int kend = c == nchunk - 1 ? 4 * Wks : k0 + kw;
    float4* out = reinterpret_cast<float4*>(xfr + (fb * Wks + k0 / 4) * 64);
    const int n4 = (kend - k0) * 4;
    for (int i = t; i < n4; i += SB * 16)
        out[i] = 4 * i < kw * 16 ? *reinterpret_cast<const float4*>(st + 4 * i) : make_float4(0.f, 0.f, 0.f, 0.f);
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


}  // namespace

void build_w_fp32_frags(svdphat_plan* p) {
    const int Wk = round_up(2 * p->L, 4) / 4;
    p->Wks = Wk;
    p->Wrows_pad = round_up(p->Q, 128);
    const int64_t total = (int64_t)p->Wrows_pad * Wk * 4;
    if (dev_malloc((void**)&p->Wfr, total * sizeof(float)) != hipSuccess) {
        p->Wfr = nullptr;
        fail(SVDPHAT_E_NOMEM, "device allocation of W (" + std::to_string(total * 4) + " bytes) failed");
    }
    p->device_bytes += total * (int64_t)sizeof(float);
    double* dtau = nullptr;
    dev_alloc((void**)&dtau, p->tau.size() * sizeof(double), "steering delays");
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
    // runs of 16 bins (4 above 8 microphones, to bound the LDS); a run of
    // SB bins starts at column SB 2P c, a multiple of 4
    const int sb = p->M <= 8 ? 16 : 4;
    const int nchunk = (p->B + sb - 1) / sb;
    const int64_t nblk = (Fp / 16) * nchunk;
    SP_REQUIRE(nblk < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "too many frames for one call");
    const size_t lds = (size_t)sb * 2 * p->P * 16 * sizeof(float);
    if (p->M <= 8)
        k_phat_frag<8, 16><<<dim3((unsigned)nblk), 256, lds, s>>>(X, F, p->M, p->P, p->B, Wks, nchunk, xfr);
    else
        k_phat_frag<16, 4><<<dim3((unsigned)nblk), 64, lds, s>>>(X, F, p->M, p->P, p->B, Wks, nchunk, xfr);
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
