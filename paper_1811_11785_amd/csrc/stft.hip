// STFT front end (Section 2): each microphone signal analysed in frames of
// N samples, hop samples apart, with the sine window w[n] = sin(pi n / N):
//   X_m[f, k] = sum_{n<N} w[n] x_m[f hop + n] exp(-2 pi i k n / N),
//   k = 0 .. N/2, written as complex64 [F][M][N/2+1], the layout the
//   localisation path reads.
//
// One wave per (frame, microphone), grid-stride over the F M pairs.  The N
// windowed real samples are taken as N/2 complex points z[n] = x[2n] +
// i x[2n+1]; their FFT (Stockham radix-4 stages and at most one radix-2
// stage, natural order, in the wave's two LDS buffers) gives the N/2+1
// real-input bins by the even/odd split
//   X[k] = (Z[k] + conj Z[N/2-k]) / 2 + e^{-2 pi i k / N} (Z[k] - conj Z[N/2-k]) / 2i.
// The twiddles and the window are evaluated once per workgroup in FP64 and
// kept in LDS as FP32.  All arithmetic is FP32.
#include "device.h"

namespace svdphat {

namespace {

constexpr int STFT_WAVES = 4;  // waves (pairs in flight) per workgroup

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

__device__ __forceinline__ float2 cmul(float2 u, float2 w) {
    return float2{u.x * w.x - u.y * w.y, u.x * w.y + u.y * w.x};
}

// NL = max(1, N / 64) samples per lane; NC = N where it is fixed by NL
// (N >= 64), so the stages unroll, else 0 (N from the argument)
template <int NL, int NC>
__global__ __launch_bounds__(256) void k_stft(const float* __restrict__ pcm, int M, int64_t ld, int Nrt, int hop,
                                              float2* __restrict__ X, int64_t npair) {
    extern __shared__ __align__(16) char smem[];
    const int N = NC > 0 ? NC : Nrt;
    const int N2 = N / 2, B = N2 + 1;
    float2* tw1 = reinterpret_cast<float2*>(smem);  // e^{-2 pi i j / N2}, j < N2
    float2* tw2 = tw1 + N2;                          // e^{-2 pi i k / N}, k <= N2
    float* win = reinterpret_cast<float*>(tw2 + N2 + 2);
    float2* bufs = reinterpret_cast<float2*>(win + N);  // per wave: two buffers of N2 points
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int j = tid; j < N2; j += 256) {
        double s, c;
        sincospi(-2.0 * j / N2, &s, &c);
        tw1[j] = float2{(float)c, (float)s};
    }
    for (int k = tid; k <= N2; k += 256) {
        double s, c;
        sincospi(-2.0 * k / N, &s, &c);
        tw2[k] = float2{(float)c, (float)s};
    }
    for (int n = tid; n < N; n += 256) win[n] = (float)sinpi((double)n / N);
    __syncthreads();

    float2* b0 = bufs + (size_t)wave * 2 * N2;
    float2* b1 = b0 + N2;
    float* b0f = reinterpret_cast<float*>(b0);
    const int64_t step = (int64_t)gridDim.x * STFT_WAVES;
    // R1 (N >= 512, so N2 / 4 >= 64): the first radix-4 stage runs in
    // registers.  Lane l loads the inputs of its butterflies j = l + 64 b
    // straight from memory, z[j + r N2/4] for r < 4 (sample index
    // smp(i) below), and writes each butterfly's four outputs, which are
    // adjacent, as two 16-byte LDS stores; the windowed samples never pass
    // through LDS.  Otherwise sample n = lane + 64 i is staged in LDS.
    constexpr bool R1 = NC >= 512;
    auto smp = [&](int i) {
        if constexpr (R1) {
            const int bq = i >> 3, r = (i >> 1) & 3, e = i & 1;
            return 2 * (lane + 64 * bq + r * (N2 / 4)) + e;
        } else {
            return min(lane + 64 * i, N - 1);
        }
    };
    // the samples of the wave's next pair are loaded into registers while
    // the current pair's transform runs (without R1, lanes past N re-read
    // sample N - 1 and are not used)
    float xs[NL];
    // (frame, microphone) of the pair to fetch, moved by the grid stride
    // without a division per pair
    const int64_t pr0 = (int64_t)blockIdx.x * STFT_WAVES + wave;
    int64_t ff = pr0 / M;
    int fm = (int)(pr0 - ff * M);
    const int64_t sf = step / M;
    const int sm = (int)(step - sf * M);
    auto fetch = [&]() {
        const float* src = pcm + (int64_t)fm * ld + ff * hop;
#pragma unroll
        for (int i = 0; i < NL; ++i) xs[i] = src[smp(i)];
        ff += sf;
        fm += sm;
        if (fm >= M) {
            fm -= M;
            ++ff;
        }
    };
    // the lane's window values and split twiddles stay in registers
    float wr[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) wr[i] = win[smp(i)];
    // a pair's bins k = lane + 64 i stay in registers until the next pair's
    // samples are in LDS; their stores then go out before the next prefetch,
    // so they drain during a whole transform (vector stores count in the same
    // in-order counter as the loads)
    constexpr int KO = NC > 0 ? (NC / 2 + 64) / 64 : 1;
    float2 xo[KO];
    int64_t opr = -1;  // pair whose bins are in xo
    auto store = [&]() {
        float2* out = X + opr * B;  // pair index f M + m is the row of X
#pragma unroll
        for (int i = 0; i < KO; ++i)
            if (lane + 64 * i <= N2) out[lane + 64 * i] = xo[i];
    };
    float2 w2r[KO];
#pragma unroll
    for (int i = 0; i < KO; ++i) w2r[i] = tw2[min(lane + 64 * i, N2)];
    int64_t pr = pr0;
    if (pr < npair) fetch();
    for (; pr < npair; pr += step) {
        wave_sync();  // the previous pair's reads of the buffers are done
        if constexpr (R1) {
            // stage 1 (span 1, unit twiddles) into b1
#pragma unroll
            for (int bq = 0; bq < NL / 8; ++bq) {
                float2 v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    v[r] = float2{wr[8 * bq + 2 * r] * xs[8 * bq + 2 * r], wr[8 * bq + 2 * r + 1] * xs[8 * bq + 2 * r + 1]};
                const float2 s02 = float2{v[0].x + v[2].x, v[0].y + v[2].y}, d02 = float2{v[0].x - v[2].x, v[0].y - v[2].y};
                const float2 s13 = float2{v[1].x + v[3].x, v[1].y + v[3].y}, d13 = float2{v[1].x - v[3].x, v[1].y - v[3].y};
                float4* o = reinterpret_cast<float4*>(b1 + 4 * (lane + 64 * bq));
                o[0] = make_float4(s02.x + s13.x, s02.y + s13.y, d02.x + d13.y, d02.y - d13.x);
                o[1] = make_float4(s02.x - s13.x, s02.y - s13.y, d02.x - d13.y, d02.y + d13.x);
            }
        } else {
            // windowed samples, read as z[n] = x[2n] + i x[2n+1]
#pragma unroll
            for (int i = 0; i < NL; ++i)
                if (lane + 64 * i < N) b0f[lane + 64 * i] = wr[i] * xs[i];
        }
        wave_sync();
        if (opr >= 0) store();
        if (pr + step < npair) fetch();
        float2* a = R1 ? b1 : b0;
        float2* b = R1 ? b0 : b1;
        // radix-4 stages while four spans fit, then one radix-2 stage if
        // log2(N/2) is odd.  Butterfly j of span Ns takes inputs j + r N2/R,
        // multiplies input r by e^{-2 pi i r (j mod Ns) / (R Ns)}, and writes
        // the R-point DFT to R (j - j mod Ns) + j mod Ns + r Ns
        const int lg = NC > 0 ? ilog2c(NC / 2) : 31 - __builtin_clz(N2);
        int Ns = R1 ? 4 : 1;
#pragma unroll
        for (int r4 = R1 ? 1 : 0; r4 < lg / 2; ++r4, Ns *= 4) {
            const int Q = N2 / 4, ts = N2 / (4 * Ns);
#pragma unroll
            for (int j = lane; j < Q; j += 64) {
                const int k = j & (Ns - 1);
                const float2 v0 = a[j];
                const float2 v1 = cmul(a[j + Q], tw1[k * ts]);
                const float2 v2 = cmul(a[j + 2 * Q], tw1[2 * k * ts]);
                const float2 v3 = cmul(a[j + 3 * Q], tw1[3 * k * ts]);
                const float2 s02 = float2{v0.x + v2.x, v0.y + v2.y}, d02 = float2{v0.x - v2.x, v0.y - v2.y};
                const float2 s13 = float2{v1.x + v3.x, v1.y + v3.y}, d13 = float2{v1.x - v3.x, v1.y - v3.y};
                const int idx = ((j - k) << 2) + k;
                b[idx] = float2{s02.x + s13.x, s02.y + s13.y};
                b[idx + Ns] = float2{d02.x + d13.y, d02.y - d13.x};  // d02 - i d13
                b[idx + 2 * Ns] = float2{s02.x - s13.x, s02.y - s13.y};
                b[idx + 3 * Ns] = float2{d02.x - d13.y, d02.y + d13.x};  // d02 + i d13
            }
            wave_sync();
            float2* tmp = a;
            a = b;
            b = tmp;
        }
        if (lg & 1) {
            const int ts = N2 / (2 * Ns);
#pragma unroll
            for (int t = lane; t < N2 / 2; t += 64) {
                const int k = t & (Ns - 1);
                const float2 v0 = a[t], v1 = cmul(a[t + N2 / 2], tw1[k * ts]);
                const int idx = ((t - k) << 1) + k;
                b[idx] = float2{v0.x + v1.x, v0.y + v1.y};
                b[idx + Ns] = float2{v0.x - v1.x, v0.y - v1.y};
            }
            wave_sync();
            float2* tmp = a;
            a = b;
            b = tmp;
        }
        // even/odd split into the real-input bins (lanes past bin N/2 compute
        // bin N/2 again; it is not stored)
#pragma unroll
        for (int i = 0; i < KO; ++i) {
            const int k = min(lane + 64 * i, N2);
            const float2 zk = a[k & (N2 - 1)], zn = a[(N2 - k) & (N2 - 1)];
            const float er = 0.5f * (zk.x + zn.x), ei = 0.5f * (zk.y - zn.y);   // (Z[k] + conj Z[N2-k]) / 2
            const float orr = 0.5f * (zk.y + zn.y), oi = -0.5f * (zk.x - zn.x);  // (Z[k] - conj Z[N2-k]) / 2i
            const float2 w = w2r[i];
            xo[i] = float2{er + w.x * orr - w.y * oi, ei + w.x * oi + w.y * orr};
        }
        opr = pr;
    }
    if (opr >= 0) store();
}

}  // namespace

size_t stft_lds_bytes(int N) {
    const int N2 = N / 2;
    return sizeof(float2) * (2 * (size_t)N2 + 2) + sizeof(float) * (size_t)N +
           sizeof(float2) * (size_t)STFT_WAVES * 2 * N2;
}

void launch_stft(const float* pcm, int M, int64_t ld, int N, int hop, float2* X, int64_t F, int device,
                 hipStream_t s) {
    const int64_t npair = F * M;
    const int64_t want = (npair + STFT_WAVES - 1) / STFT_WAVES;
    // as many workgroups as the LDS lets one CU hold
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(160 * 1024) / (int64_t)stft_lds_bytes(N)));
    const int64_t cap = (int64_t)cu_count(device) * per_cu;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(want, cap));
    const size_t lds = stft_lds_bytes(N);
    switch (N) {
        case 16: case 32: k_stft<1, 0><<<grid, 64 * STFT_WAVES, lds, s>>>(pcm, M, ld, N, hop, X, npair); break;
        case 64: k_stft<1, 64><<<grid, 64 * STFT_WAVES, lds, s>>>(pcm, M, ld, N, hop, X, npair); break;
        case 128: k_stft<2, 128><<<grid, 64 * STFT_WAVES, lds, s>>>(pcm, M, ld, N, hop, X, npair); break;
        case 256: k_stft<4, 256><<<grid, 64 * STFT_WAVES, lds, s>>>(pcm, M, ld, N, hop, X, npair); break;
        case 512: k_stft<8, 512><<<grid, 64 * STFT_WAVES, lds, s>>>(pcm, M, ld, N, hop, X, npair); break;
        case 1024: k_stft<16, 1024><<<grid, 64 * STFT_WAVES, lds, s>>>(pcm, M, ld, N, hop, X, npair); break;
        default: k_stft<32, 2048><<<grid, 64 * STFT_WAVES, lds, s>>>(pcm, M, ld, N, hop, X, npair); break;
    }
}

}  // namespace svdphat
