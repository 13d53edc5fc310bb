// STFT front end (Section 2): each microphone signal analysed in frames of
// N samples, hop samples apart, with the sine window w[n] = sin(pi n / N):
//   X_m[f, k] = sum_{n<N} w[n] x_m[f hop + n] exp(-2 pi i k n / N),
//   k = 0 .. N/2, written as complex64 [F][M][N/2+1], the layout the
//   localisation path reads.
//
// One wave per (frame, microphone), grid-stride over the F M pairs.  The N
// windowed real samples are taken as N/2 complex points z[n] = x[2n] +
// i x[2n+1]; their FFT (radix-2 Stockham, natural order, in the wave's two
// LDS buffers) gives the N/2+1 real-input bins by the even/odd split
//   X[k] = (Z[k] + conj Z[N/2-k]) / 2 + e^{-2 pi i k / N} (Z[k] - conj Z[N/2-k]) / 2i.
// The twiddles and the window are evaluated once per workgroup in FP64 and
// kept in LDS as FP32.  All arithmetic is FP32.
#include "device.h"

namespace svdphat {

namespace {

constexpr int STFT_WAVES = 4;  // waves (pairs in flight) per workgroup

__global__ __launch_bounds__(256) void k_stft(const float* __restrict__ pcm, int M, int64_t ld, int N, int hop,
                                              float2* __restrict__ X, int64_t npair) {
    extern __shared__ __align__(16) char smem[];
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
    for (int64_t pr = (int64_t)blockIdx.x * STFT_WAVES + wave; pr < npair; pr += step) {
        const int64_t f = pr / M;
        const int m = (int)(pr - f * M);
        const float* src = pcm + (int64_t)m * ld + f * hop;
        wave_sync();  // the previous pair's reads of the buffers are done
        // windowed samples, read as z[n] = x[2n] + i x[2n+1]
        for (int n = lane; n < N; n += 64) b0f[n] = win[n] * src[n];
        wave_sync();
        float2* a = b0;
        float2* b = b1;
        for (int Ns = 1; Ns < N2; Ns <<= 1) {
            // butterflies t of span Ns: inputs t and t + N2/2, twiddle
            // e^{-2 pi i (t mod Ns) / (2 Ns)}, outputs 2 (t - t mod Ns) + t mod Ns
            // and that + Ns
            const int ts = N2 / (2 * Ns);
            for (int t = lane; t < N2 / 2; t += 64) {
                const int k = t & (Ns - 1);
                const float2 w = tw1[k * ts];
                const float2 v0 = a[t], u = a[t + N2 / 2];
                const float2 v1 = float2{u.x * w.x - u.y * w.y, u.x * w.y + u.y * w.x};
                const int idx = ((t - k) << 1) + k;
                b[idx] = float2{v0.x + v1.x, v0.y + v1.y};
                b[idx + Ns] = float2{v0.x - v1.x, v0.y - v1.y};
            }
            wave_sync();
            float2* tmp = a;
            a = b;
            b = tmp;
        }
        // even/odd split into the real-input bins; pair index f M + m is the
        // row of X
        float2* out = X + pr * B;
        for (int k = lane; k <= N2; k += 64) {
            const float2 zk = a[k & (N2 - 1)], zn = a[(N2 - k) & (N2 - 1)];
            const float er = 0.5f * (zk.x + zn.x), ei = 0.5f * (zk.y - zn.y);   // (Z[k] + conj Z[N2-k]) / 2
            const float orr = 0.5f * (zk.y + zn.y), oi = -0.5f * (zk.x - zn.x);  // (Z[k] - conj Z[N2-k]) / 2i
            const float2 w = tw2[k];
            out[k] = float2{er + w.x * orr - w.y * oi, ei + w.x * oi + w.y * orr};
        }
    }
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
    const int64_t cap = (int64_t)cu_count(device) * 6;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min(want, cap));
    k_stft<<<grid, 64 * STFT_WAVES, stft_lds_bytes(N), s>>>(pcm, M, ld, N, hop, X, npair);
}

}  // namespace svdphat
