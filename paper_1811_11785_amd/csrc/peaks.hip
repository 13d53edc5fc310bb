// Several sources per frame (the paper leaves multiple-source localisation
// to future work, Section 5): the n peaks of a frame's powers y over the
// grid, taken greedily.  Peak p is the largest y among the directions that
// are not an earlier peak and lie farther than the separation from every
// earlier peak (unit-vector dot product below cos_sep), ties to the lowest
// index; with no direction left the peak is -1 with value -inf.  The dot
// products are formed without fused multiply-adds ((x x' + y y') + z z',
// each product rounded), so that the comparisons with cos_sep are decided
// exactly as a float32 reference decides them.
//
// One wave per frame: each pass scans the frame's Q powers (lane-strided,
// coalesced) and takes the wave-wide (value, lowest index) maximum in
// registers; the chosen peaks' directions are wave-uniform.
#include "device.h"

namespace svdphat {

namespace {

constexpr int PEAKS_MAX = 16;

__device__ __forceinline__ float dot3(const float* a, float bx, float by, float bz) {
    return __fadd_rn(__fadd_rn(__fmul_rn(a[0], bx), __fmul_rn(a[1], by)), __fmul_rn(a[2], bz));
}

__global__ __launch_bounds__(256) void k_peaks(const float* __restrict__ y, int64_t F, int Q, int64_t ldy,
                                               const float* __restrict__ dirs, int n, float cos_sep,
                                               int32_t* __restrict__ idx, float* __restrict__ val) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t f = (int64_t)blockIdx.x * 4 + wave;
    if (f >= F) return;
    const float* yf = y + f * ldy;
    float px[PEAKS_MAX], py[PEAKS_MAX], pz[PEAKS_MAX];
    int pq[PEAKS_MAX];
    int np = 0;  // peaks found (wave-uniform)
    for (int p = 0; p < n; ++p) {
        float best = -INFINITY;
        int bi = 0x7fffffff;
        for (int q = lane; q < Q; q += 64) {
            const float v = yf[q];
            bool ok = v == v;  // NaN never counts
#pragma unroll
            for (int j = 0; j < PEAKS_MAX; ++j)
                if (j < np) ok = ok && q != pq[j] && !(dot3(dirs + 3 * (int64_t)q, px[j], py[j], pz[j]) >= cos_sep);
            if (ok && (bi == 0x7fffffff || v > best)) {  // lane-strided q rises, so ties keep the lower index
                best = v;
                bi = q;
            }
        }
        uint32_t w[2] = {__float_as_uint(best), (uint32_t)bi};
        wave_reduce(w, [](uint32_t (&x)[2], const uint32_t (&o)[2]) {
            const float xv = __uint_as_float(x[0]), ov = __uint_as_float(o[0]);
            const int xi = (int)x[1], oi = (int)o[1];
            // a found direction beats none; then the larger value; then the lower index
            const bool ob = oi != 0x7fffffff && (xi == 0x7fffffff || ov > xv || (ov == xv && oi < xi));
#pragma unroll
            for (int i = 0; i < 2; ++i) x[i] = blend(x[i], o[i], ob);
        });
        const int qb = __builtin_amdgcn_readfirstlane((int)w[1]);
        const float vb = __uint_as_float(__builtin_amdgcn_readfirstlane(w[0]));
        if (qb == 0x7fffffff) break;  // nothing left
        if (lane == 0) {
            idx[f * n + p] = qb;
            val[f * n + p] = vb;
        }
#pragma unroll
        for (int j = 0; j < PEAKS_MAX; ++j)
            if (j == np) {
                px[j] = dirs[3 * (int64_t)qb];
                py[j] = dirs[3 * (int64_t)qb + 1];
                pz[j] = dirs[3 * (int64_t)qb + 2];
                pq[j] = qb;
            }
        ++np;
    }
    for (int p = np + lane; p < n; p += 64) {
        idx[f * n + p] = -1;
        val[f * n + p] = -INFINITY;
    }
}

}  // namespace

int peaks_max() { return PEAKS_MAX; }

void launch_peaks(const float* y, int64_t F, int Q, int64_t ldy, const float* dirs, int n, float cos_sep,
                  int32_t* idx, float* val, hipStream_t s) {
    k_peaks<<<dim3((unsigned)((F + 3) / 4)), 256, 0, s>>>(y, F, Q, ldy, dirs, n, cos_sep, idx, val);
}

}  // namespace svdphat
