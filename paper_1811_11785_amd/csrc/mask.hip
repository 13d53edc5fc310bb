// Binary time-frequency mask (the paper names masks for several sources as
// future work, Section 5): bins a mask drops are removed from the
// cross-spectra of eq. (7), x_{p,k} = 0 for every pair p at a dropped bin k
// of that frame.  Eq. (3) gives 0 for a silent bin (|X|^2 below the
// smallest normal float counts as silent in every kernel), so a dropped bin
// written as 0 into a copy of the STFT frames gives exactly the masked x on
// the whole path, the row power of Algorithm 1 step 4 included.  Where the
// streamed GEMM1 serves a call, GEMM1 and the power read the mask
// themselves and only the hi/lo pass's listed frames are copied (here);
// otherwise every frame is.
#include "internal.h"

namespace svdphat {
namespace {

// four floats moved with one 16-byte access at an 8-byte aligned address
// (frames of an odd number of values start at any multiple of 8 bytes)
struct __attribute__((aligned(8))) f4u {
    float x, y, z, w;
};

// one thread per (frame, microphone, bin pair): 16-byte loads and stores of
// two bins, the mask byte(s) of the frame's bins
__global__ __launch_bounds__(256) void k_mask_x(const float2* __restrict__ X, int64_t F, int M, int B,
                                                const uint8_t* __restrict__ mask, float2* __restrict__ xm) {
    const int64_t n = F * M * B;
    for (int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2; i < n; i += (int64_t)gridDim.x * 512) {
        const int64_t f = i / ((int64_t)M * B);
        const int b = (int)(i % B);
        if (i + 1 < n && b + 1 < B) {
            const f4u v = *reinterpret_cast<const f4u*>(X + i);
            const uint8_t m0 = mask[f * B + b], m1 = mask[f * B + b + 1];
            *reinterpret_cast<f4u*>(xm + i) = f4u{m0 ? v.x : 0.f, m0 ? v.y : 0.f, m1 ? v.z : 0.f, m1 ? v.w : 0.f};
        } else {
            for (int64_t j = i; j < i + 2 && j < n; ++j) {
                const int64_t fj = j / ((int64_t)M * B);
                const int bj = (int)(j % B);
                xm[j] = mask[fj * B + bj] ? X[j] : make_float2(0.f, 0.f);
            }
        }
    }
}

// the listed frames only (the hi/lo pass's few frames): one workgroup per
// listed frame, grid-stride; a thread's MASK_PT values of the frame and
// their mask bytes are all loaded before any is stored, so a frame costs
// one round trip to memory instead of one per bin
constexpr int MASK_PT = 8;
__global__ __launch_bounds__(256) void k_mask_list(const float2* __restrict__ X, int M, int B,
                                                   const uint8_t* __restrict__ mask, const int* __restrict__ flist,
                                                   const int* __restrict__ fcount, float2* __restrict__ xm) {
    const int n = *fcount, MB = M * B;
    for (int pos = blockIdx.x; pos < n; pos += gridDim.x) {
        const int64_t f = flist[pos];
        const float2* xf = X + f * MB;
        const uint8_t* mk = mask + f * B;
        float2* out = xm + f * MB;
        for (int i0 = 0; i0 < MB; i0 += 256 * MASK_PT) {
            float2 v[MASK_PT];
            bool keep[MASK_PT];
#pragma unroll
            for (int j = 0; j < MASK_PT; ++j) {
                const int i = i0 + (int)threadIdx.x + 256 * j;
                const int ic = i < MB ? i : 0;
                v[j] = xf[ic];
                keep[j] = mk[ic % B] != 0;
            }
#pragma unroll
            for (int j = 0; j < MASK_PT; ++j) {
                const int i = i0 + (int)threadIdx.x + 256 * j;
                if (i < MB) out[i] = keep[j] ? v[j] : make_float2(0.f, 0.f);
            }
        }
    }
}

}  // namespace

void launch_mask_list(const svdphat_plan* p, const float2* X, const uint8_t* mask, const int* flist,
                      const int* fcount, float2* xm, hipStream_t s) {
    k_mask_list<<<dim3(256), 256, 0, s>>>(X, p->M, p->B, mask, flist, fcount, xm);
    SP_HIP(hipGetLastError());
}

void launch_mask(const svdphat_plan* p, const float2* X, int64_t F, const uint8_t* mask, float2* xm, hipStream_t s) {
    const int64_t pairs = (F * p->M * p->B + 1) / 2;
    const int64_t blocks = std::min<int64_t>((pairs + 255) / 256, 8192);
    k_mask_x<<<dim3((unsigned)blocks), 256, 0, s>>>(X, F, p->M, p->B, mask, xm);
    SP_HIP(hipGetLastError());
}

}  // namespace svdphat
