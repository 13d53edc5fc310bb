// Learned coarse-cell proposal for the search of eq. (14) (Section 3 replaces
// the O(Q) scan by a k-d tree over the normalised rows; this replaces it by
// a small network): an MLP maps the normalised projection
// f = [Re Z; Im Z] / ||Z|| (Z of eq. (12), S folded in) to C coarse cells of
// the direction grid; the scored directions inside the top cells are rescored
// exactly in FP32, and frames whose top probability is below a threshold fall
// back to the full search.  The network is trained on the GPU on
// (f, cell of the method's own argmax) pairs with hand-written FP16 MFMA
// kernels (forward, backward, weight gradients), FP32 master weights and Adam.
//
// Network: f (2K) -> GELU(W1 f + b1) (H) -> GELU(W2 . + b2) (H) -> W3 . + b3
// (C), GELU(v) = v (1 + erf(v / sqrt 2)) / 2 with erf to 1.5e-7, softmax
// cross-entropy.
#include "device.h"

#include <cstring>
#include <random>

namespace svdphat {

namespace {

constexpr int GT = 64;   // output tile (rows and columns) of the MLP GEMM
constexpr int GK = 32;   // reduction step
constexpr int GPAD = 8;

enum { EPI_GELU = 0, EPI_BIAS = 1, EPI_DGELU = 2, EPI_F32 = 3 };

// erf by formula 7.1.26 of Abramowitz and Stegun's Handbook of Mathematical
// Functions (absolute error at most 1.5e-7), without branches; ex receives
// exp(-x^2), which GELU' needs as well
__device__ __forceinline__ float erf_as(float x, float& ex) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.f));
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    ex = __expf(-ax * ax);
    return copysignf(fmaf(-q * t, ex, 1.f), x);
}
__device__ __forceinline__ float gelu_f(float v) {
    float e;
    return 0.5f * v * (1.f + erf_as(v * 0.70710678118654752f, e));
}
// GELU'(v) = (1 + erf(v / sqrt 2)) / 2 + v exp(-v^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_d(float v) {
    float e;
    const float er = erf_as(v * 0.70710678118654752f, e);
    return 0.5f * (1.f + er) + v * 0.39894228040143268f * e;
}

// C(m, n) = sum_k A(m, k) B(n, k) for m < M, n < N, k in [kbeg, kend), f16
// operands, FP32 accumulation on 16x16x32 MFMA.  A(m, k) = A[m*lda + k]
// (AT false) or A[k*lda + m] (AT true); B(n, k) = B[n*ldb + k] (BT false)
// or B[k*ldb + n] (BT true).  Workgroup: 4 waves, 64 x 64 outputs, each
// wave 16 rows x 64 columns.  Epilogues:
//   EPI_GELU   pre = acc + bias[n] -> out32 (pre-activation), out16 = GELU(pre)
//   EPI_BIAS   out32 = acc + bias[n]
//   EPI_DGELU  out16 = acc * GELU'(pre32[m, n])
//   EPI_F32    out32[split][m][n] = acc (split-K partials over blockIdx.z)
template <int EPI>
__device__ __forceinline__ void mlp_epilogue(const f4 (&acc)[4], int m0, int n0, int wave, int lane, int M, int N,
                                             const float* __restrict__ bias, const float* __restrict__ pre32,
                                             float* __restrict__ out32, _Float16* __restrict__ out16, int ldo) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = m0 + wave * 16 + 4 * (lane >> 4) + e;
            const int n = n0 + j * 16 + (lane & 15);
            if (m >= M || n >= N) continue;
            const float v = acc[j][e];
            const int64_t o = (int64_t)m * ldo + n;
            if (EPI == EPI_GELU) {
                const float pv = v + bias[n];
                out32[o] = pv;
                out16[o] = (_Float16)gelu_f(pv);
            } else if (EPI == EPI_BIAS) {
                out32[o] = v + bias[n];
            } else if (EPI == EPI_DGELU) {
                out16[o] = (_Float16)(v * gelu_d(pre32[o]));
            } else {
                out32[(int64_t)blockIdx.z * M * ldo + o] = v;
            }
        }
}

template <bool AT, bool BT, int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm(const _Float16* __restrict__ A, int lda,
                                                  const _Float16* __restrict__ Bm, int ldb, int M, int N, int K,
                                                  int ksplit, const float* __restrict__ bias,
                                                  const float* __restrict__ pre32, float* __restrict__ out32,
                                                  _Float16* __restrict__ out16, int ldo) {
    __shared__ __align__(16) _Float16 As[GT][GK + GPAD];
    __shared__ __align__(16) _Float16 Bs[GT][GK + GPAD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
    const int kper = (K + ksplit - 1) / ksplit;
    const int kbeg = blockIdx.z * kper, kend = min(K, kbeg + kper);
    f4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    // a transposed operand's 8 consecutive elements of a row in one 16-byte
    // load where the row pitch and the pointer allow it
    const bool va = AT && lda % 8 == 0 && ((uintptr_t)A & 15) == 0;
    const bool vb = BT && ldb % 8 == 0 && ((uintptr_t)Bm & 15) == 0;
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        // stage 64 x 32 tiles of A and B with the reduction axis contiguous
        if (!AT) {
            const int r = tid >> 2, kk = (tid & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int m = m0 + r, k = k0 + kk + e;
                As[r][kk + e] = (m < M && k < kend) ? A[(int64_t)m * lda + k] : (_Float16)0.f;
            }
        } else {
            const int kk = tid >> 3, r = (tid & 7) * 8;
            if (va && m0 + r + 8 <= M && k0 + kk < kend) {
                const h8 v = *reinterpret_cast<const h8*>(A + (int64_t)(k0 + kk) * lda + m0 + r);
#pragma unroll
                for (int e = 0; e < 8; ++e) As[r + e][kk] = v[e];
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int m = m0 + r + e, k = k0 + kk;
                    As[r + e][kk] = (m < M && k < kend) ? A[(int64_t)k * lda + m] : (_Float16)0.f;
                }
            }
        }
        if (!BT) {
            const int r = tid >> 2, kk = (tid & 3) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int n = n0 + r, k = k0 + kk + e;
                Bs[r][kk + e] = (n < N && k < kend) ? Bm[(int64_t)n * ldb + k] : (_Float16)0.f;
            }
        } else {
            const int kk = tid >> 3, r = (tid & 7) * 8;
            if (vb && n0 + r + 8 <= N && k0 + kk < kend) {
                const h8 v = *reinterpret_cast<const h8*>(Bm + (int64_t)(k0 + kk) * ldb + n0 + r);
#pragma unroll
                for (int e = 0; e < 8; ++e) Bs[r + e][kk] = v[e];
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int n = n0 + r + e, k = k0 + kk;
                    Bs[r + e][kk] = (n < N && k < kend) ? Bm[(int64_t)k * ldb + n] : (_Float16)0.f;
                }
            }
        }
        __syncthreads();
        const h8 a = *reinterpret_cast<const h8*>(&As[wave * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const h8 b = *reinterpret_cast<const h8*>(&Bs[j * 16 + (lane & 15)][8 * (lane >> 4)]);
            acc[j] = mfma(a, b, acc[j]);
        }
        __syncthreads();
    }
    mlp_epilogue<EPI>(acc, m0, n0, wave, lane, M, N, bias, pre32, out32, out16, ldo);
}

// The same for row-major operands whose reduction axis is contiguous (A(m,
// k) = A[m lda + k], B(n, k) = B[n ldb + k]) with lda, ldb, the k range and
// the pointers multiples of 8 elements: each thread stages one 16-byte piece
// of each 64 x 32 tile, and the next tile's pieces are loaded before the
// current tile's MFMAs.
template <int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm_v(const _Float16* __restrict__ A, int lda,
                                                    const _Float16* __restrict__ Bm, int ldb, int M, int N, int K,
                                                    int ksplit, const float* __restrict__ bias,
                                                    const float* __restrict__ pre32, float* __restrict__ out32,
                                                    _Float16* __restrict__ out16, int ldo) {
    __shared__ __align__(16) _Float16 As[GT][GK + GPAD];
    __shared__ __align__(16) _Float16 Bs[GT][GK + GPAD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
    const int kper = (K + ksplit - 1) / ksplit;
    const int kbeg = blockIdx.z * kper, kend = min(K, kbeg + kper);
    const int r = tid >> 2, kk = (tid & 3) * 8;
    const int m = m0 + r, n = n0 + r;
    const _Float16* pa = A + (int64_t)min(m, M - 1) * lda;
    const _Float16* pb = Bm + (int64_t)min(n, N - 1) * ldb;
    f4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    const h8 zero = {};
    h8 va = zero, vb = zero;
    auto load = [&](int k0) {
        // rows past M or N and k past the range stage zeros (the clamped
        // address stays inside the operand)
        // (k range and lengths are multiples of 8: a piece is all inside or
        // all outside; the clamped offset keeps its 8 elements in the row)
        const bool ka = k0 + kk < kend;
        const int ko = min(k0 + kk, kend - 8);
        const h8 la = *reinterpret_cast<const h8*>(pa + ko);
        const h8 lb = *reinterpret_cast<const h8*>(pb + ko);
        va = (m < M && ka) ? la : zero;
        vb = (n < N && ka) ? lb : zero;
    };
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        *reinterpret_cast<h8*>(&As[r][kk]) = va;
        *reinterpret_cast<h8*>(&Bs[r][kk]) = vb;
        __syncthreads();
        if (k0 + GK < kend) load(k0 + GK);
        const h8 a = *reinterpret_cast<const h8*>(&As[wave * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const h8 b = *reinterpret_cast<const h8*>(&Bs[j * 16 + (lane & 15)][8 * (lane >> 4)]);
            acc[j] = mfma(a, b, acc[j]);
        }
        __syncthreads();
    }
    mlp_epilogue<EPI>(acc, m0, n0, wave, lane, M, N, bias, pre32, out32, out16, ldo);
}

// f = z / ||z|| in f16 (0 for z = 0); z32 rows [F][Rp] already stacked.
__global__ void k_features(const float* __restrict__ z32, const float* __restrict__ zn, int64_t F, int Rp,
                           _Float16* __restrict__ feat) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F * Rp) return;
    const int64_t f = i / Rp;
    const float n = zn[f];
    feat[i] = (_Float16)(n > 0.f ? z32[i] / n : 0.f);
}

// FP16 network input [F][ld] widened to FP32 [F][D] (testing aid)
__global__ void k_widen(const _Float16* __restrict__ h, int64_t F, int D, int ld, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F * D) return;
    out[i] = (float)h[(i / D) * ld + i % D];
}

__global__ void k_labels(const int32_t* __restrict__ doa, const int32_t* __restrict__ cell_of_dir, int64_t F,
                         int32_t* __restrict__ lab) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < F) lab[f] = cell_of_dir[doa[f]];
}

// Softmax cross-entropy, one wave per frame: loss[f] = -log p[label], and
// d logits = p - onehot (summed over frames, i.e. the mean loss scaled by F;
// the weight update divides by F).
__global__ __launch_bounds__(256) void k_xent(const float* __restrict__ logits, int ld, int C,
                                              const int32_t* __restrict__ lab, int64_t F, _Float16* __restrict__ dlog,
                                              float* __restrict__ loss) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t f = (int64_t)blockIdx.x * 4 + wave;
    if (f >= F) return;
    const float* l = logits + f * ld;
    float mx = -INFINITY;
    for (int c = lane; c < C; c += 64) mx = fmaxf(mx, l[c]);
    mx = wave_max(mx);
    float se = 0.f;
    for (int c = lane; c < C; c += 64) se += __expf(l[c] - mx);
    se = wave_sum(se);
    const int y = lab[f];
    for (int c = lane; c < ld; c += 64) {
        const float p = c < C ? __expf(l[c] - mx) / se : 0.f;
        dlog[f * ld + c] = (_Float16)(p - (c == y ? 1.f : 0.f));
    }
    if (lane == 0) loss[f] = -(l[y] - mx - __logf(se));
}

// Column sums over frames of an f16 matrix [F][ld] (bias gradients), in
// gridDim.y partial sums over equal runs of frames: out[part][n] (the Adam
// step adds the partials in order).
__global__ void k_colsum(const _Float16* __restrict__ d, int64_t F, int N, int ld, float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t per = (F + gridDim.y - 1) / gridDim.y;
    const int64_t fb = (int64_t)blockIdx.y * per, fe = min(F, fb + per);
    float s = 0.f;
    for (int64_t f = fb; f < fe; ++f) s += (float)d[f * ld + n];
    out[(int64_t)blockIdx.y * N + n] = s;
}

// partial sums of a bias gradient over F frames (runs of at least 128)
constexpr int BSPLIT = 64;
inline int bias_parts(int64_t F) { return (int)std::max<int64_t>(1, std::min<int64_t>(BSPLIT, (F + 127) / 128)); }

struct AdamSeg {
    int64_t off;       // offset in the flat parameter arrays
    int rows, cols;    // weight shape (cols = 1 for a bias)
    int parts;         // split-K partials of the gradient
    const float* g;    // [parts][rows][cols] (weights) or [rows] (bias)
    _Float16* wh;      // f16 copy [rows][cols] or null
    _Float16* wt;      // f16 transpose [cols][rows] or null
    int ldh, ldt;      // leading dimensions of the copies
};

// Adam (Kingma & Ba) with bias correction; gradients are the sum over the
// batch's frames and are divided by F here.
__global__ void k_adam(AdamSeg sg, float* __restrict__ P, float* __restrict__ Mm, float* __restrict__ Vv, float inv_f,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)sg.rows * sg.cols;
    if (i >= n) return;
    float g = 0.f;
    for (int s = 0; s < sg.parts; ++s) g += sg.g[(int64_t)s * n + i];
    g *= inv_f;
    const int64_t o = sg.off + i;
    const float m = b1 * Mm[o] + (1.f - b1) * g;
    const float v = b2 * Vv[o] + (1.f - b2) * g * g;
    Mm[o] = m;
    Vv[o] = v;
    const float p = P[o] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    P[o] = p;
    const int r = (int)(i / sg.cols), c = (int)(i % sg.cols);
    if (sg.wh) sg.wh[(int64_t)r * sg.ldh + c] = (_Float16)p;
    if (sg.wt) sg.wt[(int64_t)c * sg.ldt + r] = (_Float16)p;
}

// f16 copies of the FP32 weights (after set_params)
__global__ void k_cast_w(const float* __restrict__ W, int rows, int cols, _Float16* __restrict__ wh, int ldh,
                         _Float16* __restrict__ wt, int ldt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * cols) return;
    const int r = (int)(i / cols), c = (int)(i % cols);
    wh[(int64_t)r * ldh + c] = (_Float16)W[i];
    wt[(int64_t)c * ldt + r] = (_Float16)W[i];
}

// Wf: W [N][K] (f16, N a multiple of 64, K of 32) in the MFMA B-fragment
// order of k_mlp_infer: element (n, k) at ((((n / 64) (K / 32) + k / 32) 4 +
// (n / 16) mod 4) 64 + n mod 16 + 16 ((k / 8) mod 4)) 8 + k mod 8.  One
// thread per 8 consecutive k of a row.
__global__ void k_pack_wf(const _Float16* __restrict__ wh, int N, int K, _Float16* __restrict__ wf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int kc = K / 8;
    if (i >= (int64_t)N * kc) return;
    const int n = (int)(i / kc), k = (int)(i - (int64_t)n * kc) * 8;
    const int g = n >> 6, cb = (n >> 4) & 3, ks = k >> 5, lane = (n & 15) + 16 * ((k >> 3) & 3);
    const int64_t off = ((((int64_t)g * (K / 32) + ks) * 4 + cb) * 64 + lane) * 8;
    *reinterpret_cast<h8*>(wf + off) = *reinterpret_cast<const h8*>(wh + (int64_t)n * K + k);
}

// ------------------------------------------------------------- inference
// Inference runs in stages:
//   k_mlp_infer   the forward pass of FT frames per workgroup, activations in
//                 LDS, FP32 logits out;
//   k_select      per frame the softmax top probability (below conf_min: the
//                 full search) and the topk most probable cells that hold
//                 scored rows, each entered in its cell's pair list;
//   k_cell_scan   list offsets per cell, the rescoring work items (a cell
//                 and up to PT of its frames) and the list of frames for the
//                 full search, in frame order;
//   k_scatter     the pair lists (the frames of each cell);
//   k_rescore     per work item the cell's scored rows against its frames'
//                 z in FP32 on MFMA (rows staged once for the item), the best
//                 (y, lowest direction) per frame into a 64-bit atomic max;
//   k_prop_final  direction and row power (Algorithm 1 step 4) per frame.
// Grouping the pairs by cell reads each cell's rows once per PT frames
// instead of once per frame.

constexpr int PT = 64;       // frames per rescoring item
constexpr int SEL_FPW = 2;   // frames per wave in the selection

// The forward pass for inference: features f = z / ||z|| (f16), GELU(W1 f +
// b1), GELU(W2 . + b2), W3 . + b3, for FT frames per workgroup of 4 waves.
// Activations stay in LDS in two buffers ([FT][max(D0, H) + 8] and [FT][H +
// 8] halves); the weights are read as B fragments from their f16 copies
// (L2-resident; packed in fragment order, so that a fragment load reads
// 1 KB in one piece), two k-steps ahead of their MFMAs.  The arithmetic is that
// of the training path (f16 operands, FP32 accumulation, bias and GELU in
// FP32, f16 hidden activations).  Writes FP32 logits [F][Cp].
template <int FT>
__global__ __launch_bounds__(256) void k_mlp_infer(const float* __restrict__ z32, const float* __restrict__ zn,
                                                   int64_t F, int D0, int H, int Cp,
                                                   const _Float16* __restrict__ W1, const float* __restrict__ b1,
                                                   const _Float16* __restrict__ W2, const float* __restrict__ b2,
                                                   const _Float16* __restrict__ W3, const float* __restrict__ b3,
                                                   float* __restrict__ logits) {
    constexpr int RB = FT / 16;
    extern __shared__ __align__(16) char smem[];
    const int L0 = max(D0, H) + 8, L1 = H + 8;
    _Float16* buf0 = reinterpret_cast<_Float16*>(smem);
    _Float16* buf1 = buf0 + FT * L0;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t f0 = (int64_t)blockIdx.x * FT;
    // features (frames past F: 0)
    const int q4 = D0 / 4;
    for (int i = tid; i < FT * q4; i += 256) {
        const int r = i / q4, c = 4 * (i - r * q4);
        const int64_t f = f0 + r;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        float n = 0.f;
        if (f < F) {
            v = *reinterpret_cast<const float4*>(z32 + f * D0 + c);
            n = zn[f];
        }
        _Float16* d = buf0 + r * L0 + c;
        d[0] = (_Float16)(n > 0.f ? v.x / n : 0.f);
        d[1] = (_Float16)(n > 0.f ? v.y / n : 0.f);
        d[2] = (_Float16)(n > 0.f ? v.z / n : 0.f);
        d[3] = (_Float16)(n > 0.f ? v.w / n : 0.f);
    }
    __syncthreads();
    // out(m, n) = sum_k in(m, k) W(n, k) for the FT rows and n < N, in
    // groups of 64 columns (wave w: groups w, w + 4, ...); epi(acc, group)
    auto layer = [&](const _Float16* in, int ldi, int K, const _Float16* __restrict__ W, int N, auto&& epi) {
        for (int g = wave; g * 64 < N; g += 4) {
            f4 acc[RB][4];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
            // W in fragment order: fragment (k-step ks, column block cb) of
            // group g is 64 lanes x 8 halves at wp + (ks 4 + cb) 512
            const int nks = K / 32;
            const _Float16* wp = W + ((int64_t)g * nks * 4 * 64 + lane) * 8;
            auto frag = [&](int ks, int cb) {
                return *reinterpret_cast<const h8*>(wp + (int64_t)(ks * 4 + cb) * 512);
            };
            // B fragments two k-steps ahead (k-steps past the end reload the
            // last one)
            h8 b1[4], b2[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                b1[cb] = frag(0, cb);
                b2[cb] = frag(min(1, nks - 1), cb);
            }
            for (int k0 = 0, ks = 0; k0 < K; k0 += 32, ++ks) {
                h8 b[4];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    b[cb] = b1[cb];
                    b1[cb] = b2[cb];
                }
                const int kn = min(ks + 2, nks - 1);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) b2[cb] = frag(kn, cb);
                h8 a[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    a[rb] = *reinterpret_cast<const h8*>(in + (rb * 16 + (lane & 15)) * ldi + k0 + 8 * (lane >> 4));
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = mfma(a[rb], b[cb], acc[rb][cb]);
            }
            epi(acc, g);
        }
    };
    // hidden epilogue: GELU(acc + bias) in f16 into out [FT][ldo]
    // (D layout: lane holds rows 4 (lane / 16) + e of column lane % 16)
    auto hidden = [&](const float* __restrict__ bias, _Float16* out, int ldo) {
        return [=](f4 (&acc)[RB][4], int g) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int n = g * 64 + cb * 16 + (lane & 15);
                const float bv = bias[n];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        out[(rb * 16 + 4 * (lane >> 4) + e) * ldo + n] = (_Float16)gelu_f(acc[rb][cb][e] + bv);
            }
        };
    };
    layer(buf0, L0, D0, W1, H, hidden(b1, buf1, L1));
    __syncthreads();
    layer(buf1, L1, H, W2, H, hidden(b2, buf0, L0));
    __syncthreads();
    layer(buf0, L0, H, W3, Cp, [&](f4 (&acc)[RB][4], int g) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int n = g * 64 + cb * 16 + (lane & 15);
            const float bv = b3[n];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t f = f0 + rb * 16 + 4 * (lane >> 4) + e;
                    // (streamed past the caches: read once, by the selection)
                    if (f < F) __builtin_nontemporal_store(acc[rb][cb][e] + bv, logits + f * Cp + n);
                }
        }
    });
}

// LDS bytes of k_mlp_infer for FT frames
inline size_t mlp_infer_lds(int FT, int D0, int H) {
    return (size_t)FT * (std::max(D0, H) + 8 + H + 8) * sizeof(_Float16);
}

// Selection, one wave per frame, SEL_FPW frames per wave (C <= 1024).  A
// frame whose top probability is below conf_min, or whose topk cells hold
// no scored row, takes the full search (fell = 1, ntop = 0).  Otherwise its
// ntop cells with rows (in order of probability, lowest index on ties) go to
// cand[f topk + t], with their slot in the cell's pair list in slot[..]:
// a slot in a workgroup histogram (LDS) plus the workgroup's base, one
// global add per cell the workgroup names.  stats (optional): rows to be
// rescored and frames that take the proposal.
// NJ = ceil(C / 64) logits per lane: the selection is VALU-bound, and every
// slot costs in each of its passes (maximum, exponentials, keys, topk rounds)
template <int NJ>
__global__ __launch_bounds__(256) void k_select(const float* __restrict__ logits, int ld, int C, int topk,
                                                float conf_min, const int32_t* __restrict__ cstart, int64_t F,
                                                uint8_t* __restrict__ fell, int32_t* __restrict__ ntop,
                                                int32_t* __restrict__ cand, int32_t* __restrict__ slot,
                                                int* __restrict__ ccount, unsigned long long* __restrict__ best,
                                                unsigned long long* __restrict__ stats) {
    __shared__ int hist[1024];
    __shared__ int base[1024];
    __shared__ int cnr[1024];  // scored rows of each cell
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int c = tid; c < C; c += 256) {
        hist[c] = 0;
        cnr[c] = cstart[c + 1] - cstart[c];
    }
    __syncthreads();
    const int64_t fw = ((int64_t)blockIdx.x * 4 + wave) * SEL_FPW;
    int nsel[SEL_FPW];
    unsigned long long rows_sum = 0, nconf = 0;
    // logits of a frame's cells, up to 64 NJ in registers (lane + 64 j)
    // (frame index clamped into range, so that the loads need no branch)
    float lv[NJ];
    auto load = [&](float (&v)[NJ], int64_t f) {
        const float* l = logits + min(f, F - 1) * ld;
#pragma unroll
        for (int j = 0; j < NJ; ++j) v[j] = __builtin_nontemporal_load(l + min(lane + 64 * j, C - 1));
    };
#pragma unroll
    for (int i = 0; i < SEL_FPW; ++i) {
        nsel[i] = 0;
        const int64_t f = fw + i;
        load(lv, f);
        if (f < F) {
            float mx = -INFINITY;
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                if (lane + 64 * j >= C) lv[j] = -INFINITY;
                mx = fmaxf(mx, lv[j]);
            }
            mx = wave_max(mx);
            float se = 0.f;
#pragma unroll
            for (int j = 0; j < NJ; ++j) se += lv[j] > -INFINITY ? __expf(lv[j] - mx) : 0.f;
            se = wave_sum(se);
            int n = 0;
            unsigned long long rs = 0;
            if (1.f / se >= conf_min) {
                // cells ranked by one 32-bit key: the logit's order-preserving
                // bits to 13 mantissa bits, then the lowest index (key 0: none)
                uint32_t key[NJ];
                uint32_t km = 0;
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const uint32_t b = __float_as_uint(lv[j]);
                    const uint32_t o = b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
                    key[j] = lv[j] > -INFINITY ? ((o & ~0x3FFu) | (uint32_t)(1023 - (lane + 64 * j))) : 0u;
                    km = max(km, key[j]);
                }
                for (int t = 0; t < topk; ++t) {
                    uint32_t w[1] = {km};
                    wave_reduce(w, [](uint32_t (&x)[1], const uint32_t (&o)[1]) { x[0] = max(x[0], o[0]); });
                    const uint32_t kw = __builtin_amdgcn_readfirstlane(w[0]);
                    if (kw == 0u) break;
                    const int c = 1023 - (int)(kw & 0x3FFu);
                    km = 0;
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        key[j] = key[j] == kw ? 0u : key[j];
                        km = max(km, key[j]);
                    }
                    const int nr = cnr[c];
                    if (nr == 0) continue;  // an empty cell: nothing to rescore
                    rs += (unsigned long long)nr;
                    if (lane == 0) {
                        cand[f * topk + n] = c;
                        slot[f * topk + n] = atomicAdd(&hist[c], 1);
                    }
                    ++n;
                }
            }
            nsel[i] = n;
            if (n > 0) {
                rows_sum += rs;
                nconf += 1;
            }
            if (lane == 0) {
                fell[f] = n == 0 ? 1 : 0;
                ntop[f] = n;
                best[f] = 0ull;
            }
        }
    }
    __syncthreads();
    for (int c = tid; c < C; c += 256)
        if (hist[c] > 0) base[c] = atomicAdd(&ccount[c], hist[c]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SEL_FPW; ++i) {
        const int64_t f = fw + i;
        for (int t = lane; t < nsel[i]; t += 64) {
            const int64_t e = f * topk + t;
            slot[e] += base[cand[e]];
        }
    }
    if (stats && lane == 0 && nconf > 0) {
        atomicAdd(&stats[0], rows_sum);
        atomicAdd(&stats[1], nconf);
    }
}

// Exclusive prefix sum over the 1024 threads of the workgroup (total in
// *tot): a scan within each wave, then over the 16 wave totals; every
// thread must call it.  sw: 16 ints of LDS.
__device__ __forceinline__ int block_exscan1024(int v, int* sw, int* tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) sw[wave] = x;
    __syncthreads();
    int below = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const int t = sw[w];
        below += w < wave ? t : 0;
        all += t;
    }
    *tot = all;
    __syncthreads();  // (sw free for the next scan)
    return below + x - v;
}

// One workgroup of 1024 threads: cell list offsets, rescoring items and the
// full-search frame list in frame order (fell set).
__global__ __launch_bounds__(1024) void k_cell_scan(const int* __restrict__ ccount, int C, int* __restrict__ cpos,
                                                    int4* __restrict__ items, int* __restrict__ nitems,
                                                    const uint8_t* __restrict__ fell, int64_t F,
                                                    int* __restrict__ flist, int* __restrict__ fcount) {
    __shared__ int sa[16];
    const int t = threadIdx.x;
    const int cnt = t < C ? ccount[t] : 0;
    const int nch = (cnt + PT - 1) / PT;
    int tot_pairs = 0, tot_items = 0;
    const int pa = block_exscan1024(cnt, sa, &tot_pairs);
    const int pb = block_exscan1024(nch, sa, &tot_items);
    if (t < C) {
        cpos[t] = pa;
        for (int j = 0; j < nch; ++j) items[pb + j] = int4{t, pa + j * PT, min(PT, cnt - j * PT), 0};
    }
    if (t == 0) *nitems = tot_items;
    int run = 0;
    for (int64_t f0 = 0; f0 < F; f0 += 4096) {
        int k = 0;
        uint8_t fl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t f = f0 + 4 * t + j;
            fl[j] = f < F ? fell[f] : 0;
            k += fl[j] ? 1 : 0;
        }
        int tot = 0;
        int o = run + block_exscan1024(k, sa, &tot);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (fl[j]) flist[o++] = (int)(f0 + 4 * t + j);
        run += tot;
    }
    if (t == 0) *fcount = run;
}

// The pair lists: frame f at cpos[cell] + slot for each of its entries.
__global__ void k_scatter(const int32_t* __restrict__ ntop, const int32_t* __restrict__ cand,
                          const int32_t* __restrict__ slot, const int* __restrict__ cpos, int64_t F, int topk,
                          int32_t* __restrict__ pairs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F * topk) return;
    const int64_t f = e / topk;
    if (e - f * topk >= ntop[f]) return;
    pairs[cpos[cand[e]] + slot[e]] = (int)f;
}

// 64-bit key of (y, direction q): larger y first, then lower q
__device__ __forceinline__ unsigned long long yq_key(float y, int q) {
    uint32_t u = __float_as_uint(y);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)q);
}

// Rescoring, one workgroup per item (cell c, up to PT frames): the cell's
// scored rows (FP32, cell-ordered copy of U) in chunks of 64 rows against the
// frames' z in FP32 on 16x16x4 MFMA.  The frames' z and the chunk's rows go
// through LDS ([PT + 64][KC + 4] floats, the reduction axis in chunks of KC),
// each thread issuing four 16-byte loads before their four stores.  Per
// frame the best (y, lowest q) over the cell goes into best[f] (64-bit atomic
// max, so the order of items does not matter).
__global__ __launch_bounds__(256) void k_rescore(const int4* __restrict__ items, const int* __restrict__ nitems,
                                                 const int32_t* __restrict__ pairs, const float* __restrict__ z32,
                                                 int Rp, int KC, const float* __restrict__ U32C,
                                                 const int32_t* __restrict__ cstart, const int32_t* __restrict__ cdir,
                                                 unsigned long long* __restrict__ best) {
    if ((int)blockIdx.x >= *nitems) return;
    extern __shared__ __align__(16) char smem[];
    const int LD = KC + 4;
    float* zs = reinterpret_cast<float*>(smem);  // rows 0 .. PT-1: z; PT .. PT+63: U
    const float* us = zs + PT * LD;
    __shared__ int frm[PT];
    __shared__ int qd[64];
    __shared__ unsigned long long kb[PT];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int4 w = items[blockIdx.x];
    const int c = w.x, p0 = w.y, n = w.z;
    const int r0 = cstart[c], nr = cstart[c + 1] - r0;
    if (tid < PT) {
        frm[tid] = tid < n ? pairs[p0 + tid] : -1;
        kb[tid] = 0ull;
    }
    const int nfb = (n + 15) / 16;
    for (int rc = 0; rc < nr; rc += 64) {
        const int nrc = min(64, nr - rc);
        const int nrb = (nrc + 15) / 16, ntile = nrb * nfb;
        const int nt = ntile > wave ? (ntile - wave + 3) / 4 : 0;  // tiles of this wave: wave, wave + 4, ...
        f4 acc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < Rp; k0 += KC) {
            const int kn = min(KC, Rp - k0), q4 = kn / 4, tot = (PT + 64) * q4;
            __syncthreads();  // (frm ready; the previous chunk's reads of LDS done)
            if (k0 == 0 && tid < 64) qd[tid] = tid < nrc ? cdir[r0 + rc + tid] : 0;
            for (int i0 = 0; i0 < tot; i0 += 1024) {
                float4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = min(i0 + tid + 256 * u, tot - 1);
                    const int j = i / q4, cc = 4 * (i - j * q4);
                    const float* src = j < PT ? z32 + (int64_t)max(frm[j], 0) * Rp + k0 + cc
                                              : U32C + (int64_t)(r0 + rc + min(j - PT, nrc - 1)) * Rp + k0 + cc;
                    v[u] = *reinterpret_cast<const float4*>(src);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + tid + 256 * u;
                    if (i < tot) {
                        const int j = i / q4, cc = 4 * (i - j * q4);
                        const bool ok = j < PT ? frm[j] >= 0 : j - PT < nrc;
                        const float4 x = v[u];
                        *reinterpret_cast<float4*>(zs + j * LD + cc) =
                            make_float4(ok ? x.x : 0.f, ok ? x.y : 0.f, ok ? x.z : 0.f, ok ? x.w : 0.f);
                    }
                }
            }
            __syncthreads();
            // the wave's tiles, their MFMAs interleaved (independent accumulators)
            const float* ua[4];
            const float* zb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int tile = min(wave + 4 * i, ntile - 1);
                const int rb = tile / nfb, fb = tile - rb * nfb;
                ua[i] = us + (rb * 16 + (lane & 15)) * LD + (lane >> 4);
                zb[i] = zs + (fb * 16 + (lane & 15)) * LD + (lane >> 4);
            }
            if (nt == 4) {
                for (int k = 0; k < kn; k += 4)
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[i] = mfma(ua[i][k], zb[i][k], acc[i]);
            } else if (nt == 3) {
                for (int k = 0; k < kn; k += 4)
#pragma unroll
                    for (int i = 0; i < 3; ++i) acc[i] = mfma(ua[i][k], zb[i][k], acc[i]);
            } else if (nt == 2) {
                for (int k = 0; k < kn; k += 4)
#pragma unroll
                    for (int i = 0; i < 2; ++i) acc[i] = mfma(ua[i][k], zb[i][k], acc[i]);
            } else if (nt == 1) {
                for (int k = 0; k < kn; k += 4) acc[0] = mfma(ua[0][k], zb[0][k], acc[0]);
            }
        }
        // per frame: best over the chunk's rows (D layout: lane holds rows
        // 4 (lane / 16) + e of frame column lane % 16)
        auto epi = [&](const f4& av, int i) {
            const int tile = min(wave + 4 * i, ntile - 1);
            const bool live = wave + 4 * i < ntile;
            const int rb = tile / nfb, fb = tile - rb * nfb;
            unsigned long long k = 0ull;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rb * 16 + 4 * (lane >> 4) + e;
                const unsigned long long ke = yq_key(av[e], qd[min(row, 63)]);
                k = (live && row < nrc && ke > k) ? ke : k;
            }
            const unsigned long long k16 = (unsigned long long)__shfl_xor((long long)k, 16);
            k = k16 > k ? k16 : k;
            const unsigned long long k32 = (unsigned long long)__shfl_xor((long long)k, 32);
            k = k32 > k ? k32 : k;
            const int j = fb * 16 + lane;
            if (live && lane < 16 && j < n) atomicMax(&kb[j], k);
        };
        epi(acc[0], 0);
        epi(acc[1], 1);
        epi(acc[2], 2);
        epi(acc[3], 3);
    }
    __syncthreads();
    if (tid < n) atomicMax(&best[frm[tid]], kb[tid]);
}

// Direction and row power (Algorithm 1 step 4) of the frames that took the
// proposal, one wave per frame.
template <int MAXM>
__global__ __launch_bounds__(256) void k_prop_final(const uint8_t* __restrict__ fell,
                                                    const unsigned long long* __restrict__ best,
                                                    const float2* __restrict__ X, int M, int B,
                                                    const float* __restrict__ tauM, int64_t F,
                                                    int32_t* __restrict__ doa, float* __restrict__ power) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t f = (int64_t)blockIdx.x * 4 + wave;
    if (f >= F || __builtin_amdgcn_readfirstlane(fell[f])) return;
    const unsigned long long k = best[f];
    const int q = __builtin_amdgcn_readfirstlane((int)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull)));
    float t[MAXM];
#pragma unroll
    for (int m = 0; m < MAXM; ++m) t[m] = m < M ? tauM[(int64_t)q * M + m] : 0.f;
    const float acc = power_ds<MAXM>(X + f * M * B, M, B, t, lane);
    if (lane == 0) {
        doa[f] = q;
        power[f] = acc;
    }
}

// Gathers the z of the listed frames to positions 0..count-1 in the GEMM2
// operand layout (FP16, per-frame power-of-two scale) and as FP32 rows.
__global__ __launch_bounds__(256) void k_gather_z(const int* __restrict__ flist, const int* __restrict__ fcount,
                                                  const float* __restrict__ z32, int Rp, float* __restrict__ zg32,
                                                  _Float16* __restrict__ zgfrag, float* __restrict__ zgsc) {
    constexpr int KS = Mf<_Float16>::KSTEP, EPL = Mf<_Float16>::EPL;
    const int64_t pos = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (pos >= *fcount) return;
    const int64_t f = flist[pos];
    float mx = 0.f;
    for (int r = lane; r < Rp; r += 64) {
        const float v = z32[f * Rp + r];
        zg32[pos * Rp + r] = v;
        mx = fmaxf(mx, fabsf(v));
    }
    mx = wave_max(mx);
    float sc = 1.f;
    if (mx > 0.f) {
        int e;
        frexpf(mx, &e);
        sc = ldexpf(1.f, 14 - e);
    }
    if (lane == 0) zgsc[pos] = sc;
    const int64_t fb = pos >> 4;
    const int nn = (int)(pos & 15);
    const int KSn = Rp / KS;
    for (int r = lane; r < Rp; r += 64) {
        const int ks = r / KS, kin = r % KS;
        zgfrag[((fb * KSn + ks) * 64 + nn + 16 * (kin / EPL)) * EPL + kin % EPL] = (_Float16)(zg32[pos * Rp + r] * sc);
    }
}

template <bool AT, bool BT, int EPI>
void mlp_gemm(const _Float16* A, int lda, const _Float16* Bm, int ldb, int M, int N, int K, int ksplit,
              const float* bias, const float* pre32, float* out32, _Float16* out16, int ldo, hipStream_t s) {
    dim3 grid(cdiv(M, GT), cdiv(N, GT), ksplit);
    const int kper = cdiv(K, ksplit);
    const bool vec = !AT && !BT && lda % 8 == 0 && ldb % 8 == 0 && K % 8 == 0 && kper % 8 == 0 && K >= 8 &&
                     M > 0 && N > 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)Bm % 16) == 0;
    if constexpr (!AT && !BT) {
        if (vec) {
            k_mlp_gemm_v<EPI><<<grid, 256, 0, s>>>(A, lda, Bm, ldb, M, N, K, ksplit, bias, pre32, out32, out16, ldo);
            SP_HIP(hipGetLastError());
            return;
        }
    }
    k_mlp_gemm<AT, BT, EPI><<<grid, 256, 0, s>>>(A, lda, Bm, ldb, M, N, K, ksplit, bias, pre32, out32, out16, ldo);
    SP_HIP(hipGetLastError());
}

struct PW {  // workspace carve-up for F frames
    float *zpart, *z32, *zsc, *zn, *a1, *a2, *logits, *loss, *g[6], *pmax, *zg32, *zgsc;
    _Float16 *zfrag, *feat, *h1, *h2, *dlog, *d2, *d1, *zgfrag;
    int32_t *lab, *doa, *flist;
    float* pw;
    // inference: selection, pair lists, rescoring items, best keys
    int32_t *ntop, *cand, *slot, *pairs;
    int *ccount, *cpos, *nitems;
    int4* items;
    unsigned long long* best;
    int64_t Fc, nitem_max;
};

constexpr int WSPLIT = 8;  // split-K partials of the weight gradients

PW carve(svdphat_proposal* pr, int64_t F, hipStream_t s, int topk = 0) {
    svdphat_plan* p = pr->plan;
    const int64_t Fc = round_up64(std::max<int64_t>(F, 1), 64);
    const int H = pr->H, Cp = pr->Cp, D0 = pr->D0, Rp = p->Rp;
    const int ntile = p->ncls_pad / QTILE;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += round_up64((int64_t)b, 256);
        return o;
    };
    const size_t o_zp = take(sizeof(float) * front_zpart_floats(p, F));
    const size_t o_z = take(sizeof(float) * Fc * Rp), o_sc = take(sizeof(float) * Fc), o_zn = take(sizeof(float) * Fc);
    const size_t o_zf = take(sizeof(_Float16) * Fc * Rp), o_ft = take(sizeof(_Float16) * Fc * D0);
    const size_t o_a1 = take(sizeof(float) * Fc * H), o_h1 = take(sizeof(_Float16) * Fc * H);
    const size_t o_a2 = take(sizeof(float) * Fc * H), o_h2 = take(sizeof(_Float16) * Fc * H);
    const size_t o_lg = take(sizeof(float) * Fc * Cp), o_dl = take(sizeof(_Float16) * Fc * Cp);
    const size_t o_d2 = take(sizeof(_Float16) * Fc * H), o_d1 = take(sizeof(_Float16) * Fc * H);
    const size_t o_ls = take(sizeof(float) * Fc), o_lab = take(sizeof(int32_t) * Fc), o_doa = take(sizeof(int32_t) * Fc);
    const size_t o_pw = take(sizeof(float) * Fc), o_fl = take(sizeof(int32_t) * Fc);
    const size_t o_g0 = take(sizeof(float) * WSPLIT * H * D0), o_g1 = take(sizeof(float) * BSPLIT * H);
    const size_t o_g2 = take(sizeof(float) * WSPLIT * H * H), o_g3 = take(sizeof(float) * BSPLIT * H);
    const size_t o_g4 = take(sizeof(float) * WSPLIT * Cp * H), o_g5 = take(sizeof(float) * BSPLIT * Cp);
    const size_t o_pm = take(sizeof(float) * pmax_stride(p) * Fc), o_zg = take(sizeof(float) * Fc * Rp);
    const size_t o_zgf = take(sizeof(_Float16) * Fc * Rp), o_zgs = take(sizeof(float) * Fc);
    const int64_t npair = std::max<int64_t>(1, F * topk), nitem = (npair + PT - 1) / PT + pr->C;
    const size_t o_nt = take(sizeof(int32_t) * Fc), o_cd = take(sizeof(int32_t) * npair);
    const size_t o_sl = take(sizeof(int32_t) * npair), o_pr = take(sizeof(int32_t) * npair);
    const size_t o_cc = take(sizeof(int) * (pr->C + 1)), o_cp = take(sizeof(int) * pr->C);
    const size_t o_it = take(sizeof(int4) * nitem), o_bs = take(sizeof(unsigned long long) * Fc);
    if (pr->ws_bytes < off) {
        // a grown-out buffer is kept until the proposal is destroyed (a graph
        // captured earlier may reference it); no growth during a capture
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        SP_HIP(hipStreamIsCapturing(s, &cs));
        SP_REQUIRE(cs == hipStreamCaptureStatusNone, SVDPHAT_E_INVAL,
                   "the proposal workspace must grow while the stream is being captured");
        const size_t n = std::max(off, pr->ws_bytes + pr->ws_bytes / 2);
        void* nb = nullptr;
        if (dev_malloc(&nb, n) != hipSuccess) {
            (void)hipGetLastError();
            fail(SVDPHAT_E_NOMEM, "proposal workspace of " + std::to_string(n) + " bytes");
        }
        if (pr->ws) pr->ws_retired.push_back(pr->ws);
        pr->ws = nb;
        pr->ws_bytes = n;
    }
    char* w = (char*)pr->ws;
    PW o;
    o.Fc = Fc;
    o.zpart = (float*)(w + o_zp);
    o.z32 = (float*)(w + o_z);
    o.zsc = (float*)(w + o_sc);
    o.zn = (float*)(w + o_zn);
    o.zfrag = (_Float16*)(w + o_zf);
    o.feat = (_Float16*)(w + o_ft);
    o.a1 = (float*)(w + o_a1);
    o.h1 = (_Float16*)(w + o_h1);
    o.a2 = (float*)(w + o_a2);
    o.h2 = (_Float16*)(w + o_h2);
    o.logits = (float*)(w + o_lg);
    o.dlog = (_Float16*)(w + o_dl);
    o.d2 = (_Float16*)(w + o_d2);
    o.d1 = (_Float16*)(w + o_d1);
    o.loss = (float*)(w + o_ls);
    o.lab = (int32_t*)(w + o_lab);
    o.doa = (int32_t*)(w + o_doa);
    o.pw = (float*)(w + o_pw);
    o.flist = (int32_t*)(w + o_fl);
    o.g[0] = (float*)(w + o_g0);
    o.g[1] = (float*)(w + o_g1);
    o.g[2] = (float*)(w + o_g2);
    o.g[3] = (float*)(w + o_g3);
    o.g[4] = (float*)(w + o_g4);
    o.g[5] = (float*)(w + o_g5);
    o.pmax = (float*)(w + o_pm);
    o.zg32 = (float*)(w + o_zg);
    o.zgfrag = (_Float16*)(w + o_zgf);
    o.zgsc = (float*)(w + o_zgs);
    o.ntop = (int32_t*)(w + o_nt);
    o.cand = (int32_t*)(w + o_cd);
    o.slot = (int32_t*)(w + o_sl);
    o.pairs = (int32_t*)(w + o_pr);
    o.ccount = (int*)(w + o_cc);
    o.nitems = o.ccount + pr->C;  // (cleared with the counts; written by the scan)
    o.cpos = (int*)(w + o_cp);
    o.items = (int4*)(w + o_it);
    o.best = (unsigned long long*)(w + o_bs);
    o.nitem_max = nitem;
    return o;
}

// forward pass on features o.feat for F frames -> o.logits
void forward(svdphat_proposal* pr, const PW& o, int64_t F, hipStream_t s) {
    const int H = pr->H, Cp = pr->Cp, D0 = pr->D0;
    mlp_gemm<false, false, EPI_GELU>(o.feat, D0, pr->Wh[0], D0, (int)F, H, D0, 1, pr->P + pr->off[1], nullptr, o.a1,
                                     o.h1, H, s);
    mlp_gemm<false, false, EPI_GELU>(o.h1, H, pr->Wh[1], H, (int)F, H, H, 1, pr->P + pr->off[3], nullptr, o.a2, o.h2,
                                     H, s);
    mlp_gemm<false, false, EPI_BIAS>(o.h2, H, pr->Wh[2], H, (int)F, Cp, H, 1, pr->P + pr->off[5], nullptr, o.logits,
                                     nullptr, Cp, s);
}

// backward pass from o.dlog (summed over frames) -> gradient partials o.g
void backward(svdphat_proposal* pr, const PW& o, int64_t F, hipStream_t s) {
    const int H = pr->H, Cp = pr->Cp, D0 = pr->D0;
    const int ks = std::max(1, std::min(WSPLIT, (int)((F + 255) / 256)));
    auto zero = [&](float* g, size_t n) { zero_async(g, n * sizeof(float), s); };
    // layer 3: dW3[c][h] = sum_f dlog[f][c] h2[f][h]; db3; dh2 = dlog W3, da2 = dh2 GELU'(a2)
    zero(o.g[4], (size_t)WSPLIT * Cp * H);
    mlp_gemm<true, true, EPI_F32>(o.dlog, Cp, o.h2, H, Cp, H, (int)F, ks, nullptr, nullptr, o.g[4], nullptr, H, s);
    const int bp = bias_parts(F);
    k_colsum<<<dim3(cdiv(Cp, 256), bp), 256, 0, s>>>(o.dlog, F, Cp, Cp, o.g[5]);
    mlp_gemm<false, false, EPI_DGELU>(o.dlog, Cp, pr->Wt[2], Cp, (int)F, H, Cp, 1, nullptr, o.a2, nullptr, o.d2, H, s);
    // layer 2
    zero(o.g[2], (size_t)WSPLIT * H * H);
    mlp_gemm<true, true, EPI_F32>(o.d2, H, o.h1, H, H, H, (int)F, ks, nullptr, nullptr, o.g[2], nullptr, H, s);
    k_colsum<<<dim3(cdiv(H, 256), bp), 256, 0, s>>>(o.d2, F, H, H, o.g[3]);
    mlp_gemm<false, false, EPI_DGELU>(o.d2, H, pr->Wt[1], H, (int)F, H, H, 1, nullptr, o.a1, nullptr, o.d1, H, s);
    // layer 1
    zero(o.g[0], (size_t)WSPLIT * H * D0);
    mlp_gemm<true, true, EPI_F32>(o.d1, H, o.feat, D0, H, D0, (int)F, ks, nullptr, nullptr, o.g[0], nullptr, D0, s);
    k_colsum<<<dim3(cdiv(H, 256), bp), 256, 0, s>>>(o.d1, F, H, H, o.g[1]);
    SP_HIP(hipGetLastError());
}

void adam(svdphat_proposal* pr, const PW& o, int64_t F, float lr, hipStream_t s, float inv_f = -1.f) {
    const int H = pr->H, Cp = pr->Cp, D0 = pr->D0;
    pr->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)pr->step), c2 = 1.f - std::pow(b2, (float)pr->step);
    const int ks = std::max(1, std::min(WSPLIT, (int)((F + 255) / 256)));
    const int bp = bias_parts(F);
    AdamSeg seg[6] = {
        {pr->off[0], H, D0, ks, o.g[0], pr->Wh[0], pr->Wt[0], D0, H},
        {pr->off[1], H, 1, bp, o.g[1], nullptr, nullptr, 0, 0},
        {pr->off[2], H, H, ks, o.g[2], pr->Wh[1], pr->Wt[1], H, H},
        {pr->off[3], H, 1, bp, o.g[3], nullptr, nullptr, 0, 0},
        {pr->off[4], Cp, H, ks, o.g[4], pr->Wh[2], pr->Wt[2], H, Cp},
        {pr->off[5], Cp, 1, bp, o.g[5], nullptr, nullptr, 0, 0},
    };
    for (auto& sg : seg) {
        const int64_t n = (int64_t)sg.rows * sg.cols;
        k_adam<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(sg, pr->P, pr->Mm, pr->Vv,
                                                                  inv_f > 0.f ? inv_f : 1.f / (float)F, lr, b1,
                                                                  b2, 1e-8f, c1, c2);
    }
    SP_HIP(hipGetLastError());
}

void cast_weights(svdphat_proposal* pr, hipStream_t s) {
    pr->wf_ok = false;
    const int H = pr->H, Cp = pr->Cp, D0 = pr->D0;
    const int dims[3][2] = {{H, D0}, {H, H}, {Cp, H}};
    const int offs[3] = {0, 2, 4};
    for (int l = 0; l < 3; ++l) {
        const int64_t n = (int64_t)dims[l][0] * dims[l][1];
        k_cast_w<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(pr->P + pr->off[offs[l]], dims[l][0], dims[l][1],
                                                                    pr->Wh[l], dims[l][1], pr->Wt[l], dims[l][0]);
    }
    SP_HIP(hipGetLastError());
}

}  // namespace

void proposal_build(svdphat_proposal* pr, const double* coarse, int C, int H, uint64_t seed) {
    svdphat_plan* p = pr->plan;
    pr->C = C;
    pr->coarse.assign(coarse, coarse + 3 * (size_t)C);
    pr->Cp = round_up(C, 64);
    pr->H = H;
    pr->D = 2 * p->K;
    pr->D0 = p->Rp;
    SP_HIP(hipSetDevice(p->device));
    // cell of every direction: nearest coarse direction (largest cosine; ties
    // within 1e-12 to the lowest cell)
    const int Q = p->Q;
    std::vector<double> cu(3 * (size_t)C);
    for (int c = 0; c < C; ++c) {
        const double* v = coarse + 3 * c;
        const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        SP_REQUIRE(n > 0.0 && std::isfinite(n), SVDPHAT_E_INVAL, "zero or non-finite coarse direction");
        for (int d = 0; d < 3; ++d) cu[3 * c + d] = v[d] / n;
    }
    pr->cell_of_dir.resize(Q);
    std::vector<double> dots(C);
    for (int q = 0; q < Q; ++q) {
        const double* sq = &p->grid[3 * (size_t)q];
        double best = -2.0;
        for (int c = 0; c < C; ++c) {
            dots[c] = sq[0] * cu[3 * c] + sq[1] * cu[3 * c + 1] + sq[2] * cu[3 * c + 2];
            best = std::max(best, dots[c]);
        }
        int bc = 0;
        while (dots[bc] < best - 1e-12) ++bc;
        pr->cell_of_dir[q] = bc;
    }
    int64_t bytes = 0;
    auto up = [&](const void* h, size_t n, void** d) {
        if (dev_malloc(d, std::max<size_t>(n, 4)) != hipSuccess) {
            *d = nullptr;
            fail(SVDPHAT_E_NOMEM, "proposal allocation of " + std::to_string(n) + " bytes");
        }
        if (n) SP_HIP(hipMemcpy(*d, h, n, hipMemcpyHostToDevice));
        bytes += (int64_t)n;
    };
    up(pr->cell_of_dir.data(), sizeof(int32_t) * Q, (void**)&pr->d_cell_of_dir);
    // scored rows grouped by the cell of their direction (CSR)
    std::vector<int32_t> start(C + 1, 0), rowsc(p->ncls);
    for (int r = 0; r < p->ncls; ++r) ++start[pr->cell_of_dir[p->rows[r]] + 1];
    for (int c = 0; c < C; ++c) start[c + 1] += start[c];
    std::vector<int32_t> fillp(start.begin(), start.end() - 1);
    for (int r = 0; r < p->ncls; ++r) rowsc[fillp[pr->cell_of_dir[p->rows[r]]]++] = r;
    up(start.data(), sizeof(int32_t) * (C + 1), (void**)&pr->d_cell_start);
    // FP32 stacked U rows in cell order, row-major [ncls][Rp], and the
    // direction of each
    std::vector<float> ur((size_t)p->ncls * p->Rp, 0.f);
    std::vector<int32_t> dirc(p->ncls);
    const int K = p->K;
    for (int i = 0; i < p->ncls; ++i) {
        const int q = p->rows[rowsc[i]];
        dirc[i] = q;
        for (int k = 0; k < K; ++k) {
            ur[(size_t)i * p->Rp + k] = (float)p->U[((size_t)q * K + k) * 2];
            ur[(size_t)i * p->Rp + K + k] = (float)(-p->U[((size_t)q * K + k) * 2 + 1]);
        }
    }
    up(ur.data(), sizeof(float) * ur.size(), (void**)&pr->d_U32C);
    up(dirc.data(), sizeof(int32_t) * p->ncls, (void**)&pr->d_cell_dir);
    // parameters: W ~ N(0, 2 / fan_in) (real inputs), biases 0; padded
    // input columns and padded cells stay 0
    const int D0 = pr->D0, Cp = pr->Cp, D = pr->D;
    pr->off[0] = 0;
    pr->off[1] = pr->off[0] + (int64_t)H * D0;
    pr->off[2] = pr->off[1] + H;
    pr->off[3] = pr->off[2] + (int64_t)H * H;
    pr->off[4] = pr->off[3] + H;
    pr->off[5] = pr->off[4] + (int64_t)Cp * H;
    pr->nparam = pr->off[5] + Cp;
    std::vector<float> P0(pr->nparam, 0.f);
    std::mt19937_64 g(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int h = 0; h < H; ++h)
        for (int k = 0; k < D; ++k) P0[pr->off[0] + (int64_t)h * D0 + k] = (float)(nd(g) * std::sqrt(2.0 / D));
    for (int h = 0; h < H; ++h)
        for (int k = 0; k < H; ++k) P0[pr->off[2] + (int64_t)h * H + k] = (float)(nd(g) * std::sqrt(2.0 / H));
    for (int c = 0; c < C; ++c)
        for (int k = 0; k < H; ++k) P0[pr->off[4] + (int64_t)c * H + k] = (float)(nd(g) * std::sqrt(1.0 / H));
    // padded cells: large negative bias so that they never win
    for (int c = C; c < Cp; ++c) P0[pr->off[5] + c] = -1e4f;
    up(P0.data(), sizeof(float) * pr->nparam, (void**)&pr->P);
    std::vector<float> zeros(pr->nparam, 0.f);
    up(zeros.data(), sizeof(float) * pr->nparam, (void**)&pr->Mm);
    up(zeros.data(), sizeof(float) * pr->nparam, (void**)&pr->Vv);
    const size_t wsz[3] = {(size_t)H * D0, (size_t)H * H, (size_t)Cp * H};
    for (int l = 0; l < 3; ++l) {
        dev_alloc((void**)&pr->Wh[l], wsz[l] * sizeof(_Float16), "proposal weights");
        dev_alloc((void**)&pr->Wt[l], wsz[l] * sizeof(_Float16), "proposal weights");
        dev_alloc((void**)&pr->Wf[l], wsz[l] * sizeof(_Float16), "proposal weights");
    }
    dev_alloc((void**)&pr->d_count, 8 * sizeof(int), "proposal counters");
    cast_weights(pr, nullptr);
    SP_HIP(hipDeviceSynchronize());
}

float proposal_train_step(svdphat_proposal* pr, const float2* X, int64_t F, float lr, hipStream_t s) {
    svdphat_plan* p = pr->plan;
    pr->wf_ok = false;  // Adam rewrites the f16 weights
    PW o = carve(pr, F, s);
    // labels: the cell of the method's own argmax (FP16, rescored, hi/lo)
    launch_locate(p, X, F, P_FP16, SVDPHAT_RESCORE | SVDPHAT_HILO, o.doa, o.pw, nullptr, nullptr, nullptr, s);
    k_labels<<<dim3((unsigned)((F + 255) / 256)), 256, 0, s>>>(o.doa, pr->d_cell_of_dir, F, o.lab);
    front_fp16(p, X, F, o.zpart, o.z32, o.zfrag, o.zsc, o.zn, s);
    k_features<<<dim3((unsigned)((F * p->Rp + 255) / 256)), 256, 0, s>>>(o.z32, o.zn, F, p->Rp, o.feat);
    forward(pr, o, F, s);
    k_xent<<<dim3((unsigned)((F + 3) / 4)), 256, 0, s>>>(o.logits, pr->Cp, pr->C, o.lab, F, o.dlog, o.loss);
    SP_HIP(hipGetLastError());
    backward(pr, o, F, s);
    adam(pr, o, F, lr, s);
    std::vector<float> loss(F);
    SP_HIP(hipMemcpyAsync(loss.data(), o.loss, sizeof(float) * F, hipMemcpyDeviceToHost, s));
    SP_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (float v : loss) sum += v;
    return (float)(sum / (double)F);
}

void proposal_locate(svdphat_proposal* pr, const float2* X, int64_t F, int topk, float conf_min, int32_t* doa,
                     float* power, uint8_t* fell, hipStream_t s) {
    svdphat_plan* p = pr->plan;
    PW o = carve(pr, F, s, topk);
    const int H = pr->H, D0 = pr->D0, Cp = pr->Cp, C = pr->C, Rp = p->Rp;
    KernelTimer kt(s);
    kt.begin("prop_front");
    front_fp16(p, X, F, o.zpart, o.z32, o.zfrag, o.zsc, o.zn, s);
    kt.end();
    // the forward pass: fused, 32 frames per workgroup (61 us per 20,000
    // frames at hidden 256, against 71 with 64 and 84 with 16: more
    // workgroups in flight hide the weight loads, fewer reuse them less),
    // 16 where 32 frames' activations do not fit; else layer by layer
    kt.begin("prop_mlp");
    const size_t lds_cap = 80 * 1024;
    const int ft = mlp_infer_lds(32, D0, H) <= lds_cap ? 32 : mlp_infer_lds(16, D0, H) <= 2 * lds_cap ? 16 : 0;
    const float* P = pr->P;
    if (ft != 0 && !pr->wf_ok) {
        // the fragment-ordered weights, after a change of the f16 weights
        const int dims[3][2] = {{H, D0}, {H, H}, {Cp, H}};
        for (int l = 0; l < 3; ++l) {
            const int64_t n = (int64_t)dims[l][0] * dims[l][1] / 8;
            k_pack_wf<<<dim3((unsigned)cdiv64(n, 256)), 256, 0, s>>>(pr->Wh[l], dims[l][0], dims[l][1], pr->Wf[l]);
        }
        SP_HIP(hipGetLastError());
        pr->wf_ok = true;
    }
    if (ft == 32)
        k_mlp_infer<32><<<dim3((unsigned)cdiv64(F, 32)), 256, mlp_infer_lds(32, D0, H), s>>>(
            o.z32, o.zn, F, D0, H, Cp, pr->Wf[0], P + pr->off[1], pr->Wf[1], P + pr->off[3], pr->Wf[2],
            P + pr->off[5], o.logits);
    else if (ft == 16)
        k_mlp_infer<16><<<dim3((unsigned)cdiv64(F, 16)), 256, mlp_infer_lds(16, D0, H), s>>>(
            o.z32, o.zn, F, D0, H, Cp, pr->Wf[0], P + pr->off[1], pr->Wf[1], P + pr->off[3], pr->Wf[2],
            P + pr->off[5], o.logits);
    else {
        k_features<<<dim3((unsigned)((F * Rp + 255) / 256)), 256, 0, s>>>(o.z32, o.zn, F, Rp, o.feat);
        forward(pr, o, F, s);
    }
    SP_HIP(hipGetLastError());
    kt.end();
    // selection, pair lists, work items and the full-search list; event
    // counts (instrumentation) in d_count[2..5] as two 64-bit counters:
    // rows rescored, frames that take the proposal
    unsigned long long* stats = counting_on() ? reinterpret_cast<unsigned long long*>(pr->d_count + 2) : nullptr;
    if (stats) zero_async(stats, 2 * sizeof(unsigned long long), s);
    kt.begin("prop_select");
    zero_async(o.ccount, sizeof(int) * (C + 1), s);
    const int64_t nwave = cdiv64(F, SEL_FPW);
    {
        const dim3 gs((unsigned)cdiv64(nwave, 4));
        switch ((C + 63) / 64) {
#define SP_SEL(NJ_)                                                                                                   \
    case NJ_:                                                                                                         \
        k_select<NJ_><<<gs, 256, 0, s>>>(o.logits, Cp, C, topk, conf_min, pr->d_cell_start, F, fell, o.ntop, o.cand, \
                                         o.slot, o.ccount, o.best, stats);                                            \
        break;
            SP_SEL(1) SP_SEL(2) SP_SEL(3) SP_SEL(4) SP_SEL(5) SP_SEL(6) SP_SEL(7) SP_SEL(8)
            SP_SEL(9) SP_SEL(10) SP_SEL(11) SP_SEL(12) SP_SEL(13) SP_SEL(14) SP_SEL(15) SP_SEL(16)
#undef SP_SEL
            default: fail(SVDPHAT_E_INVAL, "more than 1024 cells");
        }
    }
    SP_HIP(hipGetLastError());
    k_cell_scan<<<dim3(1), 1024, 0, s>>>(o.ccount, C, o.cpos, o.items, o.nitems, fell, F, o.flist, pr->d_count);
    SP_HIP(hipGetLastError());
    const int64_t ne = F * topk;
    k_scatter<<<dim3((unsigned)cdiv64(ne, 256)), 256, 0, s>>>(o.ntop, o.cand, o.slot, o.cpos, F, topk, o.pairs);
    SP_HIP(hipGetLastError());
    kt.end();
    // rescoring of each cell's rows against its frames (grid: the most
    // items there can be; the rest exit at once)
    kt.begin("prop_rescore");
    const int KC = std::min(Rp, 128);
    const size_t lds = (size_t)(PT + 64) * (KC + 4) * sizeof(float);
    k_rescore<<<dim3((unsigned)o.nitem_max), 256, lds, s>>>(o.items, o.nitems, o.pairs, o.z32, Rp, KC, pr->d_U32C,
                                                            pr->d_cell_start, pr->d_cell_dir, o.best);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("prop_power");
    const dim3 gf((unsigned)cdiv64(F, 4));
    if (p->M <= 8)
        k_prop_final<8><<<gf, 256, 0, s>>>(fell, o.best, X, p->M, p->B, p->d_tauM_all, F, doa, power);
    else
        k_prop_final<16><<<gf, 256, 0, s>>>(fell, o.best, X, p->M, p->B, p->d_tauM_all, F, doa, power);
    SP_HIP(hipGetLastError());
    kt.end();
    // low-confidence frames: the full search on the listed frames only
    kt.begin("prop_fallback");
    k_gather_z<<<dim3((unsigned)(o.Fc / 4)), 256, 0, s>>>(o.flist, pr->d_count, o.z32, Rp, o.zg32, o.zgfrag,
                                                          o.zgsc);
    SP_HIP(hipGetLastError());
    back_list_fp16(p, X, F, o.flist, pr->d_count, o.zgfrag, o.zgsc, o.zg32, o.zn, o.pmax, doa, power, nullptr, s);
    kt.end();
    kt.flush();
    if (stats) {
        unsigned long long h[2] = {0, 0};
        int fc = 0;
        SP_HIP(hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, s));
        SP_HIP(hipMemcpyAsync(&fc, pr->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
        SP_HIP(hipStreamSynchronize(s));
        // rows rescored per frame that took the proposal; frames that fell back
        timing_count("count:proposal_rows_rescored", (double)h[0], (int64_t)h[1]);
        timing_count("count:proposal_fell_back", (double)fc, F);
    }
}

// host parameters in the layout W1 [H][D], b1 [H], W2 [H][H], b2 [H],
// W3 [C][H], b3 [C] (no padding)
int64_t proposal_nparams(const svdphat_proposal* pr) {
    const int64_t H = pr->H, D = pr->D, C = pr->C;
    return H * D + H + H * H + H + C * H + C;
}

// one flat device array (parameters or an Adam moment) to or from the host
// layout W1 [H][D], b1 [H], W2 [H][H], b2 [H], W3 [C][H], b3 [C]
static void proposal_xfer(svdphat_proposal* pr, float* dev, float* host, bool set) {
    const int H = pr->H, D = pr->D, D0 = pr->D0, C = pr->C;
    std::vector<float> P(pr->nparam);
    SP_HIP(hipMemcpy(P.data(), dev, sizeof(float) * pr->nparam, hipMemcpyDeviceToHost));
    int64_t h = 0;
    auto xfer = [&](int64_t dst, int rows, int cols, int ld) {
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c, ++h) {
                if (set) P[dst + (int64_t)r * ld + c] = host[h];
                else host[h] = P[dst + (int64_t)r * ld + c];
            }
    };
    xfer(pr->off[0], H, D, D0);
    xfer(pr->off[1], 1, H, H);
    xfer(pr->off[2], H, H, H);
    xfer(pr->off[3], 1, H, H);
    xfer(pr->off[4], C, H, H);
    xfer(pr->off[5], 1, C, C);
    if (set) SP_HIP(hipMemcpy(dev, P.data(), sizeof(float) * pr->nparam, hipMemcpyHostToDevice));
}

void proposal_params(svdphat_proposal* pr, float* host, bool set) {
    proposal_xfer(pr, pr->P, host, set);
    if (set) {
        cast_weights(pr, nullptr);
        SP_HIP(hipDeviceSynchronize());
    }
}

void proposal_state(svdphat_proposal* pr, float* params, float* m, float* v, int64_t* step, bool set) {
    proposal_xfer(pr, pr->Mm, m, set);
    proposal_xfer(pr, pr->Vv, v, set);
    proposal_params(pr, params, set);
    if (set) pr->step = *step;
    else *step = pr->step;
}

// gradient of the mean cross-entropy for host features [F][D] and labels,
// in the host parameter layout (testing aid)
float proposal_grad(svdphat_proposal* pr, const float* feat, const int32_t* lab, int64_t F, float* grad) {
    const int H = pr->H, D = pr->D, D0 = pr->D0, C = pr->C, Cp = pr->Cp;
    hipStream_t s = nullptr;
    PW o = carve(pr, F, s);
    std::vector<_Float16> fh((size_t)F * D0, (_Float16)0.f);
    for (int64_t f = 0; f < F; ++f)
        for (int k = 0; k < D; ++k) fh[(size_t)f * D0 + k] = (_Float16)feat[(size_t)f * D + k];
    SP_HIP(hipMemcpy(o.feat, fh.data(), sizeof(_Float16) * fh.size(), hipMemcpyHostToDevice));
    SP_HIP(hipMemcpy(o.lab, lab, sizeof(int32_t) * F, hipMemcpyHostToDevice));
    forward(pr, o, F, s);
    k_xent<<<dim3((unsigned)((F + 3) / 4)), 256, 0, s>>>(o.logits, Cp, C, o.lab, F, o.dlog, o.loss);
    backward(pr, o, F, s);
    SP_HIP(hipDeviceSynchronize());
    const int ks = std::max(1, std::min(WSPLIT, (int)((F + 255) / 256)));
    // partials are [parts][prow][ld]; the first rows x cols are returned
    auto fetch = [&](const float* g, int rows, int cols, int prow, int ld, int parts, int64_t& h) {
        std::vector<float> t((size_t)parts * prow * ld);
        SP_HIP(hipMemcpy(t.data(), g, sizeof(float) * t.size(), hipMemcpyDeviceToHost));
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c, ++h) {
                double v = 0.0;
                for (int q = 0; q < parts; ++q) v += t[(size_t)q * prow * ld + (size_t)r * ld + c];
                grad[h] = (float)(v / (double)F);
            }
    };
    int64_t h = 0;
    fetch(o.g[0], H, D, H, D0, ks, h);
    const int bp = bias_parts(F);
    fetch(o.g[1], 1, H, 1, H, bp, h);
    fetch(o.g[2], H, H, H, H, ks, h);
    fetch(o.g[3], 1, H, 1, H, bp, h);
    fetch(o.g[4], C, H, Cp, H, ks, h);
    fetch(o.g[5], 1, C, 1, Cp, bp, h);
    std::vector<float> loss(F);
    SP_HIP(hipMemcpy(loss.data(), o.loss, sizeof(float) * F, hipMemcpyDeviceToHost));
    double sum = 0.0;
    for (float v : loss) sum += v;
    return (float)(sum / (double)F);
}

// network input of F frames as FP32 [F][2K] (testing aid)
void proposal_features(svdphat_proposal* pr, const float2* X, int64_t F, float* feat, hipStream_t s) {
    svdphat_plan* p = pr->plan;
    PW o = carve(pr, F, s);
    front_fp16(p, X, F, o.zpart, o.z32, o.zfrag, o.zsc, o.zn, s);
    k_features<<<dim3((unsigned)((F * p->Rp + 255) / 256)), 256, 0, s>>>(o.z32, o.zn, F, p->Rp, o.feat);
    k_widen<<<dim3((unsigned)((F * pr->D + 255) / 256)), 256, 0, s>>>(o.feat, F, pr->D, pr->D0, feat);
    SP_HIP(hipGetLastError());
    SP_HIP(hipStreamSynchronize(s));
}

// one Adam step with a given mean gradient in the host parameter layout
// (testing aid; the same update kernel as the training step)
void proposal_apply_grad(svdphat_proposal* pr, const float* grad, float lr) {
    const int H = pr->H, D = pr->D, D0 = pr->D0, C = pr->C, Cp = pr->Cp;
    hipStream_t s = nullptr;
    PW o = carve(pr, 1, s);
    int64_t h = 0;
    auto put = [&](float* g, int rows, int cols, int prow, int ld) {
        std::vector<float> t((size_t)prow * ld, 0.f);
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c, ++h) t[(size_t)r * ld + c] = grad[h];
        SP_HIP(hipMemcpy(g, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice));
    };
    put(o.g[0], H, D, H, D0);
    put(o.g[1], 1, H, 1, H);
    put(o.g[2], H, H, H, H);
    put(o.g[3], 1, H, 1, H);
    put(o.g[4], C, H, Cp, H);
    put(o.g[5], 1, C, 1, Cp);
    adam(pr, o, 1, lr, s, 1.f);
    SP_HIP(hipDeviceSynchronize());
}

void proposal_free(svdphat_proposal* pr) {
    if (!pr) return;
    void* bufs[] = {pr->d_cell_of_dir, pr->d_cell_start, pr->d_cell_dir, pr->d_U32C, pr->P, pr->Mm, pr->Vv,
                    pr->ws, pr->d_count, pr->Wh[0], pr->Wh[1], pr->Wh[2], pr->Wt[0], pr->Wt[1], pr->Wt[2],
                    pr->Wf[0], pr->Wf[1], pr->Wf[2]};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (void* b : pr->ws_retired) (void)hipFree(b);
    (void)hipGetLastError();  // no error of the teardown outlives it
    delete pr;
}

}  // namespace svdphat
