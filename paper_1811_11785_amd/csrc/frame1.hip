// Single frames and small batches (at most GV_MAX_FRAMES frames per call) in
// GEMV form: Algorithm 1 online steps 1-4 (Section 3) for one frame at a
// time, as a streaming caller issues them.  With a handful of frames the
// projections are matrix-vector products bound by reading their operands
// (A = S V^H and U, a few MB that stay in the L2 caches and the Infinity
// Cache between calls) and by latency, not by arithmetic, so they run in FP32
// whatever precision the batched path would use, and the argmax of eq. (14)
// is exact in FP32 over every scored row without a rescoring pass.
//
//   k_gv_z      PHAT (eqs. (3), (7)) of a slice of bins and its share of
//               Z = S V^H X (eq. (12)): grid (bin slices, frames).
//   k_gv_zsum   Z: the slices' partial sums added in slice order.
//   k_gv_score  Y = Re{U Z} (eqs. (13)-(14)) over 64-row tiles in FP32 with
//               the best and second-best class of each tile.
//   k_gv_final  per frame: the best class, the margin and the row power of
//               Algorithm 1 online step 4 of the chosen direction.
//
// Four short kernels: fewer, with a "last workgroup to finish" step, were
// slower (on this GPU a device-scope fence writes back or invalidates the
// whole L2 of the XCD, and one per workgroup cost more than the kernel
// boundaries it saves), and so was adding the partial sums in every scoring
// workgroup (all of them reading the same lines).
#include "device.h"

namespace svdphat {
namespace {

constexpr int GV_BINS = 2;      // bins per workgroup slice of k_gv_z
constexpr int GV_MAXP = 120;    // pairs (16 microphones)
// NR stacked rows per lane (Rp <= 64 NR), instantiated for NR = 2, 4, 8, 16

// Top-2 classes: best (value, class) and the best value of any other class.
struct Top2 {
    float v1;
    int c1;
    float v2;
};

__device__ __forceinline__ void top2_add(Top2& t, float v, int c) {
    if (!(v == v)) return;                       // NaN never counts
    if (better(v, c, t.v1, t.c1)) {
        if (c != t.c1) t.v2 = t.v1;
        t.v1 = v;
        t.c1 = c;
    } else if (c != t.c1 && v > t.v2) {
        t.v2 = v;
    }
}

__device__ __forceinline__ Top2 top2_merge(const Top2& a, const Top2& b) {
    // branch-free: selects by bit masks (blend), so nothing is addressed
    const bool bw = better(b.v1, b.c1, a.v1, a.c1);
    const float lose1 = __uint_as_float(blend(__float_as_uint(b.v1), __float_as_uint(a.v1), bw));
    const int losec = (int)blend((uint32_t)b.c1, (uint32_t)a.c1, bw);
    const float lose2 = __uint_as_float(blend(__float_as_uint(b.v2), __float_as_uint(a.v2), bw));
    const float win2 = __uint_as_float(blend(__float_as_uint(a.v2), __float_as_uint(b.v2), bw));
    Top2 r;
    r.v1 = __uint_as_float(blend(__float_as_uint(a.v1), __float_as_uint(b.v1), bw));
    r.c1 = (int)blend((uint32_t)a.c1, (uint32_t)b.c1, bw);
    r.v2 = fmaxf(win2, losec != r.c1 ? lose1 : lose2);
    return r;
}

__device__ __forceinline__ Top2 wave_top2(Top2 t) {
    uint32_t w[3] = {__float_as_uint(t.v1), (uint32_t)t.c1, __float_as_uint(t.v2)};
    wave_reduce(w, [](uint32_t (&x)[3], const uint32_t (&o)[3]) {
        const Top2 a{__uint_as_float(x[0]), (int)x[1], __uint_as_float(x[2])};
        const Top2 b{__uint_as_float(o[0]), (int)o[1], __uint_as_float(o[2])};
        const Top2 m = top2_merge(a, b);
        x[0] = __float_as_uint(m.v1);
        x[1] = (uint32_t)m.c1;
        x[2] = __float_as_uint(m.v2);
    });
    return Top2{__uint_as_float(w[0]), (int)w[1], __uint_as_float(w[2])};
}

// PHAT of GV_BINS bins of frame blockIdx.y and their share of Z:
// zpart[(f * nsl + slice) * Rp + r] = sum over the slice's stacked columns c
// of A32T[c][r] x_c, with x_c = Re / Im (X~_i[b] X~_j[b]^*) for column
// c = (b P + p) 2 + ri.  Eight waves take every eighth column, a wave's
// loads of up to 24 columns issued together (one round at seven
// microphones); a lane holds rows lane + 64 j.
template <int NR>
__global__ __launch_bounds__(512) void k_gv_z(const float2* __restrict__ X, int M, int P, int B,
                                              const int8_t* __restrict__ pi, const int8_t* __restrict__ pj,
                                              const float* __restrict__ A32T, int Rp, int nsl,
                                              float* __restrict__ zpart) {
    __shared__ float2 xs[16 * GV_BINS];                 // [m][bin of slice] unit spectra
    __shared__ float xc[GV_BINS * GV_MAXP * 2];          // stacked PHAT columns of the slice
    __shared__ float red[8][NR * 64];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int f = blockIdx.y, sl = blockIdx.x;
    const int b0 = sl * GV_BINS;
    const int nb = min(GV_BINS, B - b0);
    const float2* xf = X + (int64_t)f * M * B;
    const int ncol = nb * P * 2;
    const float* Ab = A32T + (int64_t)b0 * P * 2 * Rp;
    constexpr int U = NR <= 4 ? 24 : 48 / NR;   // columns of a wave per round
    float a[U][NR];
    auto load_round = [&](int c0) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int c = c0 + 8 * u;
                a[u][j] = c < ncol && lane + 64 * j < Rp ? Ab[(int64_t)c * Rp + lane + 64 * j] : 0.f;
            }
    };
    // the first round of A (which does not depend on the frame) is in flight
    // while the spectra are loaded and the PHAT columns formed
    load_round(wave);
    if (t < M * GV_BINS) {
        const int m = t / GV_BINS, bl = t % GV_BINS;
        float2 v = bl < nb ? xf[(int64_t)m * B + b0 + bl] : make_float2(0.f, 0.f);
        unit(v.x, v.y);
        xs[m * GV_BINS + bl] = v;
    }
    __syncthreads();
    for (int c = t; c < ncol; c += 512) {
        const int bl = c / (2 * P), rem = c % (2 * P), pp = rem >> 1, ri = rem & 1;
        const float2 pa = xs[pi[pp] * GV_BINS + bl], pb = xs[pj[pp] * GV_BINS + bl];
        // X~_i conj(X~_j)
        xc[c] = ri == 0 ? fmaf(pa.x, pb.x, pa.y * pb.y) : fmaf(pa.y, pb.x, -pa.x * pb.y);
    }
    __syncthreads();
    float acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = 0.f;
    for (int c0 = wave; c0 < ncol; c0 += 8 * U) {
        if (c0 != wave) load_round(c0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + 8 * u;
            const float x = c < ncol ? xc[c] : 0.f;
#pragma unroll
            for (int j = 0; j < NR; ++j) acc[j] = fmaf(a[u][j], x, acc[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) red[wave][lane + 64 * j] = acc[j];
    __syncthreads();
    float* zp = zpart + (int64_t)f * nsl * Rp;
    for (int r = t; r < Rp; r += 512)
        zp[(int64_t)sl * Rp + r] = ((red[0][r] + red[1][r]) + (red[2][r] + red[3][r])) +
                                   ((red[4][r] + red[5][r]) + (red[6][r] + red[7][r]));
}

// Z of frame blockIdx.x: the sum of its nsl slice partials (threads take
// four consecutive rows and every G-th slice, all loads issued together;
// then the G groups' sums are added in group order).
template <int NR>
__global__ __launch_bounds__(512) void k_gv_zsum(const float* __restrict__ zpart, int Rp, int nsl,
                                                 float* __restrict__ z) {
    __shared__ float4 part[512];
    const int t = threadIdx.x, f = blockIdx.x;
    const int R4 = Rp / 4;
    const float4* zp4 = reinterpret_cast<const float4*>(zpart + (int64_t)f * nsl * Rp);
    for (int r0 = 0; r0 < R4; r0 += 512) {
        const int nr4 = min(512, R4 - r0), G = 512 / nr4;
        const int r = t % nr4, g = t / nr4;
        if (g < G) {
            float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
            int q = g;
            for (; q + 15 * G < nsl; q += 16 * G) {
                float4 v[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) v[i] = zp4[(int64_t)(q + i * G) * R4 + r0 + r];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    sum.x += v[i].x;
                    sum.y += v[i].y;
                    sum.z += v[i].z;
                    sum.w += v[i].w;
                }
            }
            for (; q < nsl; q += G) {
                const float4 v = zp4[(int64_t)q * R4 + r0 + r];
                sum.x += v.x;
                sum.y += v.y;
                sum.z += v.z;
                sum.w += v.w;
            }
            part[g * nr4 + r] = sum;
        }
        __syncthreads();
        if (t < nr4) {
            float4 zz = make_float4(0.f, 0.f, 0.f, 0.f);
            for (int k = 0; k < G; ++k) {
                const float4 v = part[k * nr4 + t];
                zz.x += v.x;
                zz.y += v.y;
                zz.z += v.z;
                zz.w += v.w;
            }
            reinterpret_cast<float4*>(z)[(int64_t)f * R4 + r0 + t] = zz;
        }
        __syncthreads();
    }
}

// Y = U Z over the scored rows in FP32 for frame blockIdx.y: workgroup t
// scores the 64 rows of tile t of the transposed FP32 rows (lane = row, four
// consecutive k per 16-byte piece, the four waves a quarter of k each) and
// the tile's best two classes go to res[f][t].
template <int NR>
__global__ __launch_bounds__(256) void k_gv_score(const float* __restrict__ z, int Rp,
                                                  const float* __restrict__ U32T, int ncls,
                                                  const int32_t* __restrict__ rowcls, float4* __restrict__ res) {
    __shared__ __align__(16) float zs[NR * 64];
    __shared__ float red[4][64];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int f = blockIdx.y, ng = gridDim.x;
    for (int r = t; r < Rp; r += 256) zs[r] = z[(int64_t)f * Rp + r];
    __syncthreads();
    const int tile = blockIdx.x, K4 = Rp / 4, kq = K4 / 4;
    const float4* u = reinterpret_cast<const float4*>(U32T) + ((int64_t)tile * K4 + wave * kq) * 64 + lane;
    const float* zw = zs + 4 * wave * kq;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int k0 = 0; k0 < kq; k0 += 16) {
        float4 pc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) pc[i] = k0 + i < kq ? u[(int64_t)(k0 + i) * 64] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (k0 + i < kq) {
                const float4 zz = *reinterpret_cast<const float4*>(zw + 4 * (k0 + i));
                a0 = fmaf(pc[i].x, zz.x, a0);
                a1 = fmaf(pc[i].y, zz.y, a1);
                a2 = fmaf(pc[i].z, zz.z, a2);
                a3 = fmaf(pc[i].w, zz.w, a3);
            }
    }
    red[wave][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (wave == 0) {
        const float y = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        const int row = tile * QTILE + lane;
        Top2 best{-INFINITY, 0x7fffffff, -INFINITY};
        if (row < ncls) top2_add(best, y, rowcls[row]);
        best = wave_top2(best);
        if (lane == 0) res[(int64_t)f * ng + tile] = make_float4(best.v1, __int_as_float(best.c1), best.v2, 0.f);
    }
}

// One wave per frame: the best class over the tiles (its lowest index is the
// class id), the margin (y1 - y2) / |y1| to the best other class, the reduced
// power y1 and the row power of Algorithm 1 online step 4 of the chosen
// direction.
template <int MAXM>
__global__ __launch_bounds__(64) void k_gv_final(const float4* __restrict__ res, int ng, const float2* __restrict__ X,
                                                 int M, int B, const float* __restrict__ tauM,
                                                 const int32_t* __restrict__ rows, int32_t* __restrict__ doa,
                                                 float* __restrict__ power, float* __restrict__ yhat,
                                                 float* __restrict__ margin) {
    const int lane = threadIdx.x, f = blockIdx.x;
    Top2 w{-INFINITY, 0x7fffffff, -INFINITY};
    for (int g = lane; g < ng; g += 64) {
        const float4 r = res[(int64_t)f * ng + g];
        w = top2_merge(w, Top2{r.x, __float_as_int(r.y), r.z});
    }
    w = wave_top2(w);
    // a frame whose every power is NaN (non-finite input) keeps a valid index
    const int q = w.c1 == 0x7fffffff ? rows[0] : w.c1;
    float tq[MAXM];
#pragma unroll
    for (int m = 0; m < MAXM; ++m) tq[m] = m < M ? tauM[(int64_t)q * M + m] : 0.f;
    const float pw = power_ds<MAXM>(X + (int64_t)f * M * B, M, B, tq, lane);
    if (lane == 0) {
        doa[f] = q;
        power[f] = pw;
        if (yhat) yhat[f] = w.v1;
        if (margin) margin[f] = (w.v1 - w.v2) / fmaxf(fabsf(w.v1), 1e-30f);
    }
}

}  // namespace

bool gv_applicable(const svdphat_plan* p, int64_t F) {
    return F >= 1 && F <= GV_MAX_FRAMES && p->A32T != nullptr && p->Rp <= 1024 && p->P <= GV_MAXP && p->M <= 16;
}

int gv_score_groups(const svdphat_plan* p) { return p->ncls_pad / QTILE; }

size_t gv_scratch_bytes(const svdphat_plan* p, int64_t F) {
    const int nsl = cdiv(p->B, GV_BINS);
    const int ng = gv_score_groups(p);
    return (size_t)round_up64((int64_t)F * nsl * p->Rp * 4, 256) + (size_t)round_up64((int64_t)F * p->Rp * 4, 256) +
           (size_t)F * ng * 16;
}

void launch_gv(svdphat_plan* p, const ScoreRows& sr, const float2* X, int64_t F, int32_t* doa, float* power,
               float* yhat, float* margin, void* ws, hipStream_t s) {
    const int nsl = cdiv(p->B, GV_BINS);
    const int ng = gv_score_groups(p);
    char* w = (char*)ws;
    float* zpart = (float*)w;
    w += round_up64((int64_t)F * nsl * p->Rp * 4, 256);
    float* z = (float*)w;
    w += round_up64((int64_t)F * p->Rp * 4, 256);
    float4* res = (float4*)w;
    const int nr = cdiv(p->Rp, 64);
    const int NRc = nr <= 2 ? 2 : (nr <= 4 ? 4 : (nr <= 8 ? 8 : 16));
    KernelTimer kt(s);
    kt.begin("gv_z");
    const dim3 gz((unsigned)nsl, (unsigned)F), gs((unsigned)ng, (unsigned)F);
#define SP_GV(KER, GRID, BLK, ...)                                                                                   \
    switch (NRc) {                                                                                                   \
        case 2: KER<2><<<GRID, BLK, 0, s>>>(__VA_ARGS__); break;                                                     \
        case 4: KER<4><<<GRID, BLK, 0, s>>>(__VA_ARGS__); break;                                                     \
        case 8: KER<8><<<GRID, BLK, 0, s>>>(__VA_ARGS__); break;                                                     \
        default: KER<16><<<GRID, BLK, 0, s>>>(__VA_ARGS__); break;                                                   \
    }
    SP_GV(k_gv_z, gz, 512, X, p->M, p->P, p->B, p->d_pi, p->d_pj, p->A32T, p->Rp, nsl, zpart)
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("gv_zsum");
    SP_GV(k_gv_zsum, dim3((unsigned)F), 512, zpart, p->Rp, nsl, z)
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("gv_score");
    SP_GV(k_gv_score, gs, 256, z, p->Rp, sr.U32T, p->ncls, p->d_rowcls, res)
#undef SP_GV
    SP_HIP(hipGetLastError());
    kt.end();
    kt.begin("gv_final");
    if (p->M <= 8)
        k_gv_final<8><<<dim3((unsigned)F), 64, 0, s>>>(res, ng, X, p->M, p->B, p->d_tauM_all, p->d_rows, doa, power,
                                                       yhat, margin);
    else
        k_gv_final<16><<<dim3((unsigned)F), 64, 0, s>>>(res, ng, X, p->M, p->B, p->d_tauM_all, p->d_rows, doa,
                                                        power, yhat, margin);
    SP_HIP(hipGetLastError());
    kt.end();
    kt.flush();
}

}  // namespace svdphat
