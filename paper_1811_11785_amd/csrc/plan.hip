// Offline plan of SVD-PHAT (Algorithm 1, offline steps 1-2, Section 3):
// far-field delays (eq. (2)), the steering matrix W (eqs. (4), (8)) built in
// FP64 on the GPU, its truncated SVD (eq. (10)) through the Hermitian
// eigendecomposition of the smaller Gram matrix (rocBLAS zherk + rocSOLVER
// zheevd, FP64), the rank rule of eq. (11), direction classes, and packing
// of the device operands of the online kernels.
#include "internal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace svdphat {

namespace {

struct RB {
    rocblas_handle h = nullptr;
    ~RB() {
        if (h) rocblas_destroy_handle(h);
    }
};

void rb_check(rocblas_status s, const char* what) {
    if (s != rocblas_status_success)
        fail(SVDPHAT_E_DEVICE, std::string(what) + ": rocBLAS/rocSOLVER status " + std::to_string((int)s));
}

template <typename P>
struct DevBuf {
    P* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    void alloc(size_t n) {
        if (dev_malloc((void**)&p, n * sizeof(P)) != hipSuccess) {
            p = nullptr;
            fail(SVDPHAT_E_NOMEM, "device allocation of " + std::to_string(n * sizeof(P)) + " bytes failed");
        }
    }
};

// W[q + c Q] = exp(2 pi i bin tau[q][p] / N), column c = bin * P + p
// (bin-major; the SVD is invariant to the column order, which only permutes
// the rows of V).  Column-major Q x L for rocBLAS.  The phase is reduced to
// [-1/2, 1/2] revolutions in FP64 before the sine and cosine.
__global__ void k_build_w64(const double* __restrict__ tau, int Q, int P, int N, int64_t total,
                            rocblas_double_complex* __restrict__ W) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int q = (int)(idx % Q);
    int64_t c = idx / Q;
    int bin = (int)(c / P), p = (int)(c % P);
    double t = (double)bin * tau[(int64_t)q * P + p] / (double)N;
    t -= rint(t);
    double s, co;
    sincospi(2.0 * t, &s, &co);
    W[idx] = rocblas_double_complex(co, s);
}

template <typename T>
T to_t(float v);
template <>
float to_t<float>(float v) { return v; }
template <>
_Float16 to_t<_Float16>(float v) { return (_Float16)v; }
template <>
__bf16 to_t<__bf16>(float v) { return (__bf16)v; }
template <typename T>
float from_t(T v) { return (float)v; }

// Chunk layout of the GEMM1 reduction axis for one element type.  The x
// tile of 64 frames x CW values must fit its LDS budget; among the bin
// counts that fit, prefer little padding, then bigger chunks.
G1Layout make_layout(int P, int B, int M, int esize, int kstep, int nRB, int epl) {
    G1Layout g;
    int cws = 0, bbs = 0;
    if (esize == 2 && B >= 2 && g1s_layout(M, nRB, kstep, &cws, &bbs)) {
        // the chunk of the streamed GEMM1 kernel
        g.CW = cws;
        g.BB = bbs;
        g.nch = cdiv(B, g.BB);
        g.ks_chunk = g.CW / kstep;
        g.elems = (int64_t)g.nch * g.ks_chunk * nRB * 64 * epl;
        return g;
    }
    // CW + pad per frame row: 64 KB of x tile, or 124 KB above 8
    // microphones (120 pairs per bin at 16: two bins per chunk would leave
    // half of the workgroup's threads idle while the tile is formed)
    const int budget = (M <= 8 ? 65536 : 126976) / (64 * esize) - 8;
    const int max_bb = (M <= 8 ? G1_MAX_ITEMS8 : G1_MAX_ITEMS16) / 64;
    double best = -1.0;
    for (int bb = 1; bb <= std::min(B, max_bb); ++bb) {
        const int cw = round_up(bb * 2 * P, kstep);
        if (cw > budget) break;
        const int ks = cw / kstep;
        const int nch = cdiv(B, bb);
        // useful fraction of the chunk, of the last chunk, of the four waves'
        // round-robin k-steps, and a per-chunk overhead of about one k-step
        const double eff = (double)(bb * 2 * P) / cw * (double)B / (nch * bb) * (double)ks / (4 * cdiv(ks, 4)) *
                           (double)ks / (ks + 4);
        if (eff > best) {
            best = eff;
            g.BB = bb;
            g.CW = cw;
        }
    }
    if (g.BB == 0) fail(SVDPHAT_E_UNSUPPORTED, "too many microphone pairs for the GEMM1 tile");
    g.nch = cdiv(B, g.BB);
    g.ks_chunk = g.CW / kstep;
    g.elems = (int64_t)g.nch * g.ks_chunk * nRB * 64 * epl;
    return g;
}

}  // namespace

// Pack the stacked-real A = S_K V_K^H (rows: Re z_0..Re z_{K-1}, Im z_0..,
// padding) into MFMA A-operand fragments: for chunk ch, k-step ks, row
// block rb and lane l, the EPL elements A[rb*16 + l%16][ks*KSTEP +
// EPL*(l/16) + e] of that chunk's columns.  Column (b, p, ri) of a chunk is
// (b * P + p) * 2 + ri, bin = ch * BB + b.
// (rb0, nrb: only row blocks [rb0, rb0 + nrb), packed as blocks 0 .. nrb-1;
// nrb = 0: all)
template <typename T>
static void pack_A(const svdphat_plan* p, const G1Layout& g, std::vector<T>& hi, std::vector<T>& lo,
                   bool want_lo, int rb0 = 0, int nrb = 0) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL;
    const int K = p->K, P = p->P;
    const int nRB = nrb > 0 ? nrb : p->Rp / 16;
    const int64_t elems = (int64_t)g.nch * g.ks_chunk * nRB * 64 * EPL;
    hi.assign(elems, to_t<T>(0.f));
    if (want_lo) lo.assign(elems, to_t<T>(0.f));
    for (int ch = 0; ch < g.nch; ++ch)
        for (int ks = 0; ks < g.ks_chunk; ++ks)
            for (int rbl = 0; rbl < nRB; ++rbl)
                for (int l = 0; l < 64; ++l)
                    for (int e = 0; e < EPL; ++e) {
                        const int rb = rb0 + rbl;
                        int r = rb * 16 + l % 16;
                        int col = ks * KS + EPL * (l / 16) + e;
                        int b = col / (2 * P), rem = col % (2 * P);
                        int pp = rem / 2, ri = rem % 2;
                        int bin = ch * g.BB + b;
                        double v = 0.0;
                        if (r < 2 * K && b < g.BB && bin < p->B) {
                            int kk = r < K ? r : r - K;
                            int64_t c = (int64_t)bin * P + pp;  // internal row of V
                            double vr = p->V[(c * K + kk) * 2], vi = p->V[(c * K + kk) * 2 + 1];
                            double s = p->sigma[kk];
                            // A_c = s conj(v): re = s vr, im = -s vi
                            double ar = s * vr, ai = -s * vi;
                            if (r < K) v = ri == 0 ? ar : -ai;
                            else v = ri == 0 ? ai : ar;
                        }
                        int64_t off = ((((int64_t)ch * g.ks_chunk + ks) * nRB + rbl) * 64 + l) * EPL + e;
                        float vf = (float)v;
                        T h = to_t<T>(vf);
                        hi[off] = h;
                        if (want_lo) lo[off] = to_t<T>((float)(v - (double)from_t<T>(h)));
                    }
}

// Stacked U rows of the scored directions: [Re U_q, -Im U_q, 0-padding],
// scaled by `scale`, in MFMA A-operand fragments [rb][ks][lane][EPL].
template <typename T>
static void pack_U(const svdphat_plan* p, const std::vector<float>& Ust, float scale, std::vector<T>& out) {
    constexpr int KS = Mf<T>::KSTEP, EPL = Mf<T>::EPL;
    const int Rp = p->Rp, nRB = p->ncls_pad / 16, KSn = Rp / KS;
    out.assign((size_t)nRB * KSn * 64 * EPL, to_t<T>(0.f));
    for (int rb = 0; rb < nRB; ++rb)
        for (int ks = 0; ks < KSn; ++ks)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < EPL; ++e) {
                    int row = rb * 16 + l % 16;
                    int k = ks * KS + EPL * (l / 16) + e;
                    float v = row < p->ncls ? Ust[(size_t)row * Rp + k] * scale : 0.f;
                    out[(((size_t)rb * KSn + ks) * 64 + l) * EPL + e] = to_t<T>(v);
                }
}

template <typename T>
static void upload(const std::vector<T>& h, void** d, int64_t& bytes) {
    size_t n = h.size() * sizeof(T);
    if (dev_malloc(d, n) != hipSuccess) {
        *d = nullptr;
        fail(SVDPHAT_E_NOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    SP_HIP(hipMemcpy(*d, h.data(), n, hipMemcpyHostToDevice));
    bytes += (int64_t)n;
}

// Direction classes: rep[q] = lowest index whose delay row equals row q
// within tol samples in every pair.  Sort by the first pair's delay and
// compare only neighbours within tol in that coordinate.
static void direction_classes(const std::vector<double>& tau, int Q, int P, double tol,
                              std::vector<int32_t>& rep) {
    std::vector<int32_t> idx(Q);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return tau[(size_t)a * P] < tau[(size_t)b * P]; });
    rep.resize(Q);
    std::iota(rep.begin(), rep.end(), 0);
    for (int a = 0; a < Q; ++a) {
        const int qa = idx[a];
        const double* ta = &tau[(size_t)qa * P];
        for (int b = a + 1; b < Q; ++b) {
            const int qb = idx[b];
            const double* tb = &tau[(size_t)qb * P];
            if (tb[0] - ta[0] > tol) break;
            bool same = true;
            for (int k = 0; k < P && same; ++k) same = std::fabs(ta[k] - tb[k]) <= tol;
            if (same) {
                rep[qa] = std::min(rep[qa], qb);
                rep[qb] = std::min(rep[qb], qa);
            }
        }
    }
}

// Device tables of one set of scored rows (stacked [Re, -Im] rows of U, or
// of U / ||U sigma|| for eq. (15)): GEMM2 operands in the three precisions
// (FP16 scaled by a power of two so that the largest entry lands near 2^14),
// the FP32 rescoring copy per 64-row tile [tile][k/4][QTILE][4], each tile's
// largest row norm and the largest ||row sigma||.
static void pack_rows(svdphat_plan* p, const std::vector<float>& rows, const std::vector<float>& sg, float umax,
                      svdphat::ScoreRows& out, int64_t& bytes) {
    std::vector<float> u32;
    pack_U<float>(p, rows, 1.f, u32);
    upload(u32, &out.Ufr[P_FP32], bytes);
    out.uscale[P_FP32] = 1.f;
    float sc = 1.f;
    if (umax > 0.f) sc = std::ldexp(1.f, (int)std::floor(std::log2(16384.0 / umax)));
    std::vector<_Float16> u16;
    pack_U<_Float16>(p, rows, sc, u16);
    upload(u16, &out.Ufr[P_FP16], bytes);
    out.uscale[P_FP16] = sc;
    std::vector<__bf16> ub;
    pack_U<__bf16>(p, rows, 1.f, ub);
    upload(ub, &out.Ufr[P_BF16], bytes);
    out.uscale[P_BF16] = 1.f;
    const int ntile = p->ncls_pad / QTILE;
    std::vector<float> t((size_t)ntile * p->Rp * QTILE, 0.f);
    for (int r = 0; r < p->ncls; ++r)
        for (int k = 0; k < p->Rp; ++k)
            t[(((size_t)(r / QTILE) * (p->Rp / 4) + k / 4) * QTILE + r % QTILE) * 4 + k % 4] = rows[(size_t)r * p->Rp + k];
    void* d = nullptr;
    upload(t, &d, bytes);
    out.U32T = (float*)d;
    std::vector<float> tk(ntile, 0.f);
    double us = 0.0;
    for (int r = 0; r < p->ncls; ++r) {
        double nrm = 0.0, ns = 0.0;
        for (int k = 0; k < p->Rp; ++k) {
            const double v = rows[(size_t)r * p->Rp + k];
            const double vs = v * sg[k];
            nrm += v * v;
            ns += vs * vs;
        }
        tk[r / QTILE] = std::max(tk[r / QTILE], (float)(std::sqrt(nrm) * (1.0 + 1e-6)));
        us = std::max(us, std::sqrt(ns));
    }
    upload(tk, &d, bytes);
    out.tkappa = (float*)d;
    out.usig_max = (float)(us * (1.0 + 1e-6));
}

void build_plan(svdphat_plan* p, const double* mics, const double* grid, bool factored) {
    const int M = p->M, Q = p->Q, N = p->N;
    const int P = M * (M - 1) / 2, B = N / 2 + 1;
    const int64_t L = (int64_t)P * B;
    p->P = P;
    p->B = B;
    p->L = (int)L;

    // ---- eq. (2): tau[q][p] = fs/c (r_j - r_i) . s_q / ||s_q||, pairs i < j
    std::vector<int8_t> pi, pj;
    for (int i = 0; i < M; ++i)
        for (int j = i + 1; j < M; ++j) {
            pi.push_back((int8_t)i);
            pj.push_back((int8_t)j);
        }
    p->tau.resize((size_t)Q * P);
    p->grid.resize((size_t)Q * 3);
    for (int q = 0; q < Q; ++q) {
        const double* s = grid + 3 * q;
        double n = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        for (int d = 0; d < 3; ++d) p->grid[3 * (size_t)q + d] = s[d] / n;
        for (int k = 0; k < P; ++k) {
            const double* ri = mics + 3 * pi[k];
            const double* rj = mics + 3 * pj[k];
            double d = (rj[0] - ri[0]) * s[0] + (rj[1] - ri[1]) * s[1] + (rj[2] - ri[2]) * s[2];
            p->tau[(size_t)q * P + k] = p->fs / p->c * d / n;
        }
    }
    // per-microphone delays tau_m = fs/c r_m . s_q / ||s_q|| (tau of pair
    // (i, j) is tau_j - tau_i); used by the power of the chosen direction
    p->tauM.resize((size_t)Q * M);
    for (int q = 0; q < Q; ++q) {
        const double* s = grid + 3 * q;
        const double n = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        for (int m = 0; m < M; ++m) {
            const double* r = mics + 3 * m;
            p->tauM[(size_t)q * M + m] = p->fs / p->c * (r[0] * s[0] + r[1] * s[1] + r[2] * s[2]) / n;
        }
    }

    // ---- classes of identical delay rows
    direction_classes(p->tau, Q, P, 1e-9, p->rep);
    p->rows.clear();
    for (int q = 0; q < Q; ++q)
        if ((p->flags & SVDPHAT_NO_DEDUP) || p->rep[q] == q) p->rows.push_back(q);
    // Score rows in a space-filling-curve order of their directions (3-D
    // Morton code of the unit vector): nearby directions, whose powers are
    // close, share tiles, so few tiles are within the rescoring bound of the
    // frame maximum.  Ties of the search are still broken by direction index.
    {
        auto spread = [](uint32_t v) {
            uint64_t x = v & 0x3ff;
            x = (x | (x << 16)) & 0x30000ff;
            x = (x | (x << 8)) & 0x300f00f;
            x = (x | (x << 4)) & 0x30c30c3;
            x = (x | (x << 2)) & 0x9249249;
            return x;
        };
        std::vector<std::pair<uint64_t, int32_t>> key;
        key.reserve(p->rows.size());
        for (int32_t q : p->rows) {
            const double* sv = grid + 3 * q;
            const double nn = std::sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
            uint32_t c[3];
            for (int d = 0; d < 3; ++d) {
                double u = (sv[d] / nn + 1.0) * 0.5;
                c[d] = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(u * 1024.0)));
            }
            key.emplace_back(spread(c[0]) | (spread(c[1]) << 1) | (spread(c[2]) << 2), q);
        }
        std::sort(key.begin(), key.end());
        for (size_t i = 0; i < key.size(); ++i) p->rows[i] = key[i].second;
    }
    p->ncls = (int)p->rows.size();
    p->ncls_pad = round_up(p->ncls, 256);

    p->mics_in.assign(mics, mics + 3 * (size_t)M);
    p->grid_in.assign(grid, grid + 3 * (size_t)Q);
    SP_HIP(hipSetDevice(p->device));
    // the factors (sigma, U, V, K, K_paper, fro2, residual) of a saved plan
    // are given; otherwise Algorithm 1 offline steps 1-2 compute them
    if (!factored) {
    // ---- eqs. (4), (8): W in FP64 on the device (column-major Q x L)
    RB rb;
    rb_check(rocblas_create_handle(&rb.h), "rocblas_create_handle");
    DevBuf<double> d_tau;
    d_tau.alloc((size_t)Q * P);
    SP_HIP(hipMemcpy(d_tau.p, p->tau.data(), (size_t)Q * P * sizeof(double), hipMemcpyHostToDevice));
    DevBuf<rocblas_double_complex> W;
    W.alloc((size_t)Q * L);
    {
        int64_t total = (int64_t)Q * L;
        int threads = 256;
        int64_t blocks = (total + threads - 1) / threads;
        k_build_w64<<<dim3((unsigned)blocks), dim3(threads)>>>(d_tau.p, Q, P, N, total, W.p);
        SP_HIP(hipGetLastError());
    }

    // ---- Gram matrix of the smaller side and its eigendecomposition
    const bool vside = L <= Q;  // eigenvectors of W^H W are V, else of W W^H are U
    const int n = vside ? (int)L : Q;
    DevBuf<rocblas_double_complex> G;
    G.alloc((size_t)n * n);
    {
        double one = 1.0, zero = 0.0;
        if (vside)
            rb_check(rocblas_zherk(rb.h, rocblas_fill_lower, rocblas_operation_conjugate_transpose, n, Q, &one,
                                   W.p, Q, &zero, G.p, n),
                     "zherk");
        else
            rb_check(rocblas_zherk(rb.h, rocblas_fill_lower, rocblas_operation_none, n, (int)L, &one, W.p, Q,
                                   &zero, G.p, n),
                     "zherk");
    }
    DevBuf<double> D, E;
    D.alloc(n);
    E.alloc(n);
    DevBuf<rocblas_int> info;
    info.alloc(1);
    rb_check(rocsolver_zheevd(rb.h, rocblas_evect_original, rocblas_fill_lower, n, G.p, n, D.p, E.p, info.p),
             "zheevd");
    std::vector<double> lam(n);
    rocblas_int hinfo = 0;
    SP_HIP(hipMemcpy(lam.data(), D.p, n * sizeof(double), hipMemcpyDeviceToHost));
    SP_HIP(hipMemcpy(&hinfo, info.p, sizeof(rocblas_int), hipMemcpyDeviceToHost));
    if (hinfo != 0 || fault_forced("eig"))
        fail(SVDPHAT_E_NUMERIC, "zheevd did not converge (info " + std::to_string(hinfo) + ")");

    // ---- singular values (descending) and the rank rule of eq. (11)
    p->sigma.resize(n);
    double fro2 = 0.0;
    for (int k = 0; k < n; ++k) {
        double l = lam[n - 1 - k];
        if (!std::isfinite(l)) fail(SVDPHAT_E_NUMERIC, "non-finite eigenvalue");
        fro2 += l;
        p->sigma[k] = std::sqrt(std::max(l, 0.0));
    }
    p->fro2 = fro2;
    // smallest K with sum_{k<=K} s_k^2 >= (1 - delta) ||W||_F^2 (delta > 0)
    double target = (1.0 - p->delta) * fro2, cum = 0.0;
    int Kp = n;
    for (int k = 0; k < n; ++k) {
        cum += p->sigma[k] * p->sigma[k];
        if (cum >= target) {
            Kp = k + 1;
            break;
        }
    }
    int K = Kp;
    while (K < n && p->sigma[K] >= (1.0 - 1e-9) * p->sigma[K - 1]) ++K;
    p->K_paper = Kp;
    p->K = K;
    double kept = 0.0;
    for (int k = 0; k < K; ++k) kept += p->sigma[k] * p->sigma[k];
    p->residual = std::max(0.0, 1.0 - kept / fro2);

    // ---- the other factor from one product: U = W V / s, or V = W^H U / s
    // The top-K eigenvectors are the last K columns of G (ascending order).
    const rocblas_double_complex* Ek = G.p + (size_t)(n - K) * n;
    DevBuf<rocblas_double_complex> Fk;
    const int other = vside ? Q : (int)L;
    Fk.alloc((size_t)other * K);
    {
        rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
        if (vside)
            rb_check(rocblas_zgemm(rb.h, rocblas_operation_none, rocblas_operation_none, Q, K, (int)L, &one, W.p, Q,
                                   Ek, n, &zero, Fk.p, Q),
                     "zgemm");
        else
            rb_check(rocblas_zgemm(rb.h, rocblas_operation_conjugate_transpose, rocblas_operation_none, (int)L, K,
                                   Q, &one, W.p, Q, Ek, n, &zero, Fk.p, (int)L),
                     "zgemm");
    }
    std::vector<double> hE((size_t)n * K * 2), hF((size_t)other * K * 2);
    SP_HIP(hipMemcpy(hE.data(), Ek, hE.size() * sizeof(double), hipMemcpyDeviceToHost));
    SP_HIP(hipMemcpy(hF.data(), Fk.p, hF.size() * sizeof(double), hipMemcpyDeviceToHost));
    // column-major, ascending -> row-major [rows][K], descending, scaled
    p->U.assign((size_t)Q * K * 2, 0.0);
    p->V.assign((size_t)L * K * 2, 0.0);
    for (int kk = 0; kk < K; ++kk) {
        int col = K - 1 - kk;
        double inv = 1.0 / p->sigma[kk];
        if (!(p->sigma[kk] > 0.0)) fail(SVDPHAT_E_NUMERIC, "zero singular value inside the kept rank");
        std::vector<double>& eig = vside ? p->V : p->U;
        std::vector<double>& oth = vside ? p->U : p->V;
        for (int r = 0; r < n; ++r) {
            eig[((size_t)r * K + kk) * 2] = hE[((size_t)col * n + r) * 2];
            eig[((size_t)r * K + kk) * 2 + 1] = hE[((size_t)col * n + r) * 2 + 1];
        }
        for (int r = 0; r < other; ++r) {
            oth[((size_t)r * K + kk) * 2] = hF[((size_t)col * other + r) * 2] * inv;
            oth[((size_t)r * K + kk) * 2 + 1] = hF[((size_t)col * other + r) * 2 + 1] * inv;
        }
    }
    for (double v : p->U)
        if (!std::isfinite(v)) fail(SVDPHAT_E_NUMERIC, "non-finite U");
    for (double v : p->V)
        if (!std::isfinite(v)) fail(SVDPHAT_E_NUMERIC, "non-finite V");
    }

    // ---- packing
    const int K = p->K;
    p->R = 2 * K;
    p->Rp = round_up(p->R, 32);
    if (p->Rp > 1024) fail(SVDPHAT_E_UNSUPPORTED, "rank K above 512 is not supported");
    const int nRB = p->Rp / 16;
    p->g1[P_FP32] = make_layout(P, B, M, 4, Mf<float>::KSTEP, nRB, Mf<float>::EPL);
    p->g1[P_FP16] = make_layout(P, B, M, 2, Mf<_Float16>::KSTEP, nRB, Mf<_Float16>::EPL);
    p->g1[P_BF16] = make_layout(P, B, M, 2, Mf<__bf16>::KSTEP, nRB, Mf<__bf16>::EPL);
    int64_t bytes = 0;
    {
        std::vector<float> a32, dummy;
        pack_A<float>(p, p->g1[P_FP32], a32, dummy, false);
        upload(a32, &p->A[P_FP32], bytes);
        std::vector<_Float16> h, l;
        pack_A<_Float16>(p, p->g1[P_FP16], h, l, true);
        upload(h, &p->A[P_FP16], bytes);
        upload(l, &p->Alo[P_FP16], bytes);
        std::vector<__bf16> bh, bl;
        pack_A<__bf16>(p, p->g1[P_BF16], bh, bl, true);
        upload(bh, &p->A[P_BF16], bytes);
        upload(bl, &p->Alo[P_BF16], bytes);
        // two row-group passes of the streamed GEMM1 where Z has 8 to 12 row
        // blocks (6 in the first pass, the rest in the second)
        int cws = 0, bbs = 0;
        p->as_split = 0;
        if ((nRB == 8 || nRB == 10 || nRB == 12) && B >= 2 && g1s_layout(M, 6, Mf<_Float16>::KSTEP, &cws, &bbs)) {
            p->as_split = 6;
            for (int pr : {P_FP16, P_BF16}) {
                G1Layout& gs = p->g1s[pr];
                gs.CW = cws;
                gs.BB = bbs;
                gs.nch = cdiv(B, bbs);
                gs.ks_chunk = cws / Mf<_Float16>::KSTEP;
                gs.elems = 0;
                for (int g = 0; g < 2; ++g) {
                    const int rb0 = g == 0 ? 0 : 6, nrb = g == 0 ? 6 : nRB - 6;
                    if (pr == P_FP16) {
                        std::vector<_Float16> sh, sl;
                        pack_A<_Float16>(p, gs, sh, sl, false, rb0, nrb);
                        upload(sh, &p->As[pr][g], bytes);
                    } else {
                        std::vector<__bf16> sh, sl;
                        pack_A<__bf16>(p, gs, sh, sl, false, rb0, nrb);
                        upload(sh, &p->As[pr][g], bytes);
                    }
                }
            }
        }
        // FP32 rows of A = S V^H transposed for the GEMV form of small
        // batches: [(b P + p) 2 + ri][Rp], stacked as in pack_A
        std::vector<float> at((size_t)B * P * 2 * p->Rp, 0.f);
        for (int bin = 0; bin < B; ++bin)
            for (int pp = 0; pp < P; ++pp) {
                const int64_t c = (int64_t)bin * P + pp;
                for (int kk = 0; kk < K; ++kk) {
                    const double vr = p->V[(c * K + kk) * 2], vi = p->V[(c * K + kk) * 2 + 1];
                    const double ar = p->sigma[kk] * vr, ai = -p->sigma[kk] * vi;
                    float* re = &at[(size_t)(c * 2) * p->Rp];
                    float* im = &at[(size_t)(c * 2 + 1) * p->Rp];
                    re[kk] = (float)ar;
                    re[K + kk] = (float)ai;
                    im[kk] = (float)(-ai);
                    im[K + kk] = (float)ar;
                }
            }
        void* d = nullptr;
        upload(at, &d, bytes);
        p->A32T = (float*)d;
    }
    // stacked U rows (FP32) of the scored directions
    std::vector<float> Ust((size_t)p->ncls_pad * p->Rp, 0.f);
    double kappa = 0.0;
    float umax = 0.f;
    for (int r = 0; r < p->ncls; ++r) {
        int q = p->rows[r];
        double nrm = 0.0;
        for (int kk = 0; kk < K; ++kk) {
            double ur = p->U[((size_t)q * K + kk) * 2], ui = p->U[((size_t)q * K + kk) * 2 + 1];
            Ust[(size_t)r * p->Rp + kk] = (float)ur;
            Ust[(size_t)r * p->Rp + K + kk] = (float)(-ui);
            nrm += ur * ur + ui * ui;
            umax = std::max(umax, std::max(std::fabs((float)ur), std::fabs((float)ui)));
        }
        kappa = std::max(kappa, std::sqrt(nrm));
    }
    p->kappa = kappa;
    // singular value of each stacked row of Z (rows k and K + k: s_k)
    std::vector<float> sg(p->Rp, 0.f);
    for (int k = 0; k < K; ++k) sg[k] = sg[K + k] = (float)p->sigma[k];
    {
        void* d = nullptr;
        upload(sg, &d, bytes);
        p->d_sig = (float*)d;
    }
    pack_rows(p, Ust, sg, umax, p->sr[0], bytes);
    // eq. (15): the same search over the rows D_q / ||D_q|| (D_q = U_q S,
    // ||D_q|| = ||U_q sigma|| from the FP64 factors)
    {
        std::vector<float> Un(Ust.size(), 0.f);
        float unmax = 0.f;
        for (int r = 0; r < p->ncls; ++r) {
            const int q = p->rows[r];
            double nrm = 0.0;
            for (int kk = 0; kk < K; ++kk) {
                const double ur = p->U[((size_t)q * K + kk) * 2], ui = p->U[((size_t)q * K + kk) * 2 + 1];
                nrm += (ur * ur + ui * ui) * p->sigma[kk] * p->sigma[kk];
            }
            const double inv = nrm > 0.0 ? 1.0 / std::sqrt(nrm) : 0.0;
            for (int kk = 0; kk < K; ++kk) {
                const double ur = p->U[((size_t)q * K + kk) * 2], ui = p->U[((size_t)q * K + kk) * 2 + 1];
                Un[(size_t)r * p->Rp + kk] = (float)(ur * inv);
                Un[(size_t)r * p->Rp + K + kk] = (float)(-ui * inv);
                unmax = std::max(unmax, std::max(std::fabs((float)(ur * inv)), std::fabs((float)(ui * inv))));
            }
        }
        pack_rows(p, Un, sg, unmax, p->sr[1], bytes);
    }
    {
        std::vector<int32_t> rows(p->rows);
        void* d = nullptr;
        upload(rows, &d, bytes);
        p->d_rows = (int32_t*)d;
        upload(p->rep, &d, bytes);
        p->d_rep = (int32_t*)d;
        std::vector<int32_t> rowof(Q, 0), rowidx(Q, -1);
        for (int r = 0; r < p->ncls; ++r) rowidx[p->rows[r]] = r;
        for (int q = 0; q < Q; ++q) rowof[q] = rowidx[q] >= 0 ? rowidx[q] : rowidx[p->rep[q]];
        upload(rowof, &d, bytes);
        p->d_rowof = (int32_t*)d;
        std::vector<float> tn((size_t)Q * P);
        for (size_t i = 0; i < tn.size(); ++i) tn[i] = (float)(p->tau[i] / N);
        upload(tn, &d, bytes);
        p->d_tauN_all = (float*)d;
        std::vector<float> tm(p->tauM.size());
        for (size_t i = 0; i < tm.size(); ++i) tm[i] = (float)(p->tauM[i] / N);
        upload(tm, &d, bytes);
        p->d_tauM_all = (float*)d;
        // class of each scored row (padding rows: class 0)
        std::vector<int32_t> rc(p->ncls_pad, 0);
        for (int r = 0; r < p->ncls; ++r) rc[r] = p->rep[p->rows[r]];
        upload(rc, &d, bytes);
        p->d_rowcls = (int32_t*)d;
        upload(pi, &d, bytes);
        p->d_pi = (int8_t*)d;
        upload(pj, &d, bytes);
        p->d_pj = (int8_t*)d;
    }
    p->device_bytes = bytes;
    if (p->flags & SVDPHAT_KEEP_W) {
        build_w_fp32_frags(p);
        SP_HIP(hipDeviceSynchronize());
    }
    SP_HIP(hipDeviceSynchronize());
}

}  // namespace svdphat
