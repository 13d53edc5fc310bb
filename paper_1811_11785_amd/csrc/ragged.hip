// Ragged batches: many arrays (each its own plan: microphones, grid, rank)
// located in one launch of a HIP graph.  The graph holds one grouped kernel
// per search stage and template class; each walks a device work list of
// (array, tile) items built for the arrays' maximum frame counts, and items
// past an array's current frame count exit at once.  Per call only the
// per-array descriptors (input/output pointers, frame counts) are copied to
// the device before the graph launch.  GEMM1's split of the reduction axis and
// GEMM2's frames per workgroup are chosen per array by timing candidates
// (autotuner), with the winners kept in a JSON-lines cache keyed by GPU
// architecture and problem shape.
#include "internal.h"

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

struct svdphat_ragged {
    int device = 0;
    std::vector<svdphat_plan*> plans;
    std::vector<int64_t> maxF;
    std::vector<int> nsplit, cps, fch;
    svdphat::RDesc* d_desc = nullptr;
    svdphat::RDesc* h_desc = nullptr;  // pinned staging
    hipEvent_t copied = nullptr;
    bool copy_pending = false;
    void* ws = nullptr;
    std::vector<svdphat::GroupLaunch> launches;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t tuned = 0, cached = 0;
};

namespace svdphat {

namespace {

std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string shape_key(const svdphat_plan* p, int64_t F) {
    int fb = 0;
    while ((64ll << fb) < F) ++fb;
    std::ostringstream k;
    k << "M" << p->M << "_B" << p->B << "_R" << p->Rp << "_C" << p->ncls_pad << "_F" << (64ll << fb);
    return k.str();
}

// JSON lines: {"arch": "gfx950", "key": "...", "nsplit": n, "fch": f}
std::map<std::string, std::pair<int, int>> load_cache(const char* path, const std::string& arch) {
    std::map<std::string, std::pair<int, int>> m;
    if (!path || !*path) return m;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        char a[64] = {0}, k[128] = {0};
        int ns = 0, fc = 0;
        if (std::sscanf(line.c_str(), " {\"arch\": \"%63[^\"]\", \"key\": \"%127[^\"]\", \"nsplit\": %d, \"fch\": %d",
                        a, k, &ns, &fc) == 4 &&
            arch == a && ns > 0 && fc > 0)
            m[k] = {ns, fc};
    }
    return m;
}

void append_cache(const char* path, const std::string& arch, const std::string& key, int ns, int fc) {
    if (!path || !*path) return;
    std::ofstream out(path, std::ios::app);
    out << "{\"arch\": \"" << arch << "\", \"key\": \"" << key << "\", \"nsplit\": " << ns << ", \"fch\": " << fc
        << "}\n";
}

void free_ragged(svdphat_ragged* r) {
    if (!r) return;
    (void)hipSetDevice(r->device);
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    if (r->cap) (void)hipStreamDestroy(r->cap);
    if (r->copied) (void)hipEventDestroy(r->copied);
    for (auto& g : r->launches)
        if (g.work) (void)hipFree(g.work);
    if (r->d_desc) (void)hipFree(r->d_desc);
    if (r->h_desc) (void)hipHostFree(r->h_desc);
    if (r->ws) (void)hipFree(r->ws);
    (void)hipGetLastError();  // no error of the teardown outlives it
    delete r;
}

}  // namespace

void ragged_build(svdphat_ragged* r, uint32_t flags, const char* cache_path) {
    const int n = (int)r->plans.size();
    const std::string arch = arch_name(r->device);
    auto cache = load_cache(cache_path, arch);
    hipStream_t ts = nullptr;
    SP_HIP(hipStreamCreate(&ts));
    r->nsplit.resize(n);
    r->cps.resize(n);
    r->fch.resize(n);
    std::map<std::string, std::pair<int, int>> chosen;
    for (int i = 0; i < n; ++i) {
        svdphat_plan* p = r->plans[i];
        const std::string key = shape_key(p, r->maxF[i]);
        std::pair<int, int> best{0, 256};
        auto it = chosen.find(key);
        if (it != chosen.end()) best = it->second;
        else if (cache.count(key)) {
            best = cache[key];
            ++r->cached;
        } else if (flags & SVDPHAT_RAGGED_TUNE) {
            // autotune: split of GEMM1 and frames per GEMM2 workgroup
            double b1 = 1e30, b2 = 1e30;
            for (int ns : {1, 2, 4, 8}) {
                if (ns > p->g1[P_FP16].nch) break;
                double t1, t2;
                tune_time(p, r->maxF[i], ns, 256, &t1, &t2, ts);
                if (t1 < b1) {
                    b1 = t1;
                    best.first = ns;
                }
            }
            for (int fc : {64, 128, 256, 512}) {
                double t1, t2;
                tune_time(p, r->maxF[i], best.first, fc, &t1, &t2, ts);
                if (t2 < b2) {
                    b2 = t2;
                    best.second = fc;
                }
            }
            append_cache(cache_path, arch, key, best.first, best.second);
            ++r->tuned;
        }
        chosen[key] = best;
        g1_split(p, r->maxF[i], best.first, &r->nsplit[i], &r->cps[i]);
        r->fch[i] = best.second;
    }
    SP_HIP(hipStreamSynchronize(ts));
    SP_HIP(hipStreamDestroy(ts));

    // workspace and static descriptor fields
    std::vector<size_t> off(n);
    size_t total = 0;
    auto take = [&](size_t bytes) {
        size_t o = total;
        total += round_up64((int64_t)bytes, 256);
        return o;
    };
    struct Offs {
        size_t zp, z, zf, sc, zn, pm;
    };
    std::vector<Offs> of(n);
    for (int i = 0; i < n; ++i) {
        const svdphat_plan* p = r->plans[i];
        const int64_t Fc = round_up64(r->maxF[i], 64);
        const int ntile = p->ncls_pad / QTILE;
        of[i].zp = take(sizeof(float) * r->nsplit[i] * Fc * p->Rp);
        of[i].z = take(sizeof(float) * Fc * p->Rp);
        of[i].zf = take(sizeof(_Float16) * Fc * p->Rp);
        of[i].sc = take(sizeof(float) * Fc);
        of[i].zn = take(sizeof(float) * Fc);
        of[i].pm = take(sizeof(float) * pmax_stride(p) * Fc);
    }
    if (dev_malloc(&r->ws, std::max<size_t>(total, 256)) != hipSuccess) {
        r->ws = nullptr;
        fail(SVDPHAT_E_NOMEM, "ragged workspace of " + std::to_string(total) + " bytes");
    }
    SP_HIP(hipHostMalloc((void**)&r->h_desc, sizeof(RDesc) * n, hipHostMallocDefault));
    dev_alloc((void**)&r->d_desc, sizeof(RDesc) * n, "ragged descriptors");
    char* w = (char*)r->ws;
    for (int i = 0; i < n; ++i) {
        svdphat_plan* p = r->plans[i];
        const G1Layout& g = p->g1[P_FP16];
        const int64_t Fc = round_up64(r->maxF[i], 64);
        RDesc d{};
        d.X = nullptr;
        d.F = 0;
        d.M = p->M;
        d.P = p->P;
        d.B = p->B;
        d.A = p->A[P_FP16];
        d.nRB = p->Rp / 16;
        d.BB = g.BB;
        d.CW = g.CW;
        d.nch = g.nch;
        d.cps = r->cps[i];
        d.nsplit = r->nsplit[i];
        d.Rp = p->Rp;
        d.zpart = (float*)(w + of[i].zp);
        d.zstride = Fc * p->Rp;
        d.z32 = (float*)(w + of[i].z);
        d.zfrag = w + of[i].zf;
        d.zsc = (float*)(w + of[i].sc);
        d.zn = (float*)(w + of[i].zn);
        d.U = p->sr[0].Ufr[P_FP16];
        d.KSn = p->Rp / Mf<_Float16>::KSTEP;
        d.ncls = p->ncls;
        d.ntile = p->ncls_pad / QTILE;
        d.fch = r->fch[i];
        d.uinv = 1.f / p->sr[0].uscale[P_FP16];
        d.pmax = (float*)(w + of[i].pm);
        d.pstride = pmax_stride(p);
        FinalArgs& fa = d.fin;
        fa.M = p->M;
        fa.P = p->P;
        fa.B = p->B;
        fa.pmax = d.pmax;
        fa.pstride = d.pstride;
        fa.ntile = d.ntile;
        fa.ncls = p->ncls;
        fa.z32 = d.z32;
        fa.znorm1 = d.zn;
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
        fa.hilo_k = 4.f;
        fa.u = (float)u;
        r->h_desc[i] = d;
    }

    // work lists, one per (stage, class).  GEMM1's items are dealt to the
    // eight XCDs (workgroup b of a launch runs on XCD b mod 8): an array's
    // items in A-region order ((split, row group) major, frame tile minor)
    // are cut into up to eight contiguous parts, each queued for one XCD
    // (a rotating start balances the queues), so that each XCD reads its
    // part of A into its own L2 and serves every frame tile from there;
    // the queues are interleaved, shorter ones padded with empty items.
    std::map<std::pair<int, int>, std::vector<int4>> lists;
    std::map<std::pair<int, int>, size_t> lds;
    std::map<std::pair<int, int>, std::array<std::vector<int4>, 8>> xq;
    std::map<std::pair<int, int>, int> xrot;
    for (int i = 0; i < n; ++i) {
        const svdphat_plan* p = r->plans[i];
        const G1Layout& g = p->g1[P_FP16];
        const int64_t F = r->maxF[i];
        const int64_t Fc = round_up64(F, 64);
        const int nRB = p->Rp / 16;
        const int NRB = g1_nrb_class(nRB);
        const int big = p->M > 8 ? 1 : 0;
        const auto k1 = std::make_pair(0, NRB * 2 + big);
        {
            std::vector<int4> it;
            for (int sp = 0; sp < r->nsplit[i]; ++sp)
                for (int rg = 0; rg < cdiv(nRB, NRB); ++rg)
                    for (int64_t ft = 0; ft < Fc / 64; ++ft) it.push_back(int4{i, (int)ft, sp, rg});
            auto& q = xq[k1];
            int& o = xrot[k1];
            const size_t ni = it.size();
            const int parts = (int)std::min<size_t>(8, ni);
            for (int j = 0; j < parts; ++j)
                for (size_t t = j * ni / parts; t < (j + 1) * ni / parts; ++t) q[(o + j) % 8].push_back(it[t]);
            o = (o + parts) % 8;
        }
        lds[k1] = std::max(lds[k1], g1_lds_bytes(NRB, g.CW));
        for (int64_t bx = 0; bx < Fc / 4; ++bx) lists[{1, 0}].push_back(int4{i, (int)bx, 0, 0});
        const int ntile = p->ncls_pad / QTILE;
        const int ksn = p->Rp / Mf<_Float16>::KSTEP;
        const int ureg = ksn <= 6 ? ksn : 0;  // exact k-step class, 0: general form
        for (int bx = 0; bx < cdiv(ntile, 4); ++bx)
            for (int64_t by = 0; by < (F + r->fch[i] - 1) / r->fch[i]; ++by)
                lists[{2, ureg}].push_back(int4{i, bx, (int)by, 0});
        for (int64_t bx = 0; bx < (F + 3) / 4; ++bx) lists[{3, big}].push_back(int4{i, (int)bx, 0, 0});
    }
    for (auto& kv : xq) {
        size_t len = 0;
        for (auto& v : kv.second) len = std::max(len, v.size());
        auto& L = lists[kv.first];
        for (size_t k = 0; k < len; ++k)
            for (int x = 0; x < 8; ++x) L.push_back(k < kv.second[x].size() ? kv.second[x][k] : int4{-1, 0, 0, 0});
    }
    for (auto& kv : lists) {
        GroupLaunch gl;
        gl.stage = kv.first.first;
        gl.cls = kv.first.second;
        gl.nwork = (int)kv.second.size();
        gl.lds = lds.count(kv.first) ? lds[kv.first] : 0;
        dev_alloc((void**)&gl.work, sizeof(int4) * kv.second.size(), "ragged work list");
        SP_HIP(hipMemcpy(gl.work, kv.second.data(), sizeof(int4) * kv.second.size(), hipMemcpyHostToDevice));
        r->launches.push_back(gl);
    }
    std::stable_sort(r->launches.begin(), r->launches.end(),
                     [](const GroupLaunch& a, const GroupLaunch& b) { return a.stage < b.stage; });

    // capture the stage launches into one graph
    SP_HIP(hipEventCreateWithFlags(&r->copied, hipEventDisableTiming));
    SP_HIP(hipStreamCreate(&r->cap));
    SP_HIP(hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal));
    for (auto& g : r->launches) launch_grouped(g, r->d_desc, r->cap);
    hipError_t e = hipStreamEndCapture(r->cap, &r->graph);
    if (e != hipSuccess) fail(SVDPHAT_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    SP_HIP(hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0));
}

void ragged_locate(svdphat_ragged* r, const void* const* X, const int64_t* F, int32_t* const* doa,
                   float* const* power, hipStream_t s) {
    const int n = (int)r->plans.size();
    if (r->copy_pending) SP_HIP(hipEventSynchronize(r->copied));
    for (int i = 0; i < n; ++i) {
        SP_REQUIRE(F[i] >= 0 && F[i] <= r->maxF[i], SVDPHAT_E_INVAL,
                   "frame count of array " + std::to_string(i) + " above its maximum");
        SP_REQUIRE(F[i] == 0 || (X[i] && doa[i] && power[i]), SVDPHAT_E_INVAL,
                   "NULL pointer for array " + std::to_string(i));
        RDesc& d = r->h_desc[i];
        d.X = (const float2*)X[i];
        d.F = F[i];
        d.fin.X = d.X;
        d.fin.nfr = F[i];
        d.fin.doa = doa[i];
        d.fin.power = power[i];
    }
    SP_HIP(hipMemcpyAsync(r->d_desc, r->h_desc, sizeof(RDesc) * n, hipMemcpyHostToDevice, s));
    SP_HIP(hipEventRecord(r->copied, s));
    r->copy_pending = true;
    SP_HIP(hipGraphLaunch(r->exec, s));
}

void ragged_destroy(svdphat_ragged* r) { free_ragged(r); }

svdphat_ragged* ragged_new(svdphat_plan* const* plans, int n, const int64_t* maxF) {
    auto* r = new svdphat_ragged();
    r->plans.assign(plans, plans + n);
    r->maxF.assign(maxF, maxF + n);
    r->device = plans[0]->device;
    return r;
}

void ragged_stats(const svdphat_ragged* r, int64_t* tuned, int64_t* cached) {
    if (tuned) *tuned = r->tuned;
    if (cached) *cached = r->cached;
}

}  // namespace svdphat
