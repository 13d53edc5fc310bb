// C ABI of the SVD-PHAT library: argument checking, error model, workspace
// pool, and dispatch to the plan builder and the kernel launchers.
#include "internal.h"

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

namespace svdphat {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {
__global__ __launch_bounds__(256) void k_zero_words(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}
}  // namespace

void zero_async(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    k_zero_words<<<dim3((unsigned)blocks), 256, 0, s>>>((uint32_t*)p, n);
    SP_HIP(hipGetLastError());
}
void fail(int code, const std::string& msg) { throw Error{code, msg}; }

bool fault_forced(const char* kind) {
    const char* env = std::getenv("SVDPHAT_FAULT");
    if (!env || !*env) return false;
    const std::string list = std::string(",") + env + ",";
    return list.find(std::string(",") + kind + ",") != std::string::npos;
}

hipError_t dev_malloc(void** p, size_t bytes) {
    if (fault_forced("alloc")) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

void dev_alloc(void** p, size_t bytes, const char* what) {
    if (dev_malloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        fail(SVDPHAT_E_NOMEM, std::string(what) + ": device allocation of " + std::to_string(bytes) + " bytes failed");
    }
}

// Workspace of one stream on one plan, grown on demand (hipMalloc outside any
// kernel; calls on the same plan and stream are ordered by the stream).  A
// HIP graph captured earlier on the stream may still reference a superseded
// buffer, so a grown-out buffer is kept until the plan is destroyed (growth
// is by at least 1.5x, so the kept buffers add at most twice the largest).
// Growing while the stream is being captured is refused: a capture must be
// preceded by one eager call of at least its size on the same stream.
void* ws_get(svdphat_plan* p, hipStream_t s, size_t bytes, int slot) {
    std::lock_guard<std::mutex> lk(p->ws_mu);
    Workspace& w = p->ws[std::make_pair((void*)s, slot)];
    if (w.bytes < bytes) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        SP_HIP(hipStreamIsCapturing(s, &cs));
        SP_REQUIRE(cs == hipStreamCaptureStatusNone, SVDPHAT_E_INVAL,
                   "the workspace of this stream must grow to " + std::to_string(bytes) +
                       " bytes while the stream is being captured: make one call of this size on the stream "
                       "before capturing");
        size_t n = (size_t)round_up64((int64_t)std::max(bytes, w.bytes + w.bytes / 2), 1 << 20);
        void* nb = nullptr;
        if (dev_malloc(&nb, n) != hipSuccess) {
            (void)hipGetLastError();
            fail(SVDPHAT_E_NOMEM, "workspace allocation of " + std::to_string(n) + " bytes failed");
        }
        // (the superseded buffer is retired only once its successor exists,
        // so a failed growth leaves the workspace as it was)
        if (w.buf) p->ws_retired.push_back(w.buf);
        w.buf = nb;
        w.bytes = n;
    }
    return w.buf;
}

template <typename Fn>
static int guarded(Fn&& fn) {
    try {
        fn();
        g_last_error.clear();
        return SVDPHAT_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return SVDPHAT_E_NOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SVDPHAT_E_DEVICE;
    } catch (...) {
        g_last_error = "unknown failure";
        return SVDPHAT_E_DEVICE;
    }
}

static void free_plan(svdphat_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    for (int i = 0; i < 3; ++i) {
        if (p->A[i]) (void)hipFree(p->A[i]);
        if (p->Alo[i]) (void)hipFree(p->Alo[i]);
        for (auto& sr : p->sr)
            if (sr.Ufr[i]) (void)hipFree(sr.Ufr[i]);
        for (void* a : p->As[i])
            if (a) (void)hipFree(a);
    }
    void* bufs[] = {p->sr[0].U32T, p->sr[1].U32T, p->A32T, p->sr[0].tkappa, p->sr[1].tkappa, p->d_sig, p->d_rows, p->d_rep, p->d_rowof, p->d_tauN, p->d_tauN_all, p->d_tauM_all, p->d_rowcls, p->d_pi, p->d_pj, p->Wfr};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (auto& kv : p->ws)
        if (kv.second.buf) (void)hipFree(kv.second.buf);
    for (void* b : p->ws_retired) (void)hipFree(b);
    (void)hipGetLastError();  // no error of the teardown outlives it
    delete p;
}

static void require_device() {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        fail(SVDPHAT_E_NODEV, "no HIP device available");
    }
}


// ------------------------------------------------ allocation-free locate
// Intermediate results of svdphat_locate_noalloc live in this file-scope
// device array: every GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, so its
// device address is looked up once per device (with that device current) and
// only that address is ever passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> its copy of `scratch`

void* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void* ptr = nullptr;
    SP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    SP_REQUIRE(ptr != nullptr, SVDPHAT_E_DEVICE, "no device address for the scratch array");
    g_scratch_ptr[device] = ptr;
    return ptr;
}
}  // namespace

// ------------------------------------------------------------ timing
namespace {
struct TimingTable {
    std::mutex mu;
    bool on = false;
    bool counts = false;
    std::map<std::string, std::pair<double, int64_t>> t;
};
TimingTable& timing() {
    static TimingTable tt;
    return tt;
}
}  // namespace

bool timing_on() { return timing().on; }
bool counting_on() { return timing().counts; }

void timing_count(const char* name, double count, int64_t calls) {
    std::lock_guard<std::mutex> lk(timing().mu);
    auto& e = timing().t[name];
    e.first += count;
    e.second += calls;
}

void KernelTimer::begin(const char* name, hipStream_t on) {
    if (!timing_on()) return;
    Rec r{name, nullptr, nullptr, on ? on : s};
    SP_HIP(hipEventCreate(&r.a));
    SP_HIP(hipEventCreate(&r.b));
    SP_HIP(hipEventRecord(r.a, r.s));
    recs.push_back(r);
}
void KernelTimer::end() {
    if (!timing_on() || recs.empty()) return;
    SP_HIP(hipEventRecord(recs.back().b, recs.back().s));
}
void KernelTimer::flush() {
    for (auto& r : recs) {
        SP_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        SP_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        std::lock_guard<std::mutex> lk(timing().mu);
        auto& e = timing().t[r.name];
        e.first += ms;
        e.second += 1;
    }
    for (auto& r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    recs.clear();
}
KernelTimer::~KernelTimer() {
    for (auto& r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
}

}  // namespace svdphat

using namespace svdphat;

extern "C" {

int svdphat_version(void) { return 10000; }

const char* svdphat_last_error(void) { return g_last_error.c_str(); }

int svdphat_plan_create(const double* mic_xyz_m, int32_t M, const double* grid_xyz, int32_t Q, double fs,
                        double c, int32_t N, double delta, uint32_t flags, svdphat_plan** out) {
    return guarded([&] {
        SP_REQUIRE(out != nullptr, SVDPHAT_E_INVAL, "out is NULL");
        *out = nullptr;
        SP_REQUIRE(mic_xyz_m && grid_xyz, SVDPHAT_E_INVAL, "NULL geometry or grid");
        SP_REQUIRE(M >= 2 && M <= 16, SVDPHAT_E_INVAL, "M must be in [2, 16]");
        SP_REQUIRE(Q >= 1, SVDPHAT_E_INVAL, "Q must be >= 1");
        SP_REQUIRE(N >= 2 && N % 2 == 0, SVDPHAT_E_INVAL, "N must be even and >= 2");
        SP_REQUIRE(std::isfinite(fs) && fs > 0 && std::isfinite(c) && c > 0, SVDPHAT_E_INVAL,
                   "fs and c must be finite and > 0");
        SP_REQUIRE(std::isfinite(delta) && delta > 0.0 && delta < 1.0, SVDPHAT_E_INVAL, "delta must be in (0, 1)");
        SP_REQUIRE((flags & ~(uint32_t)(SVDPHAT_KEEP_W | SVDPHAT_NO_DEDUP)) == 0, SVDPHAT_E_INVAL, "unknown flags");
        for (int i = 0; i < 3 * M; ++i)
            SP_REQUIRE(std::isfinite(mic_xyz_m[i]), SVDPHAT_E_INVAL, "non-finite microphone position");
        for (int q = 0; q < Q; ++q) {
            const double* s = grid_xyz + 3 * q;
            SP_REQUIRE(std::isfinite(s[0]) && std::isfinite(s[1]) && std::isfinite(s[2]), SVDPHAT_E_INVAL,
                       "non-finite grid direction");
            SP_REQUIRE(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] > 0.0, SVDPHAT_E_INVAL,
                       "zero grid direction at row " + std::to_string(q));
        }
        const int64_t L = (int64_t)M * (M - 1) / 2 * (N / 2 + 1);
        SP_REQUIRE(L < (int64_t)1 << 30 && (int64_t)Q * L < ((int64_t)1 << 40), SVDPHAT_E_INVAL, "problem too large");
        require_device();
        svdphat_plan* p = new svdphat_plan();
        SP_HIP(hipGetDevice(&p->device));
        p->M = M;
        p->Q = Q;
        p->N = N;
        p->fs = fs;
        p->c = c;
        p->delta = delta;
        p->flags = flags;
        try {
            build_plan(p, mic_xyz_m, grid_xyz, false);
        } catch (...) {
            free_plan(p);
            throw;
        }
        *out = p;
    });
}

int svdphat_plan_save(const svdphat_plan* p, const char* path) {
    return guarded([&] {
        SP_REQUIRE(p && path, SVDPHAT_E_INVAL, "NULL plan or path");
        plan_save(p, path);
    });
}

int svdphat_plan_load(const char* path, svdphat_plan** out) {
    return guarded([&] {
        SP_REQUIRE(out != nullptr, SVDPHAT_E_INVAL, "out is NULL");
        *out = nullptr;
        SP_REQUIRE(path != nullptr, SVDPHAT_E_INVAL, "NULL path");
        *out = plan_load(path, free_plan);
    });
}

uint64_t svdphat_plan_input_hash(const double* mic_xyz_m, int32_t M, const double* grid_xyz, int32_t Q, double fs,
                                 double c, int32_t N, double delta, uint32_t flags) {
    if (!mic_xyz_m || !grid_xyz || M < 0 || Q < 0) return 0;
    return plan_input_hash(mic_xyz_m, M, grid_xyz, Q, fs, c, N, delta, flags);
}

int svdphat_plan_info(const svdphat_plan* p, svdphat_info* o) {
    return guarded([&] {
        SP_REQUIRE(p && o, SVDPHAT_E_INVAL, "NULL argument");
        std::memset(o, 0, sizeof(*o));
        o->M = p->M;
        o->P = p->P;
        o->B = p->B;
        o->L = p->L;
        o->Q = p->Q;
        o->n_classes = p->ncls;
        o->K = p->K;
        o->K_paper = p->K_paper;
        o->N = p->N;
        o->has_w = p->Wfr != nullptr;
        o->residual = p->residual;
        o->sigma1 = p->sigma.empty() ? 0.0 : p->sigma[0];
        o->sigmaK = p->K > 0 ? p->sigma[p->K - 1] : 0.0;
        o->fro2 = p->fro2;
        o->u_rownorm_max = p->kappa;
        o->device_bytes = p->device_bytes;
        o->input_hash = plan_input_hash(p->mics_in.data(), p->M, p->grid_in.data(), p->Q, p->fs, p->c, p->N,
                                        p->delta, p->flags);
    });
}

int svdphat_plan_export(const svdphat_plan* p, double* sigma, double* U, double* V, int32_t* class_rep) {
    return guarded([&] {
        SP_REQUIRE(p, SVDPHAT_E_INVAL, "NULL plan");
        if (sigma) std::memcpy(sigma, p->sigma.data(), p->sigma.size() * sizeof(double));
        if (U) std::memcpy(U, p->U.data(), p->U.size() * sizeof(double));
        if (V) {
            // internal row c = bin * P + pair -> eq. (7) row pair * B + bin
            const int K = p->K;
            for (int bin = 0; bin < p->B; ++bin)
                for (int pp = 0; pp < p->P; ++pp) {
                    const size_t src = ((size_t)bin * p->P + pp) * K * 2;
                    const size_t dst = ((size_t)pp * p->B + bin) * K * 2;
                    std::memcpy(V + dst, p->V.data() + src, (size_t)K * 2 * sizeof(double));
                }
        }
        if (class_rep) std::memcpy(class_rep, p->rep.data(), p->rep.size() * sizeof(int32_t));
    });
}

int svdphat_locate(svdphat_plan* p, const void* X, int64_t F, int32_t precision, uint32_t mode, int32_t* doa,
                   float* power, float* yhat, float* margin, float* y_opt, void* stream) {
    return guarded([&] {
        SP_REQUIRE(p, SVDPHAT_E_INVAL, "NULL plan");
        SP_REQUIRE(F >= 0 && F < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "F out of range");
        SP_REQUIRE(precision == SVDPHAT_FP32 || precision == SVDPHAT_BF16 || precision == SVDPHAT_FP16,
                   SVDPHAT_E_INVAL, "unknown precision");
        SP_REQUIRE((mode & ~(uint32_t)(SVDPHAT_RESCORE | SVDPHAT_HILO | SVDPHAT_HILO_ALL | SVDPHAT_NORMALIZED)) == 0,
                   SVDPHAT_E_INVAL, "unknown mode bits");
        if (F == 0) return;
        SP_REQUIRE(X && doa && power, SVDPHAT_E_INVAL, "NULL X, doa or power");
        SP_HIP(hipSetDevice(p->device));
        launch_locate(p, X, F, precision, mode, doa, power, yhat, margin, y_opt, (hipStream_t)stream);
    });
}

int svdphat_locate_noalloc(svdphat_plan* p, const void* X, int64_t F, int32_t precision, uint32_t mode,
                           int32_t* doa, float* power, float* yhat, float* margin, void* stream) {
    return guarded([&] {
        SP_REQUIRE(p, SVDPHAT_E_INVAL, "NULL plan");
        SP_REQUIRE(F >= 0 && F < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "F out of range");
        SP_REQUIRE(precision == SVDPHAT_FP32 || precision == SVDPHAT_BF16 || precision == SVDPHAT_FP16,
                   SVDPHAT_E_INVAL, "unknown precision");
        SP_REQUIRE((mode & ~(uint32_t)(SVDPHAT_RESCORE | SVDPHAT_HILO | SVDPHAT_HILO_ALL | SVDPHAT_NORMALIZED)) == 0,
                   SVDPHAT_E_INVAL, "unknown mode bits");
        if (F == 0) return;
        SP_REQUIRE(X && doa && power, SVDPHAT_E_INVAL, "NULL X, doa or power");
        SP_HIP(hipSetDevice(p->device));
        void* ws = scratch_ptr(p->device);
        launch_locate(p, X, F, precision, mode, doa, power, yhat, margin, nullptr, (hipStream_t)stream, ws,
                      NOALLOC_SCRATCH_BYTES);
    });
}

int64_t svdphat_noalloc_scratch_bytes(void) { return (int64_t)NOALLOC_SCRATCH_BYTES; }

int svdphat_locate_masked(svdphat_plan* p, const void* X, int64_t F, const uint8_t* mask, int32_t precision,
                          uint32_t mode, int32_t* doa, float* power, float* yhat, float* margin, float* y_opt,
                          void* stream) {
    return guarded([&] {
        SP_REQUIRE(p, SVDPHAT_E_INVAL, "NULL plan");
        SP_REQUIRE(F >= 0 && F < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "F out of range");
        SP_REQUIRE(precision == SVDPHAT_FP32 || precision == SVDPHAT_BF16 || precision == SVDPHAT_FP16,
                   SVDPHAT_E_INVAL, "unknown precision");
        SP_REQUIRE((mode & ~(uint32_t)(SVDPHAT_RESCORE | SVDPHAT_HILO | SVDPHAT_HILO_ALL | SVDPHAT_NORMALIZED)) == 0,
                   SVDPHAT_E_INVAL, "unknown mode bits");
        if (F == 0) return;
        SP_REQUIRE(X && mask && doa && power, SVDPHAT_E_INVAL, "NULL X, mask, doa or power");
        SP_HIP(hipSetDevice(p->device));
        const hipStream_t s = (hipStream_t)stream;
        const size_t xbytes = (size_t)F * p->M * p->B * sizeof(float2);
        if (mask_fused(p, F, precision, y_opt != nullptr)) {
            // the streamed GEMM1's producers and the power kernel read the
            // mask with the frames; only the hi/lo pass's listed frames are
            // copied masked, each to its own place in the stream's second
            // workspace slot
            const bool hilo = (mode & (SVDPHAT_HILO | SVDPHAT_HILO_ALL)) && precision != SVDPHAT_FP32;
            float2* xm = hilo ? (float2*)ws_get(p, s, xbytes, 1) : nullptr;
            launch_locate(p, X, F, precision, mode, doa, power, yhat, margin, y_opt, s, nullptr, 0, mask, xm);
            return;
        }
        // otherwise the masked frames are written whole into that slot, which
        // holds them for the whole call (the power of Algorithm 1 step 4
        // reads them last)
        float2* xm = (float2*)ws_get(p, s, xbytes, 1);
        launch_mask(p, (const float2*)X, F, mask, xm, s);
        launch_locate(p, xm, F, precision, mode, doa, power, yhat, margin, y_opt, s);
    });
}

int svdphat_srp_locate(svdphat_plan* p, const void* X, int64_t F, int32_t* doa, float* power, float* y_opt,
                       void* stream) {
    return guarded([&] {
        SP_REQUIRE(p, SVDPHAT_E_INVAL, "NULL plan");
        SP_REQUIRE(p->Wfr != nullptr, SVDPHAT_E_UNSUPPORTED, "plan was created without SVDPHAT_KEEP_W");
        SP_REQUIRE(F >= 0 && F < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "F out of range");
        if (F == 0) return;
        SP_REQUIRE(X && doa && power, SVDPHAT_E_INVAL, "NULL X, doa or power");
        SP_HIP(hipSetDevice(p->device));
        launch_srp(p, X, F, doa, power, y_opt, (hipStream_t)stream);
    });
}

void svdphat_plan_destroy(svdphat_plan* p) { free_plan(p); }

int svdphat_ragged_create(svdphat_plan* const* plans, int32_t n, const int64_t* max_frames, uint32_t flags,
                          const char* tune_cache, svdphat_ragged** out) {
    return guarded([&] {
        SP_REQUIRE(out != nullptr, SVDPHAT_E_INVAL, "out is NULL");
        *out = nullptr;
        SP_REQUIRE(plans && max_frames && n >= 1, SVDPHAT_E_INVAL, "need n >= 1 plans and their frame counts");
        SP_REQUIRE((flags & ~(uint32_t)SVDPHAT_RAGGED_TUNE) == 0, SVDPHAT_E_INVAL, "unknown flags");
        for (int i = 0; i < n; ++i) {
            SP_REQUIRE(plans[i] != nullptr, SVDPHAT_E_INVAL, "NULL plan " + std::to_string(i));
            SP_REQUIRE(max_frames[i] >= 1 && max_frames[i] < ((int64_t)1 << 31), SVDPHAT_E_INVAL,
                       "max_frames out of range for array " + std::to_string(i));
            SP_REQUIRE(plans[i]->device == plans[0]->device, SVDPHAT_E_INVAL, "plans on different devices");
            SP_REQUIRE(!(plans[i]->flags & SVDPHAT_NO_DEDUP), SVDPHAT_E_UNSUPPORTED,
                       "ragged batches need plans with one scored row per class");
        }
        SP_HIP(hipSetDevice(plans[0]->device));
        svdphat_ragged* r = ragged_new(plans, n, max_frames);
        try {
            ragged_build(r, flags, tune_cache);
        } catch (...) {
            ragged_destroy(r);
            throw;
        }
        *out = r;
    });
}

int svdphat_ragged_locate(svdphat_ragged* r, const void* const* X, const int64_t* F, int32_t* const* doa,
                          float* const* power, int32_t precision, void* stream) {
    return guarded([&] {
        SP_REQUIRE(r && X && F && doa && power, SVDPHAT_E_INVAL, "NULL argument");
        SP_REQUIRE(precision == SVDPHAT_FP16, SVDPHAT_E_UNSUPPORTED,
                   "ragged batches run FP16 MFMA with FP32 rescoring only");
        ragged_locate(r, X, F, doa, power, (hipStream_t)stream);
    });
}

int svdphat_ragged_info(const svdphat_ragged* r, int64_t* tuned, int64_t* from_cache) {
    return guarded([&] {
        SP_REQUIRE(r, SVDPHAT_E_INVAL, "NULL ragged batch");
        ragged_stats(r, tuned, from_cache);
    });
}

void svdphat_ragged_destroy(svdphat_ragged* r) {
    if (r) ragged_destroy(r);
}

int svdphat_proposal_create(svdphat_plan* fine, const double* coarse_xyz, int32_t C, int32_t hidden, uint64_t seed,
                            svdphat_proposal** out) {
    return guarded([&] {
        SP_REQUIRE(out != nullptr, SVDPHAT_E_INVAL, "out is NULL");
        *out = nullptr;
        SP_REQUIRE(fine && coarse_xyz, SVDPHAT_E_INVAL, "NULL plan or coarse grid");
        SP_REQUIRE(C >= 1 && C <= 1024, SVDPHAT_E_INVAL, "C must be in [1, 1024]");
        SP_REQUIRE(hidden >= 64 && hidden <= 1024 && hidden % 64 == 0, SVDPHAT_E_INVAL,
                   "hidden must be a multiple of 64 in [64, 1024]");
        SP_REQUIRE(!(fine->flags & SVDPHAT_NO_DEDUP), SVDPHAT_E_UNSUPPORTED,
                   "the proposal needs a plan with one scored row per class");
        SP_HIP(hipSetDevice(fine->device));
        svdphat_proposal* pr = new svdphat_proposal();
        pr->plan = fine;
        try {
            proposal_build(pr, coarse_xyz, C, hidden, seed);
        } catch (...) {
            proposal_free(pr);
            throw;
        }
        *out = pr;
    });
}

int svdphat_proposal_train_step(svdphat_proposal* pr, const void* X, int64_t F, float lr, float* loss_host,
                                void* stream) {
    return guarded([&] {
        SP_REQUIRE(pr && X && F >= 1 && F < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "bad proposal, X or F");
        SP_REQUIRE(std::isfinite(lr) && lr > 0.f, SVDPHAT_E_INVAL, "lr must be > 0");
        SP_HIP(hipSetDevice(pr->plan->device));
        const float l = proposal_train_step(pr, (const float2*)X, F, lr, (hipStream_t)stream);
        if (loss_host) *loss_host = l;
    });
}

int svdphat_proposal_locate(svdphat_proposal* pr, const void* X, int64_t F, int32_t topk, float conf_min,
                            int32_t* doa, float* power, uint8_t* fell_back, void* stream) {
    return guarded([&] {
        SP_REQUIRE(pr, SVDPHAT_E_INVAL, "NULL proposal");
        SP_REQUIRE(F >= 0 && F < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "F out of range");
        SP_REQUIRE(topk >= 1 && topk <= pr->C, SVDPHAT_E_INVAL, "topk must be in [1, C]");
        if (F == 0) return;
        SP_REQUIRE(X && doa && power && fell_back, SVDPHAT_E_INVAL, "NULL X or output");
        SP_HIP(hipSetDevice(pr->plan->device));
        proposal_locate(pr, (const float2*)X, F, topk, conf_min, doa, power, fell_back, (hipStream_t)stream);
    });
}

int svdphat_proposal_params(svdphat_proposal* pr, float* host, int64_t n, int32_t set) {
    return guarded([&] {
        SP_REQUIRE(pr, SVDPHAT_E_INVAL, "NULL proposal");
        const int64_t need = proposal_nparams(pr);
        if (!host) {
            SP_REQUIRE(n == 0, SVDPHAT_E_INVAL, "NULL buffer");
            return;
        }
        SP_REQUIRE(n == need, SVDPHAT_E_INVAL, "parameter count must be " + std::to_string(need));
        SP_HIP(hipSetDevice(pr->plan->device));
        proposal_params(pr, host, set != 0);
    });
}

int64_t svdphat_proposal_nparams(const svdphat_proposal* pr) { return pr ? proposal_nparams(pr) : -1; }

int svdphat_proposal_grad(svdphat_proposal* pr, const float* features, const int32_t* labels, int64_t F,
                          float* grad, float* loss_host) {
    return guarded([&] {
        SP_REQUIRE(pr && features && labels && grad && F >= 1, SVDPHAT_E_INVAL, "NULL argument or F < 1");
        for (int64_t f = 0; f < F; ++f)
            SP_REQUIRE(labels[f] >= 0 && labels[f] < pr->C, SVDPHAT_E_INVAL, "label out of range");
        SP_HIP(hipSetDevice(pr->plan->device));
        const float l = proposal_grad(pr, features, labels, F, grad);
        if (loss_host) *loss_host = l;
    });
}

int svdphat_proposal_save(const svdphat_proposal* pr, const char* path) {
    return guarded([&] {
        SP_REQUIRE(pr && path, SVDPHAT_E_INVAL, "NULL proposal or path");
        SP_HIP(hipSetDevice(pr->plan->device));
        proposal_save(pr, path);
    });
}

int svdphat_proposal_load(svdphat_plan* fine, const char* path, svdphat_proposal** out) {
    return guarded([&] {
        SP_REQUIRE(out != nullptr, SVDPHAT_E_INVAL, "out is NULL");
        *out = nullptr;
        SP_REQUIRE(fine && path, SVDPHAT_E_INVAL, "NULL plan or path");
        SP_REQUIRE(!(fine->flags & SVDPHAT_NO_DEDUP), SVDPHAT_E_UNSUPPORTED,
                   "the proposal needs a plan with one scored row per class");
        *out = proposal_load(fine, path);
    });
}

int svdphat_proposal_features(svdphat_proposal* pr, const void* X, int64_t F, float* feat, void* stream) {
    return guarded([&] {
        SP_REQUIRE(pr, SVDPHAT_E_INVAL, "NULL proposal");
        SP_REQUIRE(F >= 0 && F < ((int64_t)1 << 31), SVDPHAT_E_INVAL, "F out of range");
        if (F == 0) return;
        SP_REQUIRE(X && feat, SVDPHAT_E_INVAL, "NULL X or feat");
        SP_HIP(hipSetDevice(pr->plan->device));
        proposal_features(pr, (const float2*)X, F, feat, (hipStream_t)stream);
    });
}

int svdphat_proposal_apply_grad(svdphat_proposal* pr, const float* grad, int64_t n, float lr) {
    return guarded([&] {
        SP_REQUIRE(pr && grad, SVDPHAT_E_INVAL, "NULL proposal or gradient");
        SP_REQUIRE(n == proposal_nparams(pr), SVDPHAT_E_INVAL,
                   "gradient length must be " + std::to_string(proposal_nparams(pr)));
        SP_REQUIRE(std::isfinite(lr) && lr > 0.f, SVDPHAT_E_INVAL, "lr must be > 0");
        SP_HIP(hipSetDevice(pr->plan->device));
        proposal_apply_grad(pr, grad, lr);
    });
}

int svdphat_proposal_cells(const svdphat_proposal* pr, int32_t* cell_of_direction) {
    return guarded([&] {
        SP_REQUIRE(pr && cell_of_direction, SVDPHAT_E_INVAL, "NULL argument");
        std::memcpy(cell_of_direction, pr->cell_of_dir.data(), pr->cell_of_dir.size() * sizeof(int32_t));
    });
}

void svdphat_proposal_destroy(svdphat_proposal* pr) { proposal_free(pr); }

int svdphat_timing_enable(int enable) {
    return guarded([&] {
        std::lock_guard<std::mutex> lk(timing().mu);
        timing().on = (enable & 1) != 0;
        timing().counts = (enable & 2) != 0;
    });
}

int svdphat_timing_reset(void) {
    return guarded([&] {
        std::lock_guard<std::mutex> lk(timing().mu);
        timing().t.clear();
    });
}

int svdphat_timing_read(int32_t index, char* name, int32_t name_len, double* total_ms, int64_t* launches) {
    return guarded([&] {
        std::lock_guard<std::mutex> lk(timing().mu);
        SP_REQUIRE(index >= 0, SVDPHAT_E_INVAL, "negative index");
        if (index >= (int32_t)timing().t.size()) fail(SVDPHAT_E_INVAL, "index past the last timed kernel");
        auto it = timing().t.begin();
        std::advance(it, index);
        if (name && name_len > 0) {
            std::strncpy(name, it->first.c_str(), (size_t)name_len - 1);
            name[name_len - 1] = 0;
        }
        if (total_ms) *total_ms = it->second.first;
        if (launches) *launches = it->second.second;
    });
}

int svdphat_peaks(const float* y, int64_t F, int32_t Q, int64_t ldy, const float* dirs, int32_t n, float cos_sep,
                  int32_t* idx, float* val, void* stream) {
    return guarded([&] {
        SP_REQUIRE(F >= 0 && F < ((int64_t)1 << 31) && Q >= 1 && ldy >= Q, SVDPHAT_E_INVAL,
                   "need 0 <= F < 2^31, Q >= 1, ldy >= Q");
        SP_REQUIRE(n >= 1 && n <= peaks_max(), SVDPHAT_E_INVAL, "n must be in [1, " + std::to_string(peaks_max()) + "]");
        if (F == 0) return;
        SP_REQUIRE(y && dirs && idx && val, SVDPHAT_E_INVAL, "NULL y, dirs, idx or val");
        require_device();
        launch_peaks(y, F, Q, ldy, dirs, n, cos_sep, idx, val, (hipStream_t)stream);
        SP_HIP(hipGetLastError());
    });
}

int64_t svdphat_stft_frames(int64_t T, int32_t N, int32_t hop) {
    if (T < 0 || N < 1 || hop < 1) return -1;
    return T < N ? 0 : 1 + (T - N) / hop;
}

int svdphat_stft(const float* pcm, int32_t M, int64_t T, int64_t ld, int32_t N, int32_t hop, void* X,
                 void* stream) {
    return guarded([&] {
        SP_REQUIRE(M >= 1 && T >= 0 && ld >= T && hop >= 1, SVDPHAT_E_INVAL, "need M >= 1, 0 <= T <= ld, hop >= 1");
        SP_REQUIRE(N >= 16 && N <= 2048 && (N & (N - 1)) == 0, SVDPHAT_E_UNSUPPORTED,
                   "N must be a power of two in [16, 2048]");
        const int64_t F = svdphat_stft_frames(T, N, hop);
        SP_REQUIRE(F * M < ((int64_t)1 << 40), SVDPHAT_E_INVAL, "too many frames");
        if (F == 0) return;
        SP_REQUIRE(pcm && X, SVDPHAT_E_INVAL, "NULL pcm or X");
        require_device();
        int dev = 0;
        SP_HIP(hipGetDevice(&dev));
        launch_stft(pcm, M, ld, N, hop, (float2*)X, F, dev, (hipStream_t)stream);
        SP_HIP(hipGetLastError());
    });
}

int svdphat_sync(void* stream) {
    return guarded([&] {
        require_device();
        SP_HIP(hipStreamSynchronize((hipStream_t)stream));
        SP_HIP(hipGetLastError());
    });
}

}  // extern "C"
