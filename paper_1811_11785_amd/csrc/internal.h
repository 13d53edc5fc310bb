// Internal declarations of the SVD-PHAT gfx950 library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/svdphat.h"

namespace svdphat {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};
void set_last_error(const std::string& msg);
[[noreturn]] void fail(int code, const std::string& msg);
#define SP_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            ::svdphat::fail(SVDPHAT_E_DEVICE, std::string(#call) + ": " +         \
                                                  hipGetErrorString(e_));         \
    } while (0)
#define SP_REQUIRE(cond, code, msg)                                               \
    do {                                                                          \
        if (!(cond)) ::svdphat::fail((code), (msg));                              \
    } while (0)

// ------------------------------------------------------------ MFMA types
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Element-type traits for the three MFMA operand types.  KSTEP is the
// reduction depth of one v_mfma_f32_16x16xKSTEP instruction and EPL the
// number of operand elements each of the 64 lanes holds.
template <typename T> struct Mf;
template <> struct Mf<float> {
    static constexpr int KSTEP = 4, EPL = 1;
};
template <> struct Mf<_Float16> {
    static constexpr int KSTEP = 32, EPL = 8;
};
template <> struct Mf<__bf16> {
    static constexpr int KSTEP = 32, EPL = 8;
};

enum Prec { P_FP32 = 0, P_BF16 = 1, P_FP16 = 2 };

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }
inline int64_t round_up64(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Rows of the reduced search are scored in tiles of this many directions;
// the per-tile maximum is the unit of the candidate set that is rescored.
constexpr int QTILE = 64;

// Layout of the stacked-real GEMM1 operand for one element type: the
// reduction axis (bins x pairs x {re, im}, bin-major) is cut into chunks of
// BB bins; chunk width CW = round_up(BB * 2P, KSTEP) stacked values.
// Chunks of BB bins must fit the GEMM1 workgroup's item budget: 64 frames x
// BB <= 256 x (3 items per thread for M <= 8, 1 for M <= 16).
constexpr int G1_MAX_ITEMS8 = 768, G1_MAX_ITEMS16 = 256;
struct G1Layout {
    int BB = 0;       // bins per chunk
    int CW = 0;       // stacked values per chunk (padded)
    int nch = 0;      // chunks
    int ks_chunk = 0; // MFMA k-steps per chunk
    int64_t elems = 0;  // packed elements of A (all row blocks)
};

// Arguments of the per-frame search kernel (rescoring, margin, power).
struct FinalArgs {
    const float2* X;
    int M, P, B;
    const float* pmax;      // [frame][pstride] tile maxima
    int64_t pstride;
    int ntile, ncls;
    const float* z32;       // [pos][Rp] z used for rescoring
    const float* zpart;     // or, when set: z = sum of zp_n partials zpart[s * zp_stride + pos * Rp]
    int zp_n;
    int64_t zp_stride;
    const float* z32_first; // [F][Rp] z of the first pass (second pass only)
    const float* znorm1;    // [F] ||z|| of the first pass
    int Rp;
    float ecoef;            // eps_t = kappa_t * (ecoef ||z1|| + 1.01 ||z - z1||)
    int rescore;
    const float* U32T;      // [ntile][Rp/4][64][4]
    const float* tkappa;    // [ntile] max ||U_q|| in the tile
    const float* sig;       // [Rp] singular value of each stacked row of Z
    const int32_t* rows;    // [ncls] direction of each scored row
    const int32_t* rep;     // [Q] class representative
    const float* tauN;      // [Q][P] tau / N
    const float* tauM;      // [Q][M] per-microphone tau / N
    const int32_t* rowcls;  // [ncls_pad] class of each scored row
    float usig_max;         // max ||U_q sigma|| (cheap bound of the hi/lo test)
    int64_t nfr;
    const int* flist;       // second pass: frames to redo
    const int* fcount;
    int32_t* doa;
    float* power;
    float* yhat;
    float* margin;
    float hilo_k;           // hi/lo trigger: y1 - y2 < hilo_k u ||(U_q1 - U_q2) sigma||
    int hilo_all;           // every frame into the hi/lo list
    float u;                // unit roundoff of the GEMM1 operands
    int* hlist;
    int* hcount;
    unsigned long long* stats;  // optional: [0] tiles rescored, [1] frames queued for hi/lo
};

// Everything the four search stages need for one array of a ragged batch
// (device-resident; one entry per array).
struct RDesc {
    // GEMM1
    const float2* X;
    int64_t F;
    int M, P, B;
    const void* A;
    int nRB, BB, CW, nch, cps, nsplit, Rp;
    float* zpart;
    int64_t zstride;
    // Z prep
    float* z32;
    void* zfrag;
    float* zsc;
    float* zn;
    // GEMM2
    const void* U;
    int KSn, ncls, ntile, fch;
    float uinv;
    float* pmax;
    int64_t pstride;
    // search
    FinalArgs fin;
};

// One grouped launch: a device work list of (array, x, y, z) items run by one
// kernel instance (template class `cls`) of stage `stage`.
struct GroupLaunch {
    int stage = 0;     // 0 GEMM1, 1 Z prep, 2 GEMM2, 3 search
    int cls = 0;       // template class within the stage
    int4* work = nullptr;
    int nwork = 0;
    size_t lds = 0;
};
void launch_grouped(const GroupLaunch& g, const RDesc* d, hipStream_t s);
int g1_nrb_class(int nRB);
size_t g1_lds_bytes(int NRB, int CW);
void g1_split(const svdphat_plan* p, int64_t F, int want, int* nsplit, int* cps);
// streamed GEMM1 (16-bit operands, 6 to 8 microphones, up to 8 row blocks):
// the chunk it needs (false = not available); its schedule over F frames
// (false = not applicable to this plan and precision): G persistent
// workgroups over U = frame tiles x chunks units, `slots` partial sums per
// frame; and its launcher
bool g1s_layout(int M, int nRB, int kstep, int* CW, int* BB);
int cu_count(int device);  // compute units of a device (cached)
struct G1Sched {
    int G = 0;
    int64_t U = 0;
    int nch = 0;
    int slots = 0;
};
bool g1s_sched(int prec, const svdphat_plan* p, int64_t F, G1Sched* out);
// mask: NULL, or uint8 [F][B] (0 drops the frame's bin from the PHAT tiles)
void launch_g1_streamed(int prec, const svdphat_plan* p, const G1Sched& sc, const float2* X, int64_t F, float* zpart,
                        int64_t zstride, hipStream_t s, const uint8_t* mask = nullptr);
// times one GEMM1 + Z prep (nsplit) and one GEMM2 (fch) of plan p on F
// synthetic frames in FP16; returns microseconds
void proposal_build(svdphat_proposal* pr, const double* coarse, int C, int H, uint64_t seed);
float proposal_train_step(svdphat_proposal* pr, const float2* X, int64_t F, float lr, hipStream_t s);
void proposal_locate(svdphat_proposal* pr, const float2* X, int64_t F, int topk, float conf_min, int32_t* doa,
                     float* power, uint8_t* fell, hipStream_t s);
int64_t proposal_nparams(const svdphat_proposal* pr);
void proposal_params(svdphat_proposal* pr, float* host, bool set);
// parameters, Adam moments (host layout of proposal_params) and step count
void proposal_state(svdphat_proposal* pr, float* params, float* m, float* v, int64_t* step, bool set);
float proposal_grad(svdphat_proposal* pr, const float* feat, const int32_t* lab, int64_t F, float* grad);
void proposal_features(svdphat_proposal* pr, const float2* X, int64_t F, float* feat, hipStream_t s);
void proposal_apply_grad(svdphat_proposal* pr, const float* grad, float lr);
void proposal_free(svdphat_proposal* pr);
int64_t front_zpart_floats(const svdphat_plan* p, int64_t F);
void front_fp16(svdphat_plan* p, const float2* X, int64_t F, float* zpart, float* z32, _Float16* zfrag, float* zsc,
                float* zn, hipStream_t s);
void back_list_fp16(svdphat_plan* p, const float2* X, int64_t Fmax, const int* flist, const int* fcount,
                    const _Float16* zfrag, const float* zsc, const float* z32pos, const float* zn_frame,
                    float* pmax, int32_t* doa, float* power, float* margin, hipStream_t s);
void tune_time(svdphat_plan* p, int64_t F, int nsplit, int fch, double* us_g1, double* us_g2, hipStream_t s);

// Device tables of one set of scored rows (see pack_rows in plan.hip).
struct ScoreRows {
    void* Ufr[3] = {nullptr, nullptr, nullptr};  // GEMM2 operand per precision
    float uscale[3] = {1.f, 1.f, 1.f};           // exact power-of-two scale per precision
    float* U32T = nullptr;                       // [ntile][Rp/4][QTILE][4] FP32 rescoring rows
    float* tkappa = nullptr;                     // [ntile] largest row norm of each tile
    float usig_max = 0.f;                        // max ||row sigma|| over the rows
};

struct Workspace {
    int64_t cap_frames = 0;
    void* buf = nullptr;
    size_t bytes = 0;
};

}  // namespace svdphat

struct svdphat_plan {
    int device = 0;
    int M = 0, P = 0, B = 0, L = 0, Q = 0, N = 0, K = 0, K_paper = 0;
    double fs = 0, c = 0, delta = 0;
    uint32_t flags = 0;
    double residual = 0, fro2 = 0, kappa = 0;  // kappa = max_q ||U_q||
    std::vector<double> tau;     // [Q][P] delays in samples, eq. (2)
    std::vector<double> tauM;    // [Q][M] per-microphone delays in samples
    std::vector<double> grid;    // [Q][3] unit directions
    std::vector<double> mics_in, grid_in;  // the inputs as given (M x 3, Q x 3)
    std::vector<int32_t> rep;    // [Q] class representative
    std::vector<int32_t> rows;   // [ncls] direction index of each scored row
    std::vector<double> sigma;   // all singular values, descending
    std::vector<double> U, V;    // FP64 factors, complex interleaved [Q][K], [L][K] (eq. (7) order)
    int ncls = 0;                // scored rows
    int ncls_pad = 0;            // rows padded to a multiple of 256
    int R = 0;                   // 2K stacked rows of Z
    int Rp = 0;                  // R padded to 32
    svdphat::G1Layout g1[3];     // per precision
    int64_t device_bytes = 0;

    // device operands (all owned)
    void* A[3] = {nullptr, nullptr, nullptr};    // GEMM1 operand per precision
    void* Alo[3] = {nullptr, nullptr, nullptr};  // low parts (16-bit only)
    // streamed GEMM1 in two row-group passes (8 to 12 row blocks of Z, 6 to
    // 8 microphones, 16-bit operands): A of row blocks [0, as_split) and
    // [as_split, Rp / 16) in the streamed chunk layout g1s; as_split = 0: none
    void* As[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
    int as_split = 0;
    svdphat::G1Layout g1s[3];
    svdphat::ScoreRows sr[2];                    // scored rows: [0] U (eq. (14)), [1] U / ||U sigma|| (eq. (15))
    float* A32T = nullptr;                       // [B P 2][Rp] FP32 A = S V^H, transposed (GEMV form)
    float* d_sig = nullptr;                      // [Rp] singular value of each stacked row of Z
    int32_t* d_rows = nullptr;                   // [ncls] direction index of row
    int32_t* d_rep = nullptr;                    // [Q]
    int32_t* d_rowof = nullptr;                  // [Q] scored row holding each direction's class
    float* d_tauN = nullptr;                     // [ncls][P] tau / N (rows of the search)
    float* d_tauN_all = nullptr;                 // [Q][P] tau / N
    float* d_tauM_all = nullptr;                 // [Q][M] per-microphone tau / N
    int32_t* d_rowcls = nullptr;                 // [ncls_pad] class of each scored row
    int8_t* d_pi = nullptr;                      // [P] first mic of pair
    int8_t* d_pj = nullptr;                      // [P] second mic of pair
    float* Wfr = nullptr;                        // plain form operand (KEEP_W)
    int Wrows_pad = 0, Wks = 0;                  // rows padded to 128, k-steps of 4

    std::mutex ws_mu;
    std::map<std::pair<void*, int>, svdphat::Workspace> ws;  // per (stream, slot)
    std::vector<void*> ws_retired;           // grown-out workspaces (freed with the plan)
};

// Learned proposal state (see the proposal calls of the ABI).
struct svdphat_proposal {
    svdphat_plan* plan = nullptr;
    int C = 0, Cp = 0, H = 0, D = 0, D0 = 0;  // cells, padded cells, hidden, input (2K), padded input (Rp)
    std::vector<int32_t> cell_of_dir;         // [Q]
    std::vector<double> coarse;               // [C][3] coarse directions as given
    int32_t* d_cell_of_dir = nullptr;         // [Q]
    int32_t* d_cell_start = nullptr;          // [C + 1] CSR over the scored rows in cell order
    int32_t* d_cell_dir = nullptr;            // [ncls] direction of each row in cell order
    float* d_U32C = nullptr;                  // [ncls][Rp] FP32 stacked U rows in cell order
    // parameters: FP32 master, Adam moments, FP16 copies and transposes
    int64_t off[6] = {0, 0, 0, 0, 0, 0};     // W1 b1 W2 b2 W3 b3 inside the flat arrays
    int64_t nparam = 0;
    float* P = nullptr;
    float* Mm = nullptr;
    float* Vv = nullptr;
    _Float16* Wh[3] = {nullptr, nullptr, nullptr};  // [out][in]
    _Float16* Wt[3] = {nullptr, nullptr, nullptr};  // [in][out]
    // Wh in MFMA B-fragment order for inference (one contiguous 1 KB per
    // fragment load), repacked from Wh when wf_ok is false
    _Float16* Wf[3] = {nullptr, nullptr, nullptr};
    bool wf_ok = false;
    int64_t step = 0;
    // workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<void*> ws_retired;  // grown-out workspaces (freed with the proposal)
    int* d_count = nullptr;  // [8]: fallback count, then two 64-bit event counters
};

namespace svdphat {
// Row stride (floats) of the frame-major tile maxima: tiles padded to 32.
inline int pmax_stride(const svdphat_plan* p) { return round_up(p->ncls_pad / QTILE, 32); }
// launchers
// scratch: a caller-provided device buffer of scratch_bytes for the call's
// intermediate results (nullptr: the plan's workspace of stream s)
// mask: NULL, or uint8 [F][B] applied inside the kernels (only where
// mask_fused holds); xm: device float2 [F][M][B] that receives the masked
// copies of the hi/lo pass's frames (needed with SVDPHAT_HILO*)
void launch_locate(svdphat_plan* p, const void* X, int64_t F, int prec, uint32_t mode,
                   int32_t* doa, float* power, float* yhat, float* margin, float* y_opt,
                   hipStream_t s, void* scratch = nullptr, size_t scratch_bytes = 0,
                   const uint8_t* mask = nullptr, float2* xm = nullptr);
// whether launch_locate takes a mask for F frames in precision prec (the
// streamed GEMM1 serves the call)
bool mask_fused(const svdphat_plan* p, int64_t F, int prec, bool y_opt);
void launch_srp(svdphat_plan* p, const void* X, int64_t F, int32_t* doa, float* power,
                float* y_opt, hipStream_t s);
void build_w_fp32_frags(svdphat_plan* p);
// Algorithm 1 offline: geometry, classes, then (unless `factored`: sigma, U,
// V, K, K_paper, fro2 and residual already set, e.g. from a saved plan) the
// truncated SVD, then the packing of the device operands
void build_plan(svdphat_plan* p, const double* mics, const double* grid, bool factored);
// persistence (persist.cpp)
void plan_save(const svdphat_plan* p, const char* path);
svdphat_plan* plan_load(const char* path, void (*destroy)(svdphat_plan*));
uint64_t plan_input_hash(const double* mics, int M, const double* grid, int Q, double fs, double c, int N,
                         double delta, uint32_t flags);
void proposal_save(const svdphat_proposal* pr, const char* path);
svdphat_proposal* proposal_load(svdphat_plan* fine, const char* path);
// small batches in GEMV form (frame1.hip): at most GV_MAX_FRAMES frames,
// FP32 projections, exact FP32 argmax; scratch of gv_scratch_bytes()
constexpr int GV_MAX_FRAMES = 16;
bool gv_applicable(const svdphat_plan* p, int64_t F);
int gv_score_groups(const svdphat_plan* p);
size_t gv_scratch_bytes(const svdphat_plan* p, int64_t F);
void launch_gv(svdphat_plan* p, const ScoreRows& sr, const float2* X, int64_t F, int32_t* doa, float* power,
               float* yhat, float* margin, void* ws, hipStream_t s);
// the plan's workspace `slot` of stream s, grown to at least `bytes`
void* ws_get(svdphat_plan* p, hipStream_t s, size_t bytes, int slot = 0);
// binary time-frequency mask (mask.hip): xm = X where mask[f][b] != 0, else 0
void launch_mask(const svdphat_plan* p, const float2* X, int64_t F, const uint8_t* mask, float2* xm, hipStream_t s);
// the same for the frames flist[0 .. *fcount) only, each at its own place in xm
void launch_mask_list(const svdphat_plan* p, const float2* X, const uint8_t* mask, const int* flist,
                      const int* fcount, float2* xm, hipStream_t s);
// zero `bytes` (a multiple of 4) of device memory on stream s with a kernel,
// so that a caller capturing the stream into a graph records a kernel node
void zero_async(void* p, size_t bytes, hipStream_t s);
// Fault injection for tests: the environment variable SVDPHAT_FAULT holds a
// comma-separated list of faults to force ("alloc": every device allocation
// of the library fails; "eig": the eigensolver reports no convergence).
bool fault_forced(const char* kind);
// Every device allocation of the library: hipMalloc, or hipErrorOutOfMemory
// when the "alloc" fault is forced.  dev_alloc fails with SVDPHAT_E_NOMEM.
hipError_t dev_malloc(void** p, size_t bytes);
void dev_alloc(void** p, size_t bytes, const char* what);
// several peaks per frame (peaks.hip)
int peaks_max();
void launch_peaks(const float* y, int64_t F, int Q, int64_t ldy, const float* dirs, int n, float cos_sep,
                  int32_t* idx, float* val, hipStream_t s);
// STFT front end (stft.hip): F frames of M signals into X [F][M][N/2+1]
size_t stft_lds_bytes(int N);
void launch_stft(const float* pcm, int M, int64_t ld, int N, int hop, float2* X, int64_t F, int device,
                 hipStream_t s);
svdphat_ragged* ragged_new(svdphat_plan* const* plans, int n, const int64_t* maxF);
void ragged_build(svdphat_ragged* r, uint32_t flags, const char* cache_path);
void ragged_locate(svdphat_ragged* r, const void* const* X, const int64_t* F, int32_t* const* doa,
                   float* const* power, hipStream_t s);
void ragged_destroy(svdphat_ragged* r);
void ragged_stats(const svdphat_ragged* r, int64_t* tuned, int64_t* cached);

// Per-kernel timing (instrumentation): while enabled, each launch is
// bracketed by HIP events on its stream; `flush` waits for them and adds the
// elapsed times to a process-wide table keyed by kernel name.
bool timing_on();
bool counting_on();
// adds an event count to the timing table (entries named count:*)
void timing_count(const char* name, double count, int64_t calls);
struct KernelTimer {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
        hipStream_t s;
    };
    hipStream_t s;
    std::vector<Rec> recs;
    explicit KernelTimer(hipStream_t st) : s(st) {}
    // times the work enqueued on stream `on` (default: the timer's stream)
    // between begin() and the next end()
    void begin(const char* name, hipStream_t on = nullptr);
    void end();
    void flush();
    ~KernelTimer();
};
}  // namespace svdphat
