// Saved plans and proposals.  Algorithm 1 (Section 3) computes the offline
// products once per array and grid; a saved plan keeps the inputs and the
// truncated SVD (sigma, U, V, K), and loading it repeats only the host
// geometry and the packing of the device operands, so a loaded plan's device
// buffers, and every result computed from them, are identical to the
// original's.  A saved proposal keeps the coarse directions, the FP32
// parameters, the Adam moments and the step count.
//
// Both formats are little-endian binary:
//   plan      "SVDPHPLN", u32 version 1, i32 M, Q, N, K, K_paper, u32 flags,
//             f64 fs, c, delta, fro2, residual, u64 input hash, u64 n_sigma,
//             f64 mics[3M], grid[3Q] (as given), sigma[n_sigma], U[2QK],
//             V[2LK] (rows in the library's bin-major order), u64 checksum
//   proposal  "SVDPHPRP", u32 version 1, u64 input hash of the fine plan,
//             i32 C, H, D (= 2K), i32 0, i64 step, f64 coarse[3C],
//             f32 params[n], m[n], v[n] (layout of svdphat_proposal_params),
//             u64 checksum
// The checksum and the input hash are 64-bit FNV-1a (Fowler, Noll, Vo) of
// the bytes before the checksum and of (M, Q, N, flags, fs, c, delta, mics,
// grid) respectively.
#include "internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>

namespace svdphat {
namespace {

constexpr char PLAN_MAGIC[8] = {'S', 'V', 'D', 'P', 'H', 'P', 'L', 'N'};
constexpr char PROP_MAGIC[8] = {'S', 'V', 'D', 'P', 'H', 'P', 'R', 'P'};
constexpr uint32_t VERSION = 1;

struct Fnv {
    uint64_t h = 14695981039346656037ull;
    void add(const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
};

struct Writer {
    std::vector<unsigned char> buf;
    template <typename T>
    void put(const T& v) {
        const unsigned char* b = (const unsigned char*)&v;
        buf.insert(buf.end(), b, b + sizeof(T));
    }
    template <typename T>
    void put_n(const T* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        buf.insert(buf.end(), b, b + n * sizeof(T));
    }
    void finish(const char* path) {
        Fnv f;
        f.add(buf.data(), buf.size());
        put(f.h);
        std::unique_ptr<FILE, int (*)(FILE*)> fp(std::fopen(path, "wb"), std::fclose);
        SP_REQUIRE(fp != nullptr, SVDPHAT_E_IO, std::string("cannot open ") + path + " for writing");
        SP_REQUIRE(std::fwrite(buf.data(), 1, buf.size(), fp.get()) == buf.size(), SVDPHAT_E_IO,
                   std::string("cannot write ") + path);
        SP_REQUIRE(std::fflush(fp.get()) == 0, SVDPHAT_E_IO, std::string("cannot write ") + path);
    }
};

struct Reader {
    std::vector<unsigned char> buf;
    size_t pos = 0;
    explicit Reader(const char* path) {
        std::unique_ptr<FILE, int (*)(FILE*)> fp(std::fopen(path, "rb"), std::fclose);
        SP_REQUIRE(fp != nullptr, SVDPHAT_E_IO, std::string("cannot open ") + path);
        unsigned char tmp[1 << 16];
        size_t n;
        while ((n = std::fread(tmp, 1, sizeof(tmp), fp.get())) > 0) buf.insert(buf.end(), tmp, tmp + n);
        SP_REQUIRE(!std::ferror(fp.get()), SVDPHAT_E_IO, std::string("cannot read ") + path);
        SP_REQUIRE(buf.size() >= 8 + 4 + 8, SVDPHAT_E_INVAL, "file too short");
        uint64_t sum;
        std::memcpy(&sum, buf.data() + buf.size() - 8, 8);
        Fnv f;
        f.add(buf.data(), buf.size() - 8);
        SP_REQUIRE(f.h == sum, SVDPHAT_E_INVAL, "checksum mismatch: the file is damaged");
        buf.resize(buf.size() - 8);
    }
    template <typename T>
    T get() {
        SP_REQUIRE(pos + sizeof(T) <= buf.size(), SVDPHAT_E_INVAL, "file truncated");
        T v;
        std::memcpy(&v, buf.data() + pos, sizeof(T));
        pos += sizeof(T);
        return v;
    }
    template <typename T>
    void get_n(T* p, size_t n) {
        SP_REQUIRE(n <= (buf.size() - pos) / sizeof(T), SVDPHAT_E_INVAL, "file truncated");
        std::memcpy(p, buf.data() + pos, n * sizeof(T));
        pos += n * sizeof(T);
    }
    void magic(const char (&m)[8]) {
        char got[8];
        get_n(got, 8);
        SP_REQUIRE(std::memcmp(got, m, 8) == 0, SVDPHAT_E_INVAL, "not a saved SVD-PHAT file of this kind");
        const uint32_t v = get<uint32_t>();
        SP_REQUIRE(v == VERSION, SVDPHAT_E_INVAL, "unsupported file version " + std::to_string(v));
    }
    void end() { SP_REQUIRE(pos == buf.size(), SVDPHAT_E_INVAL, "trailing bytes in the file"); }
};

}  // namespace

uint64_t plan_input_hash(const double* mics, int M, const double* grid, int Q, double fs, double c, int N,
                         double delta, uint32_t flags) {
    Fnv f;
    const int32_t iv[3] = {M, Q, N};
    f.add(iv, sizeof(iv));
    f.add(&flags, sizeof(flags));
    const double dv[3] = {fs, c, delta};
    f.add(dv, sizeof(dv));
    f.add(mics, sizeof(double) * 3 * (size_t)M);
    f.add(grid, sizeof(double) * 3 * (size_t)Q);
    return f.h;
}

static uint64_t plan_hash(const svdphat_plan* p) {
    return plan_input_hash(p->mics_in.data(), p->M, p->grid_in.data(), p->Q, p->fs, p->c, p->N, p->delta, p->flags);
}

void plan_save(const svdphat_plan* p, const char* path) {
    Writer w;
    w.put_n(PLAN_MAGIC, 8);
    w.put(VERSION);
    const int32_t iv[5] = {p->M, p->Q, p->N, p->K, p->K_paper};
    w.put_n(iv, 5);
    w.put(p->flags);
    const double dv[5] = {p->fs, p->c, p->delta, p->fro2, p->residual};
    w.put_n(dv, 5);
    w.put(plan_hash(p));
    w.put((uint64_t)p->sigma.size());
    w.put_n(p->mics_in.data(), p->mics_in.size());
    w.put_n(p->grid_in.data(), p->grid_in.size());
    w.put_n(p->sigma.data(), p->sigma.size());
    w.put_n(p->U.data(), p->U.size());
    w.put_n(p->V.data(), p->V.size());
    w.finish(path);
}

svdphat_plan* plan_load(const char* path, void (*destroy)(svdphat_plan*)) {
    Reader r(path);
    r.magic(PLAN_MAGIC);
    int32_t iv[5];
    r.get_n(iv, 5);
    const int M = iv[0], Q = iv[1], N = iv[2], K = iv[3], Kp = iv[4];
    const uint32_t flags = r.get<uint32_t>();
    double dv[5];
    r.get_n(dv, 5);
    const uint64_t hash = r.get<uint64_t>();
    const uint64_t ns = r.get<uint64_t>();
    SP_REQUIRE(M >= 2 && M <= 16 && Q >= 1 && N >= 2 && N % 2 == 0, SVDPHAT_E_INVAL, "bad sizes in the file");
    SP_REQUIRE((flags & ~(uint32_t)(SVDPHAT_KEEP_W | SVDPHAT_NO_DEDUP)) == 0, SVDPHAT_E_INVAL, "bad flags in the file");
    const int64_t P = (int64_t)M * (M - 1) / 2, L = P * (N / 2 + 1);
    SP_REQUIRE(L < ((int64_t)1 << 30) && (int64_t)Q * L < ((int64_t)1 << 40), SVDPHAT_E_INVAL, "problem too large");
    SP_REQUIRE((int64_t)ns == std::min<int64_t>(Q, L) && K >= 1 && K <= (int64_t)ns && Kp >= 1 && Kp <= K,
               SVDPHAT_E_INVAL, "bad rank in the file");
    for (double v : dv) SP_REQUIRE(std::isfinite(v), SVDPHAT_E_INVAL, "non-finite value in the file");
    SP_REQUIRE(dv[0] > 0 && dv[1] > 0 && dv[2] > 0 && dv[2] < 1, SVDPHAT_E_INVAL, "bad fs, c or delta in the file");
    std::vector<double> mics(3 * (size_t)M), grid(3 * (size_t)Q), sigma(ns);
    r.get_n(mics.data(), mics.size());
    r.get_n(grid.data(), grid.size());
    r.get_n(sigma.data(), sigma.size());
    SP_REQUIRE(plan_input_hash(mics.data(), M, grid.data(), Q, dv[0], dv[1], N, dv[2], flags) == hash,
               SVDPHAT_E_INVAL, "input hash mismatch");
    for (int q = 0; q < Q; ++q) {
        const double* s = &grid[3 * (size_t)q];
        SP_REQUIRE(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] > 0.0, SVDPHAT_E_INVAL, "zero grid direction in the file");
    }
    std::vector<double> U(2 * (size_t)Q * K), V(2 * (size_t)L * K);
    r.get_n(U.data(), U.size());
    r.get_n(V.data(), V.size());
    r.end();
    for (int k = 0; k < K; ++k)
        SP_REQUIRE(std::isfinite(sigma[k]) && sigma[k] > 0.0, SVDPHAT_E_INVAL, "bad singular value in the file");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        fail(SVDPHAT_E_NODEV, "no HIP device available");
    }
    svdphat_plan* p = new svdphat_plan();
    try {
        SP_HIP(hipGetDevice(&p->device));
        p->M = M;
        p->Q = Q;
        p->N = N;
        p->fs = dv[0];
        p->c = dv[1];
        p->delta = dv[2];
        p->flags = flags;
        p->fro2 = dv[3];
        p->residual = dv[4];
        p->K = K;
        p->K_paper = Kp;
        p->sigma = std::move(sigma);
        p->U = std::move(U);
        p->V = std::move(V);
        build_plan(p, mics.data(), grid.data(), true);
    } catch (...) {
        destroy(p);
        throw;
    }
    return p;
}

void proposal_save(const svdphat_proposal* pr, const char* path) {
    svdphat_proposal* q = const_cast<svdphat_proposal*>(pr);
    const int64_t n = proposal_nparams(pr);
    std::vector<float> par(n), m(n), v(n);
    int64_t step = 0;
    proposal_state(q, par.data(), m.data(), v.data(), &step, false);
    Writer w;
    w.put_n(PROP_MAGIC, 8);
    w.put(VERSION);
    w.put(plan_hash(pr->plan));
    const int32_t iv[4] = {pr->C, pr->H, pr->D, 0};
    w.put_n(iv, 4);
    w.put(step);
    w.put_n(pr->coarse.data(), pr->coarse.size());
    w.put_n(par.data(), n);
    w.put_n(m.data(), n);
    w.put_n(v.data(), n);
    w.finish(path);
}

svdphat_proposal* proposal_load(svdphat_plan* fine, const char* path) {
    Reader r(path);
    r.magic(PROP_MAGIC);
    const uint64_t hash = r.get<uint64_t>();
    SP_REQUIRE(hash == plan_hash(fine), SVDPHAT_E_INVAL,
               "the proposal was saved for another plan (input hash mismatch)");
    int32_t iv[4];
    r.get_n(iv, 4);
    const int C = iv[0], H = iv[1], D = iv[2];
    SP_REQUIRE(C >= 1 && C <= 1024 && H >= 64 && H <= 1024 && H % 64 == 0 && D == 2 * fine->K, SVDPHAT_E_INVAL,
               "bad sizes in the file");
    const int64_t step = r.get<int64_t>();
    SP_REQUIRE(step >= 0, SVDPHAT_E_INVAL, "bad step count in the file");
    std::vector<double> coarse(3 * (size_t)C);
    r.get_n(coarse.data(), coarse.size());
    const int64_t n = (int64_t)H * D + H + (int64_t)H * H + H + (int64_t)C * H + C;
    std::vector<float> par(n), m(n), v(n);
    r.get_n(par.data(), n);
    r.get_n(m.data(), n);
    r.get_n(v.data(), n);
    r.end();
    SP_HIP(hipSetDevice(fine->device));
    svdphat_proposal* pr = new svdphat_proposal();
    pr->plan = fine;
    try {
        proposal_build(pr, coarse.data(), C, H, 0);
        SP_REQUIRE(proposal_nparams(pr) == n, SVDPHAT_E_INVAL, "parameter count mismatch");
        int64_t st = step;
        proposal_state(pr, par.data(), m.data(), v.data(), &st, true);
    } catch (...) {
        proposal_free(pr);
        throw;
    }
    return pr;
}

}  // namespace svdphat
