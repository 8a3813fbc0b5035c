// agn.hip -- C ABI of the MI355X light-curve generator (see include/agn.h).
//
// Host side: argument checks, workspace layout, descriptor upload, per-length
// plans and twiddle tables, and kernel launches.  Every step of the method
// runs in the kernels included below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/agn.h"
#include "common.hpp"
#include "lds_iterate.hpp"
#include "philox.hpp"
#include "spectrum.hpp"

using namespace agn;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err = "no error";

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                 \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(AGN_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

extern "C" const char* agn_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// sizes and plans
// ---------------------------------------------------------------------------
static const int64_t AGN_N_MAX = (int64_t)1 << 27;

static bool n_supported(int64_t n) {
    if (n < 2 || n > AGN_N_MAX || (n & 1)) return false;
    int64_t m = n;
    while ((m & 1) == 0) m >>= 1;
    return m == 1 || m == 3;
}

extern "C" int agn_supported_n(int64_t n) { return n_supported(n) ? 1 : 0; }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t prec_bytes(agn_precision p) { return p == AGN_FP32 ? 4 : 8; }

// Curves whose whole iteration runs in one workgroup's LDS.
static bool lds_path(int64_t n, agn_precision prec) {
    if (!n_supported(n)) return false;
    const bool three = (n % 3) == 0;
    if (prec == AGN_FP32) return three ? n <= 12288 : n <= 16384;
    return three ? n <= 12288 : n <= 8192;
}

// Keys per thread (IPT) of the LDS-resident kernels; the block has n / IPT
// threads (a power of two, at most 1024) and the FFT deals its M / R
// butterflies per pass round-robin over them (E = IPT / 2 values per thread).
static int lds_ipt(int64_t n) {
    if (n % 3 == 0) return n >= 12 ? 12 : 6;
    if (n >= 16384) return 16;
    return n >= 8 ? 8 : (int)n;
}

static FftPlan make_plan(int64_t M) {
    FftPlan pl;
    memset(&pl, 0, sizeof(pl));
    int64_t m = M;
    if (m % 3 == 0) { pl.radix[pl.npass++] = 3; m /= 3; }
    while (m > 1) {
        int r;
        if (m % 8 == 0) r = 8;
        else if (m % 4 == 0) r = 4;
        else r = 2;
        pl.radix[pl.npass++] = (uint8_t)r;
        m /= r;
    }
    return pl;
}

static size_t lds_iter_bytes(int64_t n, agn_precision prec) {
    const int nt = (int)(n / lds_ipt(n));
    return prec == AGN_FP32 ? lds_iter_layout<float>((int)n, nt, nullptr, nullptr, nullptr)
                            : lds_iter_layout<double>((int)n, nt, nullptr, nullptr, nullptr);
}

static size_t lds_prep_bytes(int64_t n) {
    const int nt = (int)(n / lds_ipt(n));
    return lds_prep_layout((int)n, nt, nullptr);
}

static int64_t spec_chunks(int64_t n) { return (n / 2 + 1 + SPEC_CHUNK - 1) / SPEC_CHUNK; }

static size_t spectrum_ws(int64_t n) {
    return align256((size_t)spec_chunks(n) * 8) + align256(8);
}

// Per-curve workspace: s64, sT, L, rank0, valid, amp, spectrum scratch.
static size_t curve_ws(int64_t n, agn_precision prec) {
    const size_t pb = prec_bytes(prec);
    size_t b = 0;
    b += align256((size_t)n * 8);          // s64
    b += align256((size_t)n * pb);         // sT
    b += align256((size_t)n * 8);          // L
    b += align256((size_t)n * 4);          // rank0
    b += align256(16);                     // valid
    b += align256((size_t)(n / 2 + 1) * pb);  // amp
    b += spectrum_ws(n);
    return b;
}

static size_t header_ws(int32_t nc) {
    return align256(sizeof(LcDesc) * (size_t)nc) + align256(sizeof(SpecDesc) * (size_t)nc);
}

// ---------------------------------------------------------------------------
// context: twiddle tables, kernel attributes, pinned staging ring
// ---------------------------------------------------------------------------
struct StageSlot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
};

struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};

struct agn_ctx {
    int device = 0;
    size_t lds_max = 65536;  // LDS bytes one workgroup may allocate
    bool prof = false;
    std::vector<ProfRec> prof_recs;
    std::mutex mu;
    std::map<std::pair<int64_t, int>, void*> tw;
    std::vector<StageSlot> ring;
    size_t ring_next = 0;
};

static const char* KERNEL_NAMES =
    "spectrum_partial,spectrum_norm,spectrum_amp,lds_prep,lds_iterate";

// Kernel timing: events recorded on the launch stream around each launch.
struct ProfScope {
    agn_ctx* ctx;
    const char* name;
    hipStream_t st;
    hipEvent_t a = nullptr;
    ProfScope(agn_ctx* c, const char* n, hipStream_t s) : ctx(c), name(n), st(s) {
        if (ctx && ctx->prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, st) == hipSuccess) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->prof_recs.push_back({name, a, b});
        }
    }
};

// cos and sin of 2 pi t / N with exact values at multiples of pi/2 and
// symmetric rounding: reduce to the first octant with integer arithmetic,
// evaluate in long double, round once.
static void cis_2pi(int64_t t, int64_t N, double* c, double* s) {
    t %= N;
    if (t < 0) t += N;
    const long double PI_2 = 1.5707963267948966192313216916397514L;
    const int64_t q = (4 * t) / N;
    const int64_t r = 4 * t - q * N;  // angle within the quadrant = (pi/2) r / N
    long double cc, ss;
    if (2 * r <= N) {
        const long double a = PI_2 * (long double)r / (long double)N;
        cc = cosl(a);
        ss = sinl(a);
    } else {
        const long double a = PI_2 * (long double)(N - r) / (long double)N;
        cc = sinl(a);
        ss = cosl(a);
    }
    const double c0 = (double)cc, s0 = (double)ss;
    switch (q & 3) {
        case 0: *c = c0; *s = s0; break;
        case 1: *c = -s0; *s = c0; break;
        case 2: *c = -c0; *s = -s0; break;
        default: *c = s0; *s = -c0; break;
    }
}

static int get_twiddles(agn_ctx* ctx, int64_t n, agn_precision prec, const void** out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto key = std::make_pair(n, (int)prec);
    auto it = ctx->tw.find(key);
    if (it != ctx->tw.end()) { *out = it->second; return AGN_OK; }
    const int64_t h = n / 2 + 1;
    void* dptr = nullptr;
    const size_t bytes = (size_t)h * 2 * prec_bytes(prec);
    if (hipMalloc(&dptr, bytes) != hipSuccess)
        return fail(AGN_ENOMEM, "twiddle table allocation of %zu bytes failed", bytes);
    if (prec == AGN_FP32) {
        std::vector<float> t(2 * h);
        for (int64_t i = 0; i < h; ++i) {
            double c, s;
            cis_2pi(i, n, &c, &s);
            t[2 * i] = (float)c;
            t[2 * i + 1] = (float)(-s);
        }
        HIPCHK(hipMemcpy(dptr, t.data(), bytes, hipMemcpyHostToDevice));
    } else {
        std::vector<double> t(2 * h);
        for (int64_t i = 0; i < h; ++i) {
            double c, s;
            cis_2pi(i, n, &c, &s);
            t[2 * i] = c;
            t[2 * i + 1] = -s;
        }
        HIPCHK(hipMemcpy(dptr, t.data(), bytes, hipMemcpyHostToDevice));
    }
    ctx->tw[key] = dptr;
    *out = dptr;
    return AGN_OK;
}

// Copies `bytes` of host data to device `dst` on `st` through a pinned
// staging slot (the slot is reused only after its previous copy completed).
static int stage_upload(agn_ctx* ctx, void* dst, const void* src, size_t bytes, hipStream_t st) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->ring.empty()) ctx->ring.resize(64);
    StageSlot& s = ctx->ring[ctx->ring_next++ % ctx->ring.size()];
    if (s.used) HIPCHK(hipEventSynchronize(s.ev));
    if (!s.ev) HIPCHK(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    if (s.cap < bytes) {
        if (s.host) HIPCHK(hipHostFree(s.host));
        s.host = nullptr;
        const size_t cap = std::max(bytes, (size_t)4096);
        HIPCHK(hipHostMalloc(&s.host, cap, hipHostMallocDefault));
        s.cap = cap;
    }
    memcpy(s.host, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(s.ev, st));
    s.used = true;
    return AGN_OK;
}

extern "C" int agn_ctx_create(int device, agn_ctx** out) {
    if (!out) return fail(AGN_EINVAL, "out is NULL");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(AGN_EINVAL, "device %d out of range (%d devices)", device, ndev);
    HIPCHK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    agn_ctx* c = new agn_ctx();
    c->device = device;
    c->lds_max = prop.sharedMemPerBlock;
    *out = c;
    return AGN_OK;
}

extern "C" int agn_ctx_set_profiling(agn_ctx* ctx, int on) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    ctx->prof = on != 0;
    return AGN_OK;
}

extern "C" const char* agn_ctx_kernel_names(void) { return KERNEL_NAMES; }

extern "C" int agn_ctx_kernel_time(agn_ctx* ctx, const char* name, double* total_ms,
                                   int64_t* launches, int reset) {
    if (!ctx || !name || !total_ms || !launches) return fail(AGN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& r : ctx->prof_recs) {
        if (strcmp(r.name, name) != 0) continue;
        HIPCHK(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        tot += ms;
        ++cnt;
    }
    *total_ms = tot;
    *launches = cnt;
    if (reset) {
        for (auto& r : ctx->prof_recs) {
            hipEventSynchronize(r.b);
            hipEventDestroy(r.a);
            hipEventDestroy(r.b);
        }
        ctx->prof_recs.clear();
    }
    return AGN_OK;
}

extern "C" int agn_ctx_destroy(agn_ctx* ctx) {
    if (!ctx) return AGN_OK;
    hipSetDevice(ctx->device);
    for (auto& r : ctx->prof_recs) {
        hipEventSynchronize(r.b);
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto& s : ctx->ring) {
        if (s.used && s.ev) hipEventSynchronize(s.ev);
        if (s.ev) hipEventDestroy(s.ev);
        if (s.host) hipHostFree(s.host);
    }
    for (auto& kv : ctx->tw) hipFree(kv.second);
    delete ctx;
    return AGN_OK;
}

// ---------------------------------------------------------------------------
// workspace sizes
// ---------------------------------------------------------------------------
extern "C" int agn_spectrum_workspace_size(int64_t n, size_t* bytes) {
    if (!bytes) return fail(AGN_EINVAL, "bytes is NULL");
    if (!n_supported(n)) return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [2, 2^27]", (long long)n);
    *bytes = header_ws(1) + spectrum_ws(n);
    return AGN_OK;
}

static int check_prec(agn_precision prec) {
    if (prec != AGN_FP32 && prec != AGN_FP64) return fail(AGN_EINVAL, "unknown precision %d", (int)prec);
    return AGN_OK;
}

static int check_path(int64_t n, agn_precision prec) {
    if (!n_supported(n)) return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [2, 2^27]", (long long)n);
    if (!lds_path(n, prec))
        return fail(AGN_EUNSUPPORTED_N, "n=%lld exceeds the lengths this build iterates in %s",
                    (long long)n, prec == AGN_FP32 ? "FP32" : "FP64");
    return AGN_OK;
}

extern "C" int agn_workspace_size(int64_t n, agn_precision prec, size_t* bytes) {
    if (!bytes) return fail(AGN_EINVAL, "bytes is NULL");
    int rc = check_prec(prec);
    if (rc) return rc;
    if ((rc = check_path(n, prec))) return rc;
    *bytes = header_ws(1) + curve_ws(n, prec);
    return AGN_OK;
}

extern "C" int agn_batch_workspace_size(int32_t n_curves, const int64_t* n, agn_precision prec,
                                        size_t* bytes) {
    if (!bytes || (n_curves > 0 && !n)) return fail(AGN_EINVAL, "NULL argument");
    if (n_curves < 0) return fail(AGN_EINVAL, "n_curves < 0");
    int rc = check_prec(prec);
    if (rc) return rc;
    size_t b = header_ws(n_curves);
    for (int32_t c = 0; c < n_curves; ++c) {
        if ((rc = check_path(n[c], prec))) return rc;
        b += curve_ws(n[c], prec);
    }
    *bytes = b;
    return AGN_OK;
}

// ---------------------------------------------------------------------------
// batch engine
// ---------------------------------------------------------------------------
struct CurveReq {
    int64_t n;
    double dt;
    agn_psd_params p;
    int32_t iters;
    uint64_t seed;
    uint32_t curve_id;
    const void* amp_in;  // non-null: iterate only
    const double* x0;
    double* x_out;
    double* delta_out;
    int32_t* iters_done;
    uint32_t* rank_out;
};

static bool valid_params(const agn_psd_params* p, double dt) {
    if (!p) return false;
    if (!(dt > 0.0) || !std::isfinite(dt)) return false;
    if (!(p->f_br > 0.0) || !std::isfinite(p->f_br)) return false;
    if (!std::isfinite(p->a_low) || !std::isfinite(p->a_high) || !std::isfinite(p->norm)) return false;
    return true;
}

template <typename T, int E>
static void launch_lds(agn_ctx* ctx, const LcDesc* d, int count, int nt, size_t prep_lds,
                       size_t iter_lds, hipStream_t st) {
    {
        ProfScope ps(ctx, "lds_prep", st);
        hipLaunchKernelGGL((k_lds_prep<T, E>), dim3(count), dim3(nt), prep_lds, st, d);
    }
    {
        ProfScope ps(ctx, "lds_iterate", st);
        hipLaunchKernelGGL((k_lds_iterate<T, E>), dim3(count), dim3(nt), iter_lds, st, d);
    }
}

template <typename T>
static int launch_lds_E(agn_ctx* ctx, int E, const LcDesc* d, int count, int nt, size_t prep_lds,
                        size_t iter_lds, hipStream_t st) {
    switch (E) {
        case 1: launch_lds<T, 1>(ctx, d, count, nt, prep_lds, iter_lds, st); break;
        case 2: launch_lds<T, 2>(ctx, d, count, nt, prep_lds, iter_lds, st); break;
        case 3: launch_lds<T, 3>(ctx, d, count, nt, prep_lds, iter_lds, st); break;
        case 4: launch_lds<T, 4>(ctx, d, count, nt, prep_lds, iter_lds, st); break;
        case 6: launch_lds<T, 6>(ctx, d, count, nt, prep_lds, iter_lds, st); break;
        case 8: launch_lds<T, 8>(ctx, d, count, nt, prep_lds, iter_lds, st); break;
        default: return fail(AGN_EINVAL, "internal: no kernel for E=%d", E);
    }
    return AGN_OK;
}

static void launch_spectrum(agn_ctx* ctx, const SpecDesc* d_sp, int nsp, int64_t nchunks,
                            hipStream_t st) {
    {
        ProfScope ps(ctx, "spectrum_partial", st);
        hipLaunchKernelGGL(k_spec_partial, dim3((unsigned)nchunks), dim3(SPEC_THREADS), 0, st, d_sp, nsp);
    }
    {
        ProfScope ps(ctx, "spectrum_norm", st);
        hipLaunchKernelGGL(k_spec_norm, dim3((unsigned)nsp), dim3(SPEC_THREADS), 0, st, d_sp);
    }
    {
        ProfScope ps(ctx, "spectrum_amp", st);
        hipLaunchKernelGGL(k_spec_amp, dim3((unsigned)nchunks), dim3(SPEC_THREADS), 0, st, d_sp, nsp);
    }
}

static int run_batch(agn_ctx* ctx, std::vector<CurveReq>& rq, double tol, agn_precision prec,
                     void* ws, size_t ws_bytes, hipStream_t st) {
    const int32_t nc = (int32_t)rq.size();
    if (nc == 0) return AGN_OK;
    size_t need = header_ws(nc);
    for (auto& r : rq) need += curve_ws(r.n, prec);
    if (!ws || ws_bytes < need)
        return fail(AGN_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    HIPCHK(hipSetDevice(ctx->device));

    // Curves grouped by length (stable), so that each length is one launch.
    std::vector<int> order(nc);
    for (int i = 0; i < nc; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return rq[a].n < rq[b].n; });

    unsigned char* base = (unsigned char*)ws;
    LcDesc* d_lc = (LcDesc*)base;
    SpecDesc* d_sp = (SpecDesc*)(base + align256(sizeof(LcDesc) * (size_t)nc));
    std::vector<LcDesc> lc(nc);
    std::vector<SpecDesc> sp;
    size_t off = header_ws(nc);
    int64_t chunk0 = 0;
    const size_t pb = prec_bytes(prec);
    for (int i = 0; i < nc; ++i) {
        const CurveReq& r = rq[order[i]];
        const int64_t n = r.n, M = n / 2;
        LcDesc& d = lc[i];
        memset(&d, 0, sizeof(d));
        d.n = (int32_t)n;
        d.iters = r.iters;
        d.tol = tol;
        d.x0 = r.x0;
        d.s64 = (double*)(base + off); off += align256((size_t)n * 8);
        d.sT = (void*)(base + off); off += align256((size_t)n * pb);
        d.L = (double*)(base + off); off += align256((size_t)n * 8);
        d.rank0 = (uint32_t*)(base + off); off += align256((size_t)n * 4);
        d.valid = (int32_t*)(base + off); off += align256(16);
        void* amp_ws = (void*)(base + off); off += align256((size_t)(M + 1) * pb);
        double* partial = (double*)(base + off); off += align256((size_t)spec_chunks(n) * 8);
        double* A = (double*)(base + off); off += align256(8);
        d.x_out = r.x_out;
        d.delta_out = r.delta_out;
        d.iters_done = r.iters_done;
        d.rank_out = r.rank_out;
        const void* tw = nullptr;
        int rc = get_twiddles(ctx, n, prec, &tw);
        if (rc) return rc;
        d.tw = tw;
        d.plan = make_plan(M);
        if (r.amp_in) {
            d.amp = r.amp_in;
        } else {
            d.amp = amp_ws;
            SpecDesc s;
            memset(&s, 0, sizeof(s));
            s.n = n;
            s.dt = r.dt;
            s.norm = r.p.norm;
            s.f_br = r.p.f_br;
            s.a_low = r.p.a_low;
            s.a_high = r.p.a_high;
            s.seed = r.seed;
            s.curve_id = r.curve_id;
            s.is_f32 = prec == AGN_FP32;
            s.chunk0 = chunk0;
            s.nchunk = spec_chunks(n);
            s.amp = amp_ws;
            s.partial = partial;
            s.A = A;
            chunk0 += s.nchunk;
            sp.push_back(s);
        }
    }
    // Upload descriptors (LcDesc block then SpecDesc block, one copy).
    {
        std::vector<unsigned char> hdr(header_ws(nc), 0);
        memcpy(hdr.data(), lc.data(), sizeof(LcDesc) * (size_t)nc);
        if (!sp.empty())
            memcpy(hdr.data() + align256(sizeof(LcDesc) * (size_t)nc), sp.data(), sizeof(SpecDesc) * sp.size());
        int rc = stage_upload(ctx, ws, hdr.data(), hdr.size(), st);
        if (rc) return rc;
    }
    if (!sp.empty()) {
        const int nsp = (int)sp.size();
        launch_spectrum(ctx, d_sp, nsp, chunk0, st);
        HIPCHK(hipGetLastError());
    }
    // One prep + iterate launch per distinct length.
    int i = 0;
    while (i < nc) {
        int j = i;
        while (j < nc && lc[j].n == lc[i].n) ++j;
        const int64_t n = lc[i].n;
        const int E = lds_ipt(n) / 2;
        const int nt = (int)(n / lds_ipt(n));
        const size_t pl = lds_prep_bytes(n), il = lds_iter_bytes(n, prec);
        if (pl > ctx->lds_max || il > ctx->lds_max)
            return fail(AGN_EUNSUPPORTED_N, "n=%lld needs %zu bytes of LDS per workgroup; the device allows %zu",
                        (long long)n, std::max(pl, il), ctx->lds_max);
        int rc = (prec == AGN_FP32) ? launch_lds_E<float>(ctx, E, d_lc + i, j - i, nt, pl, il, st)
                                    : launch_lds_E<double>(ctx, E, d_lc + i, j - i, nt, pl, il, st);
        if (rc) return rc;
        HIPCHK(hipGetLastError());
        i = j;
    }
    return AGN_OK;
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
extern "C" int agn_psd_spectrum(agn_ctx* ctx, const agn_psd_params* p, int64_t n, double dt,
                                uint64_t seed, uint32_t curve_id, agn_precision prec,
                                void* amp_out, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !p || !amp_out) return fail(AGN_EINVAL, "NULL argument");
    int rc = check_prec(prec);
    if (rc) return rc;
    if (!n_supported(n)) return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [2, 2^27]", (long long)n);
    if (!valid_params(p, dt)) return fail(AGN_EINVAL, "invalid PSD parameters or dt");
    const size_t need = header_ws(1) + spectrum_ws(n);
    if (!ws || ws_bytes < need) return fail(AGN_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    unsigned char* base = (unsigned char*)ws;
    SpecDesc s;
    memset(&s, 0, sizeof(s));
    s.n = n; s.dt = dt; s.norm = p->norm; s.f_br = p->f_br; s.a_low = p->a_low; s.a_high = p->a_high;
    s.seed = seed; s.curve_id = curve_id; s.is_f32 = prec == AGN_FP32;
    s.chunk0 = 0; s.nchunk = spec_chunks(n);
    s.amp = amp_out;
    s.partial = (double*)(base + header_ws(1));
    s.A = (double*)(base + header_ws(1) + align256((size_t)s.nchunk * 8));
    SpecDesc* d_sp = (SpecDesc*)base;
    if ((rc = stage_upload(ctx, d_sp, &s, sizeof(s), st))) return rc;
    launch_spectrum(ctx, d_sp, 1, s.nchunk, st);
    HIPCHK(hipGetLastError());
    return AGN_OK;
}

extern "C" int agn_lc_iterate(agn_ctx* ctx, const void* amp, const double* x0, int64_t n,
                              int32_t iters, double tol, agn_precision prec, double* x_out,
                              double* delta_out, int32_t* iters_done, uint32_t* rank_out,
                              void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !amp || !x0 || !x_out) return fail(AGN_EINVAL, "NULL argument");
    int rc = check_prec(prec);
    if (rc) return rc;
    if ((rc = check_path(n, prec))) return rc;
    if (iters < 0) return fail(AGN_EINVAL, "iters < 0");
    if (std::isnan(tol)) return fail(AGN_EINVAL, "tol is NaN");
    std::vector<CurveReq> rq(1);
    CurveReq& r = rq[0];
    memset(&r, 0, sizeof(r));
    r.n = n; r.iters = iters; r.amp_in = amp; r.x0 = x0; r.x_out = x_out;
    r.delta_out = delta_out; r.iters_done = iters_done; r.rank_out = rank_out;
    return run_batch(ctx, rq, tol, prec, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int agn_lc_generate(agn_ctx* ctx, const agn_psd_params* p, const double* erdf, int64_t n,
                               double dt, int32_t iters, double tol, uint64_t seed,
                               uint32_t curve_id, agn_precision prec, double* x_out,
                               double* delta_out, int32_t* iters_done, void* ws, size_t ws_bytes,
                               void* stream) {
    if (!ctx || !p || !erdf || !x_out) return fail(AGN_EINVAL, "NULL argument");
    int rc = check_prec(prec);
    if (rc) return rc;
    if ((rc = check_path(n, prec))) return rc;
    if (iters < 0) return fail(AGN_EINVAL, "iters < 0");
    if (std::isnan(tol)) return fail(AGN_EINVAL, "tol is NaN");
    if (!valid_params(p, dt)) return fail(AGN_EINVAL, "invalid PSD parameters or dt");
    std::vector<CurveReq> rq(1);
    CurveReq& r = rq[0];
    memset(&r, 0, sizeof(r));
    r.n = n; r.dt = dt; r.p = *p; r.iters = iters; r.seed = seed; r.curve_id = curve_id;
    r.x0 = erdf; r.x_out = x_out; r.delta_out = delta_out; r.iters_done = iters_done;
    return run_batch(ctx, rq, tol, prec, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int agn_lc_generate_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n,
                                     const int64_t* offset, const agn_psd_params* p, const double* dt,
                                     const int32_t* iters, const uint64_t* seed,
                                     const uint32_t* curve_id, const double* erdf, double tol,
                                     agn_precision prec, double* x_out, double* delta_out,
                                     int32_t* iters_done, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    if (n_curves < 0) return fail(AGN_EINVAL, "n_curves < 0");
    if (n_curves == 0) return AGN_OK;
    if (!n || !offset || !p || !dt || !iters || !seed || !curve_id || !erdf || !x_out)
        return fail(AGN_EINVAL, "NULL argument");
    int rc = check_prec(prec);
    if (rc) return rc;
    if (std::isnan(tol)) return fail(AGN_EINVAL, "tol is NaN");
    int32_t max_it = 0;
    std::vector<std::pair<int64_t, int64_t>> spans;
    for (int32_t c = 0; c < n_curves; ++c) {
        if ((rc = check_path(n[c], prec))) return rc;
        if (iters[c] < 0) return fail(AGN_EINVAL, "iters[%d] < 0", c);
        if (offset[c] < 0) return fail(AGN_EINVAL, "offset[%d] < 0", c);
        if (!valid_params(&p[c], dt[c])) return fail(AGN_EINVAL, "invalid PSD parameters or dt for curve %d", c);
        max_it = std::max(max_it, iters[c]);
        spans.push_back({offset[c], offset[c] + n[c]});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return fail(AGN_EINVAL, "curves overlap in erdf/x_out");
    std::vector<CurveReq> rq(n_curves);
    for (int32_t c = 0; c < n_curves; ++c) {
        CurveReq& r = rq[c];
        memset(&r, 0, sizeof(r));
        r.n = n[c]; r.dt = dt[c]; r.p = p[c]; r.iters = iters[c]; r.seed = seed[c];
        r.curve_id = curve_id[c];
        r.x0 = erdf + offset[c];
        r.x_out = x_out + offset[c];
        r.delta_out = delta_out ? delta_out + (size_t)c * max_it : nullptr;
        r.iters_done = iters_done ? iters_done + c : nullptr;
    }
    return run_batch(ctx, rq, tol, prec, ws, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// test exports
// ---------------------------------------------------------------------------
extern "C" int agn_test_philox(uint64_t key0, uint64_t key1, uint64_t ctr0, int64_t n_blocks,
                               uint64_t* out, void* stream) {
    if (!out || n_blocks < 0) return fail(AGN_EINVAL, "bad argument");
    if (n_blocks == 0) return AGN_OK;
    const int64_t nb = (n_blocks + 255) / 256;
    hipLaunchKernelGGL(k_philox_blocks, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, key0,
                       key1, ctr0, n_blocks, out);
    HIPCHK(hipGetLastError());
    return AGN_OK;
}
