// agn.hip -- C ABI of the MI355X light-curve generator (see include/agn.h).
//
// Host side: argument checks, workspace layout, descriptor upload, per-length
// plans and twiddle tables, and kernel launches.  Every step of the method
// runs in the kernels included below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/agn.h"
#include "common.hpp"
#include "big_path.hpp"
#include "erdf.hpp"
#include "observables.hpp"
#include "lds_iterate.hpp"
#include "philox.hpp"
#include "spectrum.hpp"
#include "test_kernels.hpp"

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

static size_t big_curve_ws(int64_t n, agn_precision prec);

// Per-curve workspace: s64, sT, L, rank0, valid, amp, spectrum scratch.
static size_t curve_ws(int64_t n, agn_precision prec) {
    if (!lds_path(n, prec)) return big_curve_ws(n, prec);
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

// Per-curve workspace of the multi-pass path.
static int64_t big_npart(int64_t n) { return n / 2048 + 1; }

static size_t big_curve_ws(int64_t n, agn_precision prec) {
    const size_t pb = prec_bytes(prec);
    const size_t region = (size_t)n * 12;  // max of (iteration key + value) and (64-bit key + value)
    const int64_t ntiles = n / BIG_TILE;
    size_t b = 0;
    b += align256((size_t)n * 8);           // s64
    b += 2 * align256((size_t)n * 8);       // X0, X1
    b += 2 * align256((size_t)n * 4);       // rankA, rankB
    b += 2 * align256(region);              // sortA, sortB
    b += align256((size_t)ntiles * 256 * 4);  // look
    b += 2 * align256(SORT_MAX_PASSES * 256 * 4);  // dcount, dstart
    b += align256(SORT_MAX_PASSES * 4);     // tickets
    b += align256((size_t)big_npart(n) * 8);  // dpart
    b += align256((size_t)big_npart(n) * 4);  // cpart
    b += align256(16);                      // state
    b += align256((size_t)(n / 2 + 1) * pb);  // amp
    b += spectrum_ws(n);
    return b;
}

static size_t header_ws(int32_t nc) {
    return align256(sizeof(LcDesc) * (size_t)nc) + align256(sizeof(SpecDesc) * (size_t)nc) +
           align256(sizeof(BigCurve) * (size_t)nc) + align256(sizeof(LdsPack) * (size_t)nc);
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

// Device memory of the allocation-free entry point (agn_psd_spectrum_noalloc):
// the curve's descriptor and the normalisation's partial sums.  Every device
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (agn_ctx::scratch_dev), never through this name.
static constexpr size_t NOALLOC_SCRATCH_BYTES = 512 * 1024;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

struct agn_ctx {
    int device = 0;
    void* scratch_dev = nullptr;  // this device's copy of `scratch` (null if the lookup failed)
    size_t lds_max = 65536;  // LDS bytes one workgroup may allocate
    int ncu = 256;           // compute units
    bool prof = false;
    std::vector<ProfRec> prof_recs;
    std::mutex mu;
    std::map<std::pair<int64_t, int>, void*> tw;
    std::map<int64_t, TwTable> tw64;
    std::vector<void*> tw64_mem;
    std::vector<StageSlot> ring;
    size_t ring_next = 0;
    std::map<std::string, std::array<int, 3>> tuned;  // batch signature -> (chains, sort tile, FFT cap) chosen by the autotuner
    int look_polls = LOOK_SPIN_MAX;  // look-back wait limit of the multi-pass sort (< 0: give up at once)
};

static const char* KERNEL_NAMES =
    "spectrum_partial,spectrum_norm,spectrum_amp,lds_prep,lds_iterate,lds_packs,big_prep,fft_pass,fft_mid,"
    "sort_hist,sort_scan,sort_scatter,delta,big_output,erdf_draw,batch_graph,periodogram,log_bins,lag_stats,psd_fit";

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
            return;
        }
        if (b) (void)hipEventDestroy(b);
        (void)hipEventDestroy(a);
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
        const hipError_t e = hipMemcpy(dptr, t.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(dptr);
            return fail(AGN_EDEVICE, "twiddle table upload: %s", hipGetErrorString(e));
        }
    } else {
        std::vector<double> t(2 * h);
        for (int64_t i = 0; i < h; ++i) {
            double c, s;
            cis_2pi(i, n, &c, &s);
            t[2 * i] = c;
            t[2 * i + 1] = -s;
        }
        const hipError_t e = hipMemcpy(dptr, t.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(dptr);
            return fail(AGN_EDEVICE, "twiddle table upload: %s", hipGetErrorString(e));
        }
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
        s.cap = 0;  // stays empty if the allocation below fails
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
    // this device's copy of the allocation-free entry point's scratch array
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess) sp = nullptr;
    agn_ctx* c = new agn_ctx();
    c->device = device;
    c->lds_max = prop.sharedMemPerBlock;
    c->ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->scratch_dev = sp;
    *out = c;
    return AGN_OK;
}

extern "C" int agn_ctx_set_profiling(agn_ctx* ctx, int on) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    ctx->prof = on != 0;
    return AGN_OK;
}

extern "C" int agn_ctx_set_lookback_polls(agn_ctx* ctx, int32_t polls) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    ctx->look_polls = polls == 0 ? LOOK_SPIN_MAX : polls;
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
            (void)hipEventSynchronize(r.b);
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        ctx->prof_recs.clear();
    }
    return AGN_OK;
}

extern "C" int agn_ctx_destroy(agn_ctx* ctx) {
    if (!ctx) return AGN_OK;
    (void)hipSetDevice(ctx->device);
    for (auto& r : ctx->prof_recs) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto& s : ctx->ring) {
        if (s.used && s.ev) (void)hipEventSynchronize(s.ev);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.host) (void)hipHostFree(s.host);
    }
    for (auto& kv : ctx->tw) (void)hipFree(kv.second);
    for (void* p : ctx->tw64_mem) (void)hipFree(p);
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
    (void)prec;
    if (!n_supported(n)) return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [2, 2^27]", (long long)n);
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
static void launch_lds(agn_ctx* ctx, const LcDesc* d, int count, int nt, bool fuse2, size_t prep_lds,
                       size_t iter_lds, hipStream_t st) {
    {
        ProfScope ps(ctx, "lds_prep", st);
        hipLaunchKernelGGL((k_lds_prep<T, E>), dim3(count), dim3(nt), prep_lds, st, d);
    }
    {
        ProfScope ps(ctx, "lds_iterate", st);
        if (fuse2) hipLaunchKernelGGL((k_lds_iterate<T, E, true>), dim3(count), dim3(nt), iter_lds, st, d);
        else hipLaunchKernelGGL((k_lds_iterate<T, E, false>), dim3(count), dim3(nt), iter_lds, st, d);
    }
}

// Whether the LDS kernel fuses the forward transform's last pass into the
// replacement: the half-length plan ends with radix 2.
static bool lds_fuse2(int64_t n) {
    const FftPlan pl = make_plan(n / 2);
    return pl.npass >= 2 && pl.radix[pl.npass - 1] == 2 && n / 2 >= 16;
}

template <typename T>
static int launch_lds_E(agn_ctx* ctx, int E, const LcDesc* d, int count, int nt, bool fuse2, size_t prep_lds,
                        size_t iter_lds, hipStream_t st) {
    if (E >= 8 && nt % 32 != 0) return fail(AGN_EINVAL, "internal: %d-thread block for E=%d", nt, E);
    switch (E) {
        case 1: launch_lds<T, 1>(ctx, d, count, nt, fuse2, prep_lds, iter_lds, st); break;
        case 2: launch_lds<T, 2>(ctx, d, count, nt, fuse2, prep_lds, iter_lds, st); break;
        case 3: launch_lds<T, 3>(ctx, d, count, nt, fuse2, prep_lds, iter_lds, st); break;
        case 4: launch_lds<T, 4>(ctx, d, count, nt, fuse2, prep_lds, iter_lds, st); break;
        case 6: launch_lds<T, 6>(ctx, d, count, nt, fuse2, prep_lds, iter_lds, st); break;
        case 8: launch_lds<T, 8>(ctx, d, count, nt, fuse2, prep_lds, iter_lds, st); break;
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

// FP64 two-level twiddle table of length n (multi-pass path), cached per n.
static int get_tw64(agn_ctx* ctx, int64_t n, TwTable* out) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tw64.find(n);
    if (it != ctx->tw64.end()) { *out = it->second; return AGN_OK; }
    const int64_t B = (int64_t)1 << TW_LO_BITS;
    const int64_t nlo = B, nhi = n / B + 2;
    std::vector<double> t(2 * (nlo + nhi));
    for (int64_t u = 0; u < nlo; ++u) {
        double c, sn;
        cis_2pi(u, n, &c, &sn);
        t[2 * u] = c;
        t[2 * u + 1] = -sn;
    }
    for (int64_t v = 0; v < nhi; ++v) {
        double c, sn;
        cis_2pi(v * B, n, &c, &sn);
        t[2 * (nlo + v)] = c;
        t[2 * (nlo + v) + 1] = -sn;
    }
    void* dptr = nullptr;
    const size_t bytes = t.size() * sizeof(double);
    if (hipMalloc(&dptr, bytes) != hipSuccess)
        return fail(AGN_ENOMEM, "twiddle table allocation of %zu bytes failed", bytes);
    const hipError_t e = hipMemcpy(dptr, t.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dptr);
        return fail(AGN_EDEVICE, "twiddle table upload: %s", hipGetErrorString(e));
    }
    TwTable tb;
    tb.lo = (const cplx<double>*)dptr;
    tb.hi = (const cplx<double>*)dptr + nlo;
    ctx->tw64[n] = tb;
    ctx->tw64_mem.push_back(dptr);
    *out = tb;
    return AGN_OK;
}

// Radices of the HBM passes of a length-M complex FFT: as few passes as the
// largest in-LDS radix (2^9 FP32, 2^8 FP64) allows, exponents split evenly;
// the factor 3, if any, joins the first pass (whose exponent is capped so that
// 3 * 2^e stays within the limit).  Every pass keeps M / R a multiple of 16.
static std::vector<int> big_radices(int64_t M, agn_precision prec) {
    const int maxlog = prec == AGN_FP32 ? 9 : 8;
    const int three = (M % 3 == 0) ? 1 : 0;
    int64_t m = three ? M / 3 : M;
    int a = 0;
    while (m > 1) { m >>= 1; ++a; }
    for (int np = 1; np <= 8; ++np) {
        const int cap0 = three ? maxlog - 2 : maxlog;
        if (a > cap0 + (np - 1) * maxlog) continue;
        std::vector<int> e(np, 0);
        const int target = (a + np - 1) / np;
        e[0] = std::min(cap0, target);
        int rest = a - e[0];
        for (int i = 1; i < np; ++i) {
            const int left = np - i;
            e[i] = std::min(maxlog, (rest + left - 1) / left);
            rest -= e[i];
        }
        if (rest != 0) continue;
        std::vector<int> r(np);
        for (int i = 0; i < np; ++i) r[i] = (1 << e[i]) * ((i == 0 && three) ? 3 : 1);
        return r;
    }
    return {};
}

// Tile of one FFT workgroup: R x cols complex values = 64 KB.
static int fft_tile(agn_precision prec) { return prec == AGN_FP32 ? 8192 : 4096; }

// Butterflies per workgroup of a pass over stride Ns: the largest power of
// two <= cap (64, or a plan's tuned cap) with R * cols within the tile,
// dividing M / R and, after the first pass, dividing Ns (a workgroup's
// columns then share one j mod Ns offset run); 0 if none >= 16.  The column
// count does not change the arithmetic: each element's twiddle chain depends
// on its row and the rows a thread steps by (R / E), not on the columns.
static int fft_cols(int64_t M, int R, int64_t Ns, agn_precision prec, int cap = FFT_COLS_MAX) {
    for (int c = cap; c >= FFT_COLS_MIN; c >>= 1)
        if ((int64_t)R * c <= fft_tile(prec) && (M / R) % c == 0 && (Ns == 1 || Ns % c == 0)) return c;
    return 0;
}

// Values per thread of the multi-pass FFT passes (R * cols / FFT_E threads,
// at most 1024 since R * cols <= 8192): 8 rather than 16 puts twice the waves
// on the same tiles (-2% per pass at 2^26).
static constexpr int FFT_E = 8;

// log2 R for the power-of-two radices that have a compile-time transform
// (k_fft_pass / k_fft_mid with LR > 0: the same arithmetic with constant
// indexing), 0 for the others (the factor 3 of 3 * 2^k lengths).
static int fft_lr(int R) {
    for (int lr = 4; lr <= 9; ++lr)
        if (R == (1 << lr)) return lr;
    return 0;
}

template <typename T, bool INV, int C, int LR>
static void launch_fft_pass_lr(const BigCurve* d, int nc, const FftPass& P, const TwTable& tb, size_t lds,
                               hipStream_t st) {
    dim3 grid((unsigned)(P.M / P.R / C), (unsigned)nc);
    hipLaunchKernelGGL((k_fft_pass<T, FFT_E, INV, C, LR>), grid, dim3(P.nthreads), lds, st, d, P, tb);
}

template <typename T, bool INV, int C>
static void launch_fft_pass_c(const BigCurve* d, int nc, const FftPass& P, const TwTable& tb, size_t lds,
                              hipStream_t st) {
    // fft_cols keeps R * C within the tile, so only those shapes are instantiated
    constexpr int TILE = sizeof(T) == 4 ? 8192 : 4096;
    switch (fft_lr(P.R)) {
        case 4: if constexpr (16 * C <= TILE) { launch_fft_pass_lr<T, INV, C, 4>(d, nc, P, tb, lds, st); return; } break;
        case 5: if constexpr (32 * C <= TILE) { launch_fft_pass_lr<T, INV, C, 5>(d, nc, P, tb, lds, st); return; } break;
        case 6: if constexpr (64 * C <= TILE) { launch_fft_pass_lr<T, INV, C, 6>(d, nc, P, tb, lds, st); return; } break;
        case 7: if constexpr (128 * C <= TILE) { launch_fft_pass_lr<T, INV, C, 7>(d, nc, P, tb, lds, st); return; } break;
        case 8: if constexpr (256 * C <= TILE) { launch_fft_pass_lr<T, INV, C, 8>(d, nc, P, tb, lds, st); return; } break;
        case 9: if constexpr (512 * C <= TILE) { launch_fft_pass_lr<T, INV, C, 9>(d, nc, P, tb, lds, st); return; } break;
        default: break;
    }
    launch_fft_pass_lr<T, INV, C, 0>(d, nc, P, tb, lds, st);
}

template <typename T>
static void launch_fft_pass(agn_ctx* ctx, const BigCurve* d, int nc, const FftPass& P, const TwTable& tb,
                            hipStream_t st) {
    const int C = P.cols;
    const size_t lds = (size_t)(P.R * C + 1 + ((P.R * C + 1) >> (sizeof(T) == 4 ? 5 : 4))) * sizeof(cplx<T>) +
                       16 + (size_t)P.R * sizeof(cplx<T>) + 16 * 8 + 16 * 4;
    ProfScope ps(ctx, "fft_pass", st);
    if (P.inverse) {
        if (C == 64) launch_fft_pass_c<T, true, 64>(d, nc, P, tb, lds, st);
        else if (C == 32) launch_fft_pass_c<T, true, 32>(d, nc, P, tb, lds, st);
        else launch_fft_pass_c<T, true, 16>(d, nc, P, tb, lds, st);
    } else {
        if (C == 64) launch_fft_pass_c<T, false, 64>(d, nc, P, tb, lds, st);
        else if (C == 32) launch_fft_pass_c<T, false, 32>(d, nc, P, tb, lds, st);
        else launch_fft_pass_c<T, false, 16>(d, nc, P, tb, lds, st);
    }
}

// Column pairs per workgroup of the middle pass: 8 (16 columns of R values,
// at most 32 KB in FP32 and 64 KB in FP64 for R <= 256), with 8 values per
// thread; 0 if 16 columns do not divide M / R.  The middle pass does two
// in-LDS transforms and the fold per trip through HBM, and more, smaller
// workgroups per CU overlap those phases better: at 2^26 (R = 256, FP32) this
// shape takes 1.22 ms per launch against 1.30-1.42 ms for 16 or 32 column
// pairs or 16 values per thread.
static constexpr int MID_E = 8;
static int mid_cols(int64_t M, int R, agn_precision prec) {
    const int c = 8;
    return ((int64_t)R * 2 * c <= fft_tile(prec) && (M / R) % (2 * c) == 0) ? c : 0;
}

static MidPass make_mid(int64_t M, int R, int src_sel, int dst_sel, agn_precision prec) {
    MidPass P;
    memset(&P, 0, sizeof(P));
    P.M = M;
    P.R = R;
    P.cols = mid_cols(M, R, prec);
    P.nthreads = R * 2 * P.cols / MID_E;
    P.src_sel = src_sel;
    P.dst_sel = dst_sel;
    P.sub = make_plan(R);
    return P;
}

template <typename T, int MODE>
static void launch_fft_mid(agn_ctx* ctx, const BigCurve* d, int nc, const MidPass& P, const TwTable& tb,
                           hipStream_t st) {
    const int C2 = 2 * P.cols;
    const size_t lds = (size_t)(P.R * C2 + 1 + ((P.R * C2 + 1) >> (sizeof(T) == 4 ? 5 : 4))) * sizeof(cplx<T>) +
                       16 + (size_t)P.R * sizeof(cplx<T>);
    const dim3 grid((unsigned)(P.M / P.R / C2), (unsigned)nc);
    ProfScope ps(ctx, "fft_mid", st);
    // the iteration's mode takes the compile-time transform for R = 2^6 .. 2^9
    // (R * 16 columns within the tile); the test exports keep the general one
    constexpr int TILE = sizeof(T) == 4 ? 8192 : 4096;
    if constexpr (MODE == MID_REPLACE) {
        switch (fft_lr(P.R)) {
            case 6: { hipLaunchKernelGGL((k_fft_mid<T, MID_E, 8, MODE, 6>), grid, dim3(P.nthreads), lds, st, d, P, tb); return; }
            case 7: { hipLaunchKernelGGL((k_fft_mid<T, MID_E, 8, MODE, 7>), grid, dim3(P.nthreads), lds, st, d, P, tb); return; }
            case 8:
                if constexpr (256 * 16 <= TILE)
                    { hipLaunchKernelGGL((k_fft_mid<T, MID_E, 8, MODE, 8>), grid, dim3(P.nthreads), lds, st, d, P, tb); return; }
                break;
            case 9:
                if constexpr (512 * 16 <= TILE)
                    { hipLaunchKernelGGL((k_fft_mid<T, MID_E, 8, MODE, 9>), grid, dim3(P.nthreads), lds, st, d, P, tb); return; }
                break;
            default: break;
        }
    }
    hipLaunchKernelGGL((k_fft_mid<T, MID_E, 8, MODE, 0>), grid, dim3(P.nthreads), lds, st, d, P, tb);
}

// One LSD sort of the keys in region src0, sizeof(K) passes of 8-bit digits:
// digit totals of every pass, their starts, then the scatter passes (the last
// in `last_mode`).  *seq counts the scatter passes of the call, which gives
// each pass its look-back epoch (consecutive passes differ).
constexpr int SORT_COUNT_WORKGROUPS = 512;  // k_sort_count workgroups over all curves of a launch

template <typename K, int TILE>
static void run_sort_t(agn_ctx* ctx, const BigCurve* d, int nc, int64_t n, int src0, int last_mode, int rank_sel,
                       int* seq, int polls, hipStream_t st) {
    const int64_t ntiles = n / TILE;
    const int npass = (int)sizeof(K);
    {
        ProfScope ps(ctx, "sort_hist", st);
        const int64_t g = std::min<int64_t>(ntiles, std::max(1, SORT_COUNT_WORKGROUPS / nc));
        hipLaunchKernelGGL((k_sort_count<K, TILE>), dim3((unsigned)g, (unsigned)nc), dim3(BIG_THREADS), 0, st, d,
                           src0, ntiles);
    }
    {
        ProfScope ps(ctx, "sort_scan", st);
        hipLaunchKernelGGL(k_sort_starts, dim3((unsigned)nc), dim3(BIG_THREADS), 0, st, d, npass);
    }
    int src = src0;
    for (int p = 0; p < npass; ++p) {
        SortPass P;
        memset(&P, 0, sizeof(P));
        P.shift = 8 * p;
        P.first = p == 0;
        P.src_sel = src;
        P.mode = p == npass - 1 ? last_mode : SORT_MODE_MOVE;
        P.rank_sel = rank_sel;
        P.pass = p;
        P.epoch = (*seq)++ % 3 + 1;
        P.spin_max = polls;
        ProfScope ps(ctx, "sort_scatter", st);
        hipLaunchKernelGGL((k_sort_scatter<K, TILE>), dim3((unsigned)ntiles, (unsigned)nc),
                           dim3(TILE / scat_ipt<K>::value), 0, st, d, P, ntiles);
        src = 1 - src;
    }
}

// Sort tile actually used for keys K on a curve of length n (a multiple of
// BIG_TILE).  want = SORT_TILE_AUTO chooses by length: the 16384-key tile for
// 32-bit keys of curves of at least 2^20 samples that it divides (its digit
// runs are twice as long; at 4 x 2^26 the scatter takes 1.94 ms per pass
// against 2.00 ms), else 8192.
constexpr int SORT_TILE_AUTO = 0;
constexpr int64_t SORT_TILE_AUTO_MIN_N = int64_t(1) << 20;
template <typename K>
static int sort_tile_for(int64_t n, int want) {
    if (sizeof(K) != 4 || n % SORT_TILE_BIG != 0) return BIG_TILE;
    if (want == SORT_TILE_AUTO) return n >= SORT_TILE_AUTO_MIN_N ? SORT_TILE_BIG : BIG_TILE;
    return want == SORT_TILE_BIG ? SORT_TILE_BIG : BIG_TILE;
}

template <typename K>
static void run_sort(agn_ctx* ctx, const BigCurve* d, int nc, int64_t n, int src0, int last_mode, int rank_sel,
                     int tile, int* seq, int polls, hipStream_t st) {
    if constexpr (sizeof(K) == 4) {
        if (sort_tile_for<K>(n, tile) == SORT_TILE_BIG) {
            run_sort_t<K, SORT_TILE_BIG>(ctx, d, nc, n, src0, last_mode, rank_sel, seq, polls, st);
            return;
        }
    }
    run_sort_t<K, BIG_TILE>(ctx, d, nc, n, src0, last_mode, rank_sel, seq, polls, st);
}

// Checks the multi-pass FFT plan of length n and resolves its twiddle table.
static int big_group_setup(agn_ctx* ctx, int64_t n, agn_precision prec, TwTable* tb, std::vector<int>* rad) {
    const int64_t M = n / 2;
    int rc = get_tw64(ctx, n, tb);
    if (rc) return rc;
    *rad = big_radices(M, prec);
    if (rad->empty()) return fail(AGN_EUNSUPPORTED_N, "internal: no FFT plan for n=%lld", (long long)n);
    // forward passes 0 .. np-2, the middle pass (radix rad[np-1]), then the
    // inverse passes in the reverse radix order
    const int np = (int)rad->size();
    bool ok = np >= 2 && mid_cols(M, rad->back(), prec) != 0 && rad->back() >= 16 && rad->back() <= 512;
    int64_t ns = 1;
    for (int p = 0; ok && p < np - 1; ++p) {
        const int r = (*rad)[p];
        const int c = fft_cols(M, r, ns, prec);
        ok = c != 0 && r <= 512 && r >= 16 && !(ns == 1 && r < 64);
        ns *= r;
    }
    ns = rad->back();
    for (int p = np - 2; ok && p >= 0; --p) {
        ok = fft_cols(M, (*rad)[p], ns, prec) != 0;
        ns *= (*rad)[p];
    }
    if (!ok) return fail(AGN_EUNSUPPORTED_N, "internal: no FFT plan for n=%lld", (long long)n);
    return AGN_OK;
}

// All curves of one length on the multi-pass path (plan checked by
// big_group_setup).  ctx may be NULL (no kernel timing, e.g. under capture).
template <typename T>
static void run_big_group(agn_ctx* ctx, const BigCurve* d, int nc, int64_t n, int32_t max_iters,
                          const TwTable& tb, const std::vector<int>& rad, int sort_tile, int fft_cap, int polls,
                          hipStream_t st) {
    typedef typename key_of<T>::type K;
    const int64_t M = n / 2, ntiles = n / BIG_TILE;
    const dim3 gt((unsigned)ntiles, (unsigned)nc);
    hipLaunchKernelGGL(k_big_init, dim3((unsigned)nc), dim3(64), 0, st, d);
    hipLaunchKernelGGL(k_sort_clear, gt, dim3(BIG_THREADS), 0, st, d);
    int seq = 0;  // scatter passes so far (look-back epochs)
    {
        ProfScope ps(ctx, "big_prep", st);
        hipLaunchKernelGGL(k_big_prep_keys, gt, dim3(BIG_THREADS), 0, st, d);
        run_sort<uint64_t>(nullptr, d, nc, n, 0, SORT_MODE_PREP, 0, BIG_TILE, &seq, polls, st);
    }
    hipLaunchKernelGGL(k_big_after_prep, dim3((unsigned)nc), dim3(64), 0, st, d);
    const int np = (int)rad.size();
    const int prec_bits = sizeof(T) == 4 ? 1 : 0;
    const agn_precision prec = prec_bits ? AGN_FP32 : AGN_FP64;
    // The first forward pass also sums the Eq. 4 terms per workgroup, so its
    // width fixes the order of that sum: it keeps the default width, and only
    // the other passes take the plan's (bit-neutral for them) width.
    const int64_t npart0 = M / rad[0] / fft_cols(M, rad[0], 1, prec);  // blocks of the first FFT pass
    for (int it = 0; it < max_iters; ++it) {
        const int cur = it & 1;  // x_it lives in X0 (even) or X1 (odd)
        int sel = 0;             // region written by the next FFT pass
        int64_t Ns = 1;
        for (int p = 0; p < np - 1; ++p) {
            FftPass P;
            memset(&P, 0, sizeof(P));
            P.M = M; P.R = rad[p]; P.cols = fft_cols(M, rad[p], Ns, prec, p == 0 ? FFT_COLS_MAX : fft_cap);
            P.nthreads = rad[p] * P.cols / FFT_E;
            P.Ns = Ns;
            P.in_mode = p == 0 ? 1 : 0; P.out_mode = 0; P.inverse = 0;
            P.x_sel = cur; P.with_delta = (p == 0 && it > 0) ? 1 : 0;
            P.src_sel = 1 - sel; P.dst_sel = sel; P.sub = make_plan(rad[p]);
            launch_fft_pass<T>(ctx, d, nc, P, tb, st);
            if (p == 0 && it > 0) {
                // delta of iteration it-1 (x_it against x_{it-1}); may stop the curve
                ProfScope ps(ctx, "delta", st);
                hipLaunchKernelGGL(k_big_delta_final, dim3((unsigned)nc), dim3(BIG_THREADS), 0, st, d, it - 1,
                                   npart0);
            }
            Ns *= rad[p];
            sel = 1 - sel;
        }
        // last forward pass + fold / replacement + first inverse pass
        launch_fft_mid<T, MID_REPLACE>(ctx, d, nc, make_mid(M, rad[np - 1], 1 - sel, sel, prec), tb, st);
        sel = 1 - sel;
        Ns = rad[np - 1];
        for (int p = np - 2; p >= 0; --p) {
            FftPass P;
            memset(&P, 0, sizeof(P));
            P.M = M; P.R = rad[p]; P.cols = fft_cols(M, rad[p], Ns, prec, fft_cap); P.nthreads = rad[p] * P.cols / FFT_E;
            P.Ns = Ns;
            P.in_mode = 0; P.out_mode = (p == 0) ? 1 : 0; P.inverse = 1;
            P.src_sel = 1 - sel; P.dst_sel = sel; P.sub = make_plan(rad[p]);
            launch_fft_pass<T>(ctx, d, nc, P, tb, st);
            Ns *= rad[p];
            sel = 1 - sel;
        }
        // keys are in region (1 - sel)
        run_sort<K>(ctx, d, nc, n, 1 - sel, SORT_MODE_RANK, 1 - cur, sort_tile, &seq, polls, st);
    }
    {
        // delta of the last iteration for curves that ran all of them: the
        // first forward pass's loads and partials without its transform, so
        // that a call that stops here and one that goes on sum the same terms
        // in the same order
        ProfScope ps(ctx, "delta", st);
        FftPass P;
        memset(&P, 0, sizeof(P));
        P.M = M; P.R = rad[0]; P.cols = fft_cols(M, rad[0], 1, prec, FFT_COLS_MAX);
        P.nthreads = rad[0] * P.cols / FFT_E;
        P.Ns = 1;
        P.in_mode = 1; P.out_mode = 2; P.inverse = 0;
        P.x_sel = max_iters & 1; P.with_delta = 1;
        P.src_sel = 1; P.dst_sel = 0; P.sub = make_plan(rad[0]);
        launch_fft_pass<T>(nullptr, d, nc, P, tb, st);
        hipLaunchKernelGGL(k_big_delta_final, dim3((unsigned)nc), dim3(BIG_THREADS), 0, st, d, max_iters - 1,
                           npart0);
    }
    {
        ProfScope ps(ctx, "big_output", st);
        hipLaunchKernelGGL(k_big_output, gt, dim3(BIG_THREADS), 0, st, d);
    }
}

// A batch prepared for launch: descriptors resident in the workspace, one
// launch group per curve length, twiddle tables resolved.  Enqueueing it is
// pure kernel launches (no allocation, copy or host synchronisation), so it
// can be replayed and captured into a HIP graph.
struct LdsGroup {
    int first, count, E, nt;
    int64_t n;
    size_t pl, il;
    // pack launch (one persistent k_lds_packs launch for every LDS length):
    // first/count unused; npacks work items at d_packs, LDS per workgroup, grid
    int npacks = 0;
    const LdsPack* d_packs = nullptr;
    size_t pack_lds = 0;
    int pack_grid = 0;
    std::string lens;  // pack launch: the lengths and curve counts it covers (plan signature)
};
struct BigGroup {
    int first, count;
    int64_t n;
    int32_t max_it;
    TwTable tb;
    std::vector<int> rad;
};

struct agn_batch_plan {
    agn_ctx* ctx = nullptr;
    agn_precision prec = AGN_FP32;
    LcDesc* d_lc = nullptr;
    SpecDesc* d_sp = nullptr;
    BigCurve* d_bg = nullptr;
    int nsp = 0;
    int64_t nchunks = 0;
    std::vector<LdsGroup> lds;
    std::vector<BigGroup> big;
    std::vector<double> lds_cost, big_cost;  // relative run time of each group
    int branches = 1;                         // concurrent launch chains
    int sort_tile = SORT_TILE_AUTO;           // requested tile of 32-bit-key sorts (multi-pass curves;
                                              // SORT_TILE_AUTO: by length)
    int fft_cap = FFT_COLS_MAX;               // most butterflies per multi-pass FFT workgroup
    int look_polls = LOOK_SPIN_MAX;           // look-back wait limit (the context's, at plan build)
    int flags = 0;
    std::vector<hipStream_t> aux;             // chains 1..branches-1 (default priority)
    std::vector<hipEvent_t> ev;               // fork + one join event per chain
    hipStream_t cap = nullptr;                // private stream graphs are captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_branches = 0;                   // chain count the graph was captured with
};

static int build_plan(agn_ctx* ctx, std::vector<CurveReq>& rq, double tol, agn_precision prec,
                      void* ws, size_t ws_bytes, hipStream_t st, agn_batch_plan& pl) {
    const int32_t nc = (int32_t)rq.size();
    pl.ctx = ctx;
    pl.look_polls = ctx->look_polls;
    pl.prec = prec;
    if (nc == 0) return AGN_OK;
    size_t need = header_ws(nc);
    for (auto& r : rq) need += curve_ws(r.n, prec);
    if (!ws || ws_bytes < need)
        return fail(AGN_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    HIPCHK(hipSetDevice(ctx->device));

    // LDS-path curves first, then multi-pass curves; each grouped by length
    // (stable), so that each length is one set of launches.
    std::vector<int> order(nc);
    for (int i = 0; i < nc; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const bool la = lds_path(rq[a].n, prec), lb = lds_path(rq[b].n, prec);
        if (la != lb) return la;
        return rq[a].n < rq[b].n;
    });
    int n_lds = 0;
    while (n_lds < nc && lds_path(rq[order[n_lds]].n, prec)) ++n_lds;

    unsigned char* base = (unsigned char*)ws;
    LcDesc* d_lc = (LcDesc*)base;
    SpecDesc* d_sp = (SpecDesc*)(base + align256(sizeof(LcDesc) * (size_t)nc));
    BigCurve* d_bg = (BigCurve*)(base + align256(sizeof(LcDesc) * (size_t)nc) +
                                 align256(sizeof(SpecDesc) * (size_t)nc));
    std::vector<LcDesc> lc(nc);
    std::vector<BigCurve> bg(nc);
    std::vector<SpecDesc> sp;
    size_t off = header_ws(nc);
    int64_t chunk0 = 0;
    const size_t pb = prec_bytes(prec);
    for (int i = 0; i < nc; ++i) {
        const CurveReq& r = rq[order[i]];
        const int64_t n = r.n, M = n / 2;
        void* amp_ws = nullptr;
        double* partial = nullptr;
        double* A = nullptr;
        if (i < n_lds) {
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
            amp_ws = (void*)(base + off); off += align256((size_t)(M + 1) * pb);
            partial = (double*)(base + off); off += align256((size_t)spec_chunks(n) * 8);
            A = (double*)(base + off); off += align256(8);
            d.x_out = r.x_out;
            d.delta_out = r.delta_out;
            d.iters_done = r.iters_done;
            d.rank_out = r.rank_out;
            const void* tw = nullptr;
            int rc = get_twiddles(ctx, n, AGN_FP64, &tw);
            if (rc) return rc;
            d.tw = tw;
            d.plan = make_plan(M);
            d.amp = r.amp_in ? r.amp_in : amp_ws;
        } else {
            BigCurve& d = bg[i];
            memset(&d, 0, sizeof(d));
            const int64_t ntiles = n / BIG_TILE;
            d.n = n;
            d.iters = r.iters;
            d.tol = tol;
            d.x0 = r.x0;
            d.s64 = (double*)(base + off); off += align256((size_t)n * 8);
            d.X0 = (double*)(base + off); off += align256((size_t)n * 8);
            d.X1 = (double*)(base + off); off += align256((size_t)n * 8);
            d.rankA = (uint32_t*)(base + off); off += align256((size_t)n * 4);
            d.rankB = (uint32_t*)(base + off); off += align256((size_t)n * 4);
            d.sortA = base + off; off += align256((size_t)n * 12);
            d.sortB = base + off; off += align256((size_t)n * 12);
            d.look = (uint32_t*)(base + off); off += align256((size_t)ntiles * 256 * 4);
            d.dcount = (uint32_t*)(base + off); off += align256(SORT_MAX_PASSES * 256 * 4);
            d.dstart = (uint32_t*)(base + off); off += align256(SORT_MAX_PASSES * 256 * 4);
            d.tickets = (uint32_t*)(base + off); off += align256(SORT_MAX_PASSES * 4);
            d.dpart = (double*)(base + off); off += align256((size_t)big_npart(n) * 8);
            d.cpart = (uint32_t*)(base + off); off += align256((size_t)big_npart(n) * 4);
            d.state = (int32_t*)(base + off); off += align256(16);
            amp_ws = (void*)(base + off); off += align256((size_t)(M + 1) * pb);
            partial = (double*)(base + off); off += align256((size_t)spec_chunks(n) * 8);
            A = (double*)(base + off); off += align256(8);
            d.x_out = r.x_out;
            d.delta_out = r.delta_out;
            d.iters_done = r.iters_done;
            d.rank_out = r.rank_out;
            d.amp = r.amp_in ? r.amp_in : amp_ws;
        }
        if (!r.amp_in) {
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
    // Upload descriptors (one copy of the whole header).
    {
        std::vector<unsigned char> hdr(header_ws(nc), 0);
        memcpy(hdr.data(), lc.data(), sizeof(LcDesc) * (size_t)nc);
        if (!sp.empty())
            memcpy(hdr.data() + align256(sizeof(LcDesc) * (size_t)nc), sp.data(), sizeof(SpecDesc) * sp.size());
        memcpy(hdr.data() + align256(sizeof(LcDesc) * (size_t)nc) + align256(sizeof(SpecDesc) * (size_t)nc),
               bg.data(), sizeof(BigCurve) * (size_t)nc);
        int rc = stage_upload(ctx, ws, hdr.data(), hdr.size(), st);
        if (rc) return rc;
    }
    pl.d_lc = d_lc;
    pl.d_sp = d_sp;
    pl.d_bg = d_bg;
    pl.nsp = (int)sp.size();
    pl.nchunks = chunk0;
    // LDS path: one prep + iterate launch per distinct length.
    int i = 0;
    while (i < n_lds) {
        int j = i;
        while (j < n_lds && lc[j].n == lc[i].n) ++j;
        LdsGroup g;
        g.first = i;
        g.count = j - i;
        g.n = lc[i].n;
        g.E = lds_ipt(g.n) / 2;
        g.nt = (int)(g.n / lds_ipt(g.n));
        g.pl = lds_prep_bytes(g.n);
        g.il = lds_iter_bytes(g.n, prec);
        if (g.pl > ctx->lds_max || g.il > ctx->lds_max)
            return fail(AGN_EUNSUPPORTED_N, "n=%lld needs %zu bytes of LDS per workgroup; the device allows %zu",
                        (long long)g.n, std::max(g.pl, g.il), ctx->lds_max);
        int32_t max_it = 0;
        for (int k = i; k < j; ++k) max_it = std::max(max_it, lc[k].iters);
        pl.lds.push_back(g);
        pl.lds_cost.push_back((double)g.count * (double)g.n * (1.0 + max_it));
        i = j;
    }
    // Several LDS-resident lengths, each with at least one whole wave per
    // curve: one persistent launch of packs instead of a launch pair per
    // length (same per-curve arithmetic; bit-identical results).
    // A length packs if a 1024-thread workgroup's worth of its curves (1024 /
    // nt of them) fits the LDS (in FP64 the 3 * 2^k lengths 768, 1536 and 3072
    // do not: they keep their own launches).
    auto pack_stride = [](const LdsGroup& g) { return (std::max(g.pl, g.il) + 15) & ~(size_t)15; };
    auto packable = [&](const LdsGroup& g) {
        return g.nt >= 64 && g.nt <= 1024 && (g.E == 4 || g.E == 6 || g.E == 8) &&
               (size_t)(1024 / g.nt) * pack_stride(g) <= ctx->lds_max;
    };
    int n_packable = 0;
    for (const LdsGroup& g : pl.lds) n_packable += packable(g) ? 1 : 0;
    if (n_packable >= 2) {
        std::vector<LdsPack> packs;
        std::vector<LdsGroup> rest;
        std::vector<double> rest_cost;
        size_t need = 0;
        double cost = 0.0;
        std::string lens;
        int packed_curves = 0;
        for (size_t q = 0; q < pl.lds.size(); ++q) {
            const LdsGroup& g = pl.lds[q];
            if (!packable(g)) {
                rest.push_back(g);
                rest_cost.push_back(pl.lds_cost[q]);
                continue;
            }
            lens += "|L" + std::to_string((long long)g.n) + ":" + std::to_string(g.count);
            packed_curves += g.count;
            const int S = 1024 / g.nt;
            const size_t stride = pack_stride(g);
            need = std::max(need, (size_t)S * stride);
            for (int c0 = 0; c0 < g.count; c0 += S) {
                LdsPack pk;
                memset(&pk, 0, sizeof(pk));
                pk.first = g.first + c0;
                pk.count = std::min(S, g.count - c0);
                pk.E = g.E;
                pk.nt = g.nt;
                pk.fuse2 = lds_fuse2(g.n) ? 1 : 0;
                for (int c = 0; c < pk.count; ++c) pk.max_iters = std::max(pk.max_iters, lc[pk.first + c].iters);
                pk.stride = (uint32_t)stride;
                packs.push_back(pk);
            }
            cost += pl.lds_cost[q];
        }
        {
            std::stable_sort(packs.begin(), packs.end(), [&](const LdsPack& a, const LdsPack& b) {
                return (double)lc[a.first].n * (1.0 + a.max_iters) > (double)lc[b.first].n * (1.0 + b.max_iters);
            });
            LdsPack* d_packs = (LdsPack*)(base + align256(sizeof(LcDesc) * (size_t)nc) +
                                          align256(sizeof(SpecDesc) * (size_t)nc) +
                                          align256(sizeof(BigCurve) * (size_t)nc));
            int rc = stage_upload(ctx, d_packs, packs.data(), sizeof(LdsPack) * packs.size(), st);
            if (rc) return rc;
            LdsGroup g;
            g.first = 0;
            g.count = packed_curves;
            g.E = 0;
            g.nt = 1024;
            g.n = 0;
            g.pl = g.il = need;
            g.npacks = (int)packs.size();
            g.d_packs = d_packs;
            g.pack_lds = need;
            const int per_cu = std::max(1, std::min(2, (int)(ctx->lds_max / need)));
            g.pack_grid = std::min(g.npacks, ctx->ncu * per_cu);
            g.lens = lens;
            pl.lds = rest;
            pl.lds_cost = rest_cost;
            pl.lds.push_back(g);
            pl.lds_cost.push_back(cost);
        }
    }
    // Multi-pass path: one launch sequence per distinct length.
    i = n_lds;
    while (i < nc) {
        int j = i;
        BigGroup g;
        g.max_it = 0;
        while (j < nc && bg[j].n == bg[i].n) { g.max_it = std::max(g.max_it, bg[j].iters); ++j; }
        g.first = i;
        g.count = j - i;
        g.n = bg[i].n;
        int rc = big_group_setup(ctx, g.n, prec, &g.tb, &g.rad);
        if (rc) return rc;
        // per sample-iteration the multi-pass path takes about 3x the LDS path
        pl.big_cost.push_back(3.0 * (double)g.count * (double)g.n * (1.0 + g.max_it));
        pl.big.push_back(std::move(g));
        i = j;
    }
    return AGN_OK;
}

static void enqueue_group(const agn_batch_plan& pl, agn_ctx* pctx, bool is_big, int k, hipStream_t st) {
    if (!is_big) {
        const LdsGroup& g = pl.lds[k];
        if (g.npacks > 0) {
            ProfScope ps(pctx, "lds_packs", st);
            if (pl.prec == AGN_FP32)
                hipLaunchKernelGGL(k_lds_packs<float>, dim3((unsigned)g.pack_grid), dim3(1024), g.pack_lds, st,
                                   pl.d_lc, g.d_packs, g.npacks);
            else
                hipLaunchKernelGGL(k_lds_packs<double>, dim3((unsigned)g.pack_grid), dim3(1024), g.pack_lds, st,
                                   pl.d_lc, g.d_packs, g.npacks);
            return;
        }
        const bool f2 = lds_fuse2(g.n);
        if (pl.prec == AGN_FP32) launch_lds_E<float>(pctx, g.E, pl.d_lc + g.first, g.count, g.nt, f2, g.pl, g.il, st);
        else launch_lds_E<double>(pctx, g.E, pl.d_lc + g.first, g.count, g.nt, f2, g.pl, g.il, st);
    } else {
        const BigGroup& g = pl.big[k];
        if (pl.prec == AGN_FP32)
            run_big_group<float>(pctx, pl.d_bg + g.first, g.count, g.n, g.max_it, g.tb, g.rad, pl.sort_tile,
                                 pl.fft_cap, pl.look_polls, st);
        else
            run_big_group<double>(pctx, pl.d_bg + g.first, g.count, g.n, g.max_it, g.tb, g.rad, pl.sort_tile,
                                  pl.fft_cap, pl.look_polls, st);
    }
}

// Launches the plan's kernels on st; with more than one chain the groups are
// dealt to the chains longest first (each to the least loaded chain) and the
// chains fork from and join back into st.  pctx NULL: no kernel timing.
static int enqueue_plan(agn_batch_plan& pl, agn_ctx* pctx, int branches, hipStream_t st) {
    if (pl.nsp > 0) launch_spectrum(pctx, pl.d_sp, pl.nsp, pl.nchunks, st);
    const int ng = (int)(pl.lds.size() + pl.big.size());
    branches = std::max(1, std::min(branches, ng));
    if (branches == 1) {
        for (int k = 0; k < (int)pl.lds.size(); ++k) enqueue_group(pl, pctx, false, k, st);
        for (int k = 0; k < (int)pl.big.size(); ++k) enqueue_group(pl, pctx, true, k, st);
        HIPCHK(hipGetLastError());
        return AGN_OK;
    }
    while ((int)pl.aux.size() < branches - 1) {
        hipStream_t s = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        pl.aux.push_back(s);
    }
    while ((int)pl.ev.size() < branches) {
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        pl.ev.push_back(e);
    }
    std::vector<std::pair<double, int>> order;  // (cost, group id; big groups offset by nlds)
    const int nl = (int)pl.lds.size();
    for (int k = 0; k < nl; ++k) order.push_back({pl.lds_cost[k], k});
    for (int k = 0; k < (int)pl.big.size(); ++k) order.push_back({pl.big_cost[k], nl + k});
    std::stable_sort(order.begin(), order.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        return a.first > b.first;
    });
    std::vector<double> load(branches, 0.0);
    std::vector<std::vector<int>> chain(branches);
    for (auto& o : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += o.first;
        chain[b].push_back(o.second);
    }
    HIPCHK(hipEventRecord(pl.ev[0], st));
    for (int b = 1; b < branches; ++b) HIPCHK(hipStreamWaitEvent(pl.aux[b - 1], pl.ev[0], 0));
    for (int b = 0; b < branches; ++b) {
        hipStream_t s = b == 0 ? st : pl.aux[b - 1];
        for (int g : chain[b]) enqueue_group(pl, pctx, g >= nl, g >= nl ? g - nl : g, s);
    }
    HIPCHK(hipGetLastError());
    for (int b = 1; b < branches; ++b) {
        HIPCHK(hipEventRecord(pl.ev[b], pl.aux[b - 1]));
        HIPCHK(hipStreamWaitEvent(st, pl.ev[b], 0));
    }
    return AGN_OK;
}

static void destroy_plan_resources(agn_batch_plan& pl) {
    if (pl.exec) (void)hipGraphExecDestroy(pl.exec);
    if (pl.graph) (void)hipGraphDestroy(pl.graph);
    pl.exec = nullptr;
    pl.graph = nullptr;
    for (hipStream_t s : pl.aux) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
    for (hipEvent_t e : pl.ev) (void)hipEventDestroy(e);
    if (pl.cap) (void)hipStreamDestroy(pl.cap);
    pl.aux.clear();
    pl.ev.clear();
    pl.cap = nullptr;
}

static int run_batch(agn_ctx* ctx, std::vector<CurveReq>& rq, double tol, agn_precision prec,
                     void* ws, size_t ws_bytes, hipStream_t st) {
    if (rq.empty()) return AGN_OK;
    agn_batch_plan pl;
    int rc = build_plan(ctx, rq, tol, prec, ws, ws_bytes, st, pl);
    if (rc) return rc;
    return enqueue_plan(pl, ctx, 1, st);
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

// The descriptor of a spectrum launch, written from a kernel argument into
// device memory (no host staging buffer).  grid 1, block 64.
__global__ void k_put_spec_desc(SpecDesc s, SpecDesc* __restrict__ dst) {
    if (threadIdx.x == 0) *dst = s;
}

extern "C" int agn_psd_spectrum_noalloc(agn_ctx* ctx, const agn_psd_params* p, int64_t n, double dt,
                                        uint64_t seed, uint32_t curve_id, agn_precision prec, void* amp_out,
                                        void* stream) {
    if (!ctx || !p || !amp_out) return fail(AGN_EINVAL, "NULL argument");
    int rc = check_prec(prec);
    if (rc) return rc;
    if (!n_supported(n)) return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [2, 2^27]", (long long)n);
    if (!valid_params(p, dt)) return fail(AGN_EINVAL, "invalid PSD parameters or dt");
    if (!ctx->scratch_dev) return fail(AGN_EDEVICE, "the scratch array's device address is unknown");
    const size_t need = align256(sizeof(SpecDesc)) + spectrum_ws(n);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(AGN_EUNSUPPORTED_N, "n=%lld needs %zu bytes of scratch; the array holds %zu", (long long)n, need,
                    NOALLOC_SCRATCH_BYTES);
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    unsigned char* base = (unsigned char*)ctx->scratch_dev;
    SpecDesc s;
    memset(&s, 0, sizeof(s));
    s.n = n; s.dt = dt; s.norm = p->norm; s.f_br = p->f_br; s.a_low = p->a_low; s.a_high = p->a_high;
    s.seed = seed; s.curve_id = curve_id; s.is_f32 = prec == AGN_FP32;
    s.chunk0 = 0; s.nchunk = spec_chunks(n);
    s.amp = amp_out;
    s.partial = (double*)(base + align256(sizeof(SpecDesc)));
    s.A = (double*)(base + align256(sizeof(SpecDesc)) + align256((size_t)s.nchunk * 8));
    SpecDesc* d_sp = (SpecDesc*)base;
    hipLaunchKernelGGL(k_put_spec_desc, dim3(1), dim3(64), 0, st, s, d_sp);
    launch_spectrum(nullptr, d_sp, 1, s.nchunk, st);  // no kernel timing: its events would be allocations
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

static int batch_requests(int32_t n_curves, const int64_t* n, const int64_t* offset, const agn_psd_params* p,
                          const double* dt, const int32_t* iters, const uint64_t* seed, const uint32_t* curve_id,
                          const double* erdf, double tol, agn_precision prec, double* x_out, double* delta_out,
                          int32_t* iters_done, std::vector<CurveReq>& rq) {
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
    rq.resize(n_curves);
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
    return AGN_OK;
}

extern "C" int agn_lc_generate_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n,
                                     const int64_t* offset, const agn_psd_params* p, const double* dt,
                                     const int32_t* iters, const uint64_t* seed,
                                     const uint32_t* curve_id, const double* erdf, double tol,
                                     agn_precision prec, double* x_out, double* delta_out,
                                     int32_t* iters_done, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    std::vector<CurveReq> rq;
    int rc = batch_requests(n_curves, n, offset, p, dt, iters, seed, curve_id, erdf, tol, prec, x_out, delta_out,
                            iters_done, rq);
    if (rc) return rc;
    return run_batch(ctx, rq, tol, prec, ws, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// batch plans: build once, launch many times (optionally as a HIP graph)
// ---------------------------------------------------------------------------
static std::string plan_signature(const agn_batch_plan& pl) {
    std::string sig = pl.prec == AGN_FP32 ? "f32" : "f64";
    char buf[96];
    for (const auto& g : pl.lds) {
        if (g.npacks > 0) {
            sig += "|packs" + g.lens;
            continue;
        }
        snprintf(buf, sizeof(buf), "|L%lld:%d", (long long)g.n, g.count);
        sig += buf;
    }
    for (const auto& g : pl.big) {
        snprintf(buf, sizeof(buf), "|B%lld:%d", (long long)g.n, g.count);
        sig += buf;
    }
    return sig;
}

// Times each candidate (chain count, sort tile) on a copy of the batch with at
// most two iterations per curve (same workspace, so the real plan is built
// after it) and returns the fastest.  Both choices leave every result
// bit-identical.  Synchronises st.
static int autotune_plan(agn_ctx* ctx, std::vector<CurveReq> rq, double tol, agn_precision prec, void* ws,
                         size_t ws_bytes, hipStream_t st, int* best_branches, int* best_tile, int* best_cap) {
    for (auto& r : rq) {
        r.iters = std::min(r.iters, 2);
        r.delta_out = nullptr;  // the real plan's delta rows are laid out for its own iteration count
    }
    agn_batch_plan tp;
    int rc = build_plan(ctx, rq, tol, prec, ws, ws_bytes, st, tp);
    if (rc) { destroy_plan_resources(tp); return rc; }
    const int ng = (int)(tp.lds.size() + tp.big.size());
    bool big_tile_ok = false;  // some 32-bit-key group whose length the larger tile divides
    for (const auto& g : tp.big)
        if (prec == AGN_FP32 && g.n % SORT_TILE_BIG == 0) big_tile_ok = true;
    const int cand[3] = {1, 2, 4};
    const int tiles[2] = {BIG_TILE, SORT_TILE_BIG};
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    float best_ms = 0.f;
    bool have = false;
    *best_branches = 1;
    *best_tile = BIG_TILE;
    *best_cap = FFT_COLS_MAX;
    rc = AGN_OK;
    // best of three launches after a warm-up one
    auto time_plan = [&](int nb, float* out_ms) -> int {
        float m = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            if (hipEventRecord(a, st) != hipSuccess) return fail(AGN_EDEVICE, "event record failed");
            int r2 = enqueue_plan(tp, nullptr, nb, st);
            if (r2) return r2;
            if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess)
                return fail(AGN_EDEVICE, "event wait failed");
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (rep == 1 || (rep == 2 && ms < m)) m = ms;
        }
        *out_ms = m;
        return AGN_OK;
    };
    for (int ti = 0; ti < 2 && rc == AGN_OK; ++ti) {
        if (ti == 1 && !big_tile_ok) break;
        tp.sort_tile = tiles[ti];
        for (int ci = 0; ci < 3 && rc == AGN_OK; ++ci) {
            if (cand[ci] > 1 && cand[ci] > ng) break;
            float m = 0.f;
            rc = time_plan(cand[ci], &m);
            if (rc == AGN_OK && (!have || m < best_ms)) {
                best_ms = m;
                *best_branches = cand[ci];
                *best_tile = tiles[ti];
                have = true;
            }
        }
    }
    // then the FFT workgroup width at that choice (multi-pass groups only)
    if (rc == AGN_OK && !tp.big.empty()) {
        tp.sort_tile = *best_tile;
        for (int cap = FFT_COLS_MAX / 2; cap >= FFT_COLS_MIN && rc == AGN_OK; cap >>= 1) {
            tp.fft_cap = cap;
            float m = 0.f;
            rc = time_plan(*best_branches, &m);
            if (rc == AGN_OK && m < best_ms) {
                best_ms = m;
                *best_cap = cap;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    destroy_plan_resources(tp);
    return rc;
}

extern "C" int agn_batch_plan_create(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const int64_t* offset,
                                     const agn_psd_params* p, const double* dt, const int32_t* iters,
                                     const uint64_t* seed, const uint32_t* curve_id, const double* erdf,
                                     double tol, agn_precision prec, double* x_out, double* delta_out,
                                     int32_t* iters_done, int flags, int branches, void* ws, size_t ws_bytes,
                                     void* stream, agn_batch_plan** out) {
    if (!ctx || !out) return fail(AGN_EINVAL, "NULL argument");
    *out = nullptr;
    if (flags & ~(AGN_PLAN_GRAPH | AGN_PLAN_AUTOTUNE | AGN_PLAN_LARGE_SORT_TILE | AGN_PLAN_NARROW_FFT))
        return fail(AGN_EINVAL, "unknown plan flags 0x%x", flags);
    if ((flags & AGN_PLAN_AUTOTUNE) && (flags & AGN_PLAN_LARGE_SORT_TILE))
        return fail(AGN_EINVAL, "AGN_PLAN_LARGE_SORT_TILE fixes the tile that AGN_PLAN_AUTOTUNE would choose");
    if ((flags & AGN_PLAN_AUTOTUNE) && (flags & AGN_PLAN_NARROW_FFT))
        return fail(AGN_EINVAL, "AGN_PLAN_NARROW_FFT fixes the FFT width that AGN_PLAN_AUTOTUNE would choose");
    if (branches < 0 || branches > 8) return fail(AGN_EINVAL, "branches must be 0..8");
    std::vector<CurveReq> rq;
    int rc = batch_requests(n_curves, n, offset, p, dt, iters, seed, curve_id, erdf, tol, prec, x_out, delta_out,
                            iters_done, rq);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<agn_batch_plan> pl(new agn_batch_plan());
    pl->flags = flags;
    if ((rc = build_plan(ctx, rq, tol, prec, ws, ws_bytes, st, *pl))) { destroy_plan_resources(*pl); return rc; }
    int nb = branches > 0 ? branches : 1;
    int tile = (flags & AGN_PLAN_LARGE_SORT_TILE) ? SORT_TILE_BIG : SORT_TILE_AUTO;
    int cap = (flags & AGN_PLAN_NARROW_FFT) ? FFT_COLS_MIN : FFT_COLS_MAX;
    if ((flags & AGN_PLAN_AUTOTUNE) && !rq.empty()) {
        const std::string sig = plan_signature(*pl);
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            auto it = ctx->tuned.find(sig);
            if (it != ctx->tuned.end()) {
                nb = it->second[0];
                tile = it->second[1];
                cap = it->second[2];
                hit = true;
            }
        }
        if (!hit) {
            if ((rc = autotune_plan(ctx, rq, tol, prec, ws, ws_bytes, st, &nb, &tile, &cap))) {
                destroy_plan_resources(*pl);
                return rc;
            }
            // the tuning runs overwrote the descriptors: build the real plan again
            destroy_plan_resources(*pl);
            pl.reset(new agn_batch_plan());
            pl->flags = flags;
            if ((rc = build_plan(ctx, rq, tol, prec, ws, ws_bytes, st, *pl))) {
                destroy_plan_resources(*pl);
                return rc;
            }
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->tuned[sig] = {nb, tile, cap};
        }
    }
    pl->branches = nb;
    pl->sort_tile = tile;
    pl->fft_cap = cap;
    *out = pl.release();
    return AGN_OK;
}

extern "C" int agn_batch_plan_launch(agn_batch_plan* pl, void* stream) {
    if (!pl) return fail(AGN_EINVAL, "plan is NULL");
    hipStream_t st = (hipStream_t)stream;
    agn_ctx* ctx = pl->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    if (!(pl->flags & AGN_PLAN_GRAPH)) return enqueue_plan(*pl, ctx, pl->branches, st);
    if (!pl->exec || pl->graph_branches != pl->branches) {
        if (pl->exec) { (void)hipGraphExecDestroy(pl->exec); pl->exec = nullptr; }
        if (pl->graph) { (void)hipGraphDestroy(pl->graph); pl->graph = nullptr; }
        if (!pl->cap) HIPCHK(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_plan(*pl, nullptr, pl->branches, pl->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(pl->cap, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return fail(AGN_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        pl->graph = g;
        HIPCHK(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0));
        pl->graph_branches = pl->branches;
    }
    {
        ProfScope ps(ctx, "batch_graph", st);
        HIPCHK(hipGraphLaunch(pl->exec, st));
    }
    return AGN_OK;
}

extern "C" int agn_batch_plan_info(const agn_batch_plan* pl, int32_t* branches, int32_t* groups,
                                   int32_t* uses_graph) {
    if (!pl) return fail(AGN_EINVAL, "plan is NULL");
    if (branches) *branches = pl->branches;
    if (groups) *groups = (int32_t)(pl->lds.size() + pl->big.size());
    if (uses_graph) *uses_graph = (pl->flags & AGN_PLAN_GRAPH) ? 1 : 0;
    return AGN_OK;
}

extern "C" int agn_batch_plan_tuning(const agn_batch_plan* pl, int32_t* branches, int32_t* sort_tile,
                                     int32_t* fft_cols) {
    if (!pl) return fail(AGN_EINVAL, "plan is NULL");
    if (branches) *branches = pl->branches;
    if (sort_tile) *sort_tile = pl->sort_tile;
    if (fft_cols) *fft_cols = pl->fft_cap;
    return AGN_OK;
}

extern "C" int agn_batch_plan_destroy(agn_batch_plan* pl) {
    if (!pl) return AGN_OK;
    (void)hipSetDevice(pl->ctx ? pl->ctx->device : 0);
    destroy_plan_resources(*pl);
    delete pl;
    return AGN_OK;
}

// ---------------------------------------------------------------------------
// observables after the path: periodogram (Eq. A2) and log-binned means
// ---------------------------------------------------------------------------
static bool pg_lds(int64_t n) {
    if (!n_supported(n)) return false;
    return (n % 3 == 0) ? n <= 12288 : n <= 16384;
}

// Bin of j >= 1: floor(log10(j) / dex + 1e-9); non-empty bins in increasing j.
static int64_t bin_of(int64_t j, double dex) { return (int64_t)std::floor(std::log10((double)j) / dex + 1e-9); }

static void log_bin_edges(int64_t n, double dex, std::vector<int64_t>* edges) {
    edges->clear();
    const int64_t h = n / 2;
    int64_t j = 1;
    while (j <= h) {
        const int64_t b = bin_of(j, dex);
        // first j' > j in a later bin: start below the estimate, step to it
        int64_t g = (int64_t)std::ceil(std::pow(10.0, (double)(b + 1) * dex)) - 2;
        if (g <= j) g = j + 1;
        while (g > j + 1 && bin_of(g - 1, dex) > b) --g;
        while (g <= h && bin_of(g, dex) <= b) ++g;
        if (g > h + 1) g = h + 1;
        edges->push_back(j);
        edges->push_back(g);
        j = g;
    }
}

extern "C" int agn_log_bin_count(int64_t n, double dex, int32_t* count) {
    if (!count) return fail(AGN_EINVAL, "count is NULL");
    if (!n_supported(n)) return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [2, 2^27]", (long long)n);
    if (!(dex > 0.0) || !std::isfinite(dex)) return fail(AGN_EINVAL, "dex must be finite and > 0");
    std::vector<int64_t> e;
    log_bin_edges(n, dex, &e);
    *count = (int32_t)(e.size() / 2);
    return AGN_OK;
}

static size_t pg_header_ws(int32_t nc) {
    return align256(sizeof(PgDesc) * (size_t)nc) + align256(sizeof(BigCurve) * (size_t)nc) +
           align256(sizeof(BinDesc) * (size_t)nc) + align256(sizeof(double*) * (size_t)nc);
}

// Bin edges per distinct length within one call (batches repeat lengths).
struct EdgeCache {
    double dex;
    std::map<int64_t, std::vector<int64_t>> by_n;
    const std::vector<int64_t>& get(int64_t n) {
        auto it = by_n.find(n);
        if (it == by_n.end()) {
            it = by_n.emplace(n, std::vector<int64_t>()).first;
            log_bin_edges(n, dex, &it->second);
        }
        return it->second;
    }
};

static size_t pg_curve_ws(int64_t n, double dex, EdgeCache* ec) {
    size_t b = 0;
    if (!pg_lds(n)) b += 2 * align256((size_t)n * 8) + align256(16);  // FFT ping-pong + state
    if (dex > 0.0) b += align256(ec->get(n).size() * sizeof(int64_t));
    return b;
}

extern "C" int agn_periodogram_workspace_size(int32_t n_curves, const int64_t* n, double dex, size_t* bytes) {
    if (!bytes || (n_curves > 0 && !n)) return fail(AGN_EINVAL, "NULL argument");
    if (n_curves < 0) return fail(AGN_EINVAL, "n_curves < 0");
    size_t b = pg_header_ws(n_curves);
    EdgeCache ec;
    ec.dex = dex;
    for (int32_t c = 0; c < n_curves; ++c) {
        if (!n_supported(n[c]) || n[c] < 4)
            return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [4, 2^27]", (long long)n[c]);
        b += pg_curve_ws(n[c], dex, &ec);
    }
    *bytes = b;
    return AGN_OK;
}

template <int E>
static void launch_pg(const PgDesc* d, int count, int nt, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((k_lds_periodogram<E>), dim3(count), dim3(nt), lds, st, d);
}

extern "C" int agn_periodogram_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const int64_t* offset,
                                     const double* x, const int64_t* p_offset, double* P_out, double dex,
                                     const int64_t* b_offset, double* bins_out, void* ws, size_t ws_bytes,
                                     void* stream) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    if (n_curves < 0) return fail(AGN_EINVAL, "n_curves < 0");
    if (n_curves == 0) return AGN_OK;
    if (!n || !offset || !x || !p_offset || !P_out) return fail(AGN_EINVAL, "NULL argument");
    if (bins_out && (!b_offset || !(dex > 0.0) || !std::isfinite(dex)))
        return fail(AGN_EINVAL, "bins_out needs b_offset and a finite dex > 0");
    const double dx = bins_out ? dex : 0.0;
    size_t need = 0;
    int rc = agn_periodogram_workspace_size(n_curves, n, dx, &need);
    if (rc) return rc;
    if (!ws || ws_bytes < need)
        return fail(AGN_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    for (int32_t c = 0; c < n_curves; ++c) {
        if (offset[c] < 0 || p_offset[c] < 0 || (bins_out && b_offset[c] < 0))
            return fail(AGN_EINVAL, "negative offset for curve %d", c);
        if (offset[c] & 1) return fail(AGN_EINVAL, "offset[%d] must be even", c);
    }
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    const int32_t nc = n_curves;
    std::vector<int> order(nc);
    for (int i = 0; i < nc; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const bool la = pg_lds(n[a]), lb = pg_lds(n[b]);
        if (la != lb) return la;
        return n[a] < n[b];
    });
    unsigned char* base = (unsigned char*)ws;
    PgDesc* d_pg = (PgDesc*)base;
    BigCurve* d_bg = (BigCurve*)(base + align256(sizeof(PgDesc) * (size_t)nc));
    BinDesc* d_bd = (BinDesc*)((unsigned char*)d_bg + align256(sizeof(BigCurve) * (size_t)nc));
    double** d_pp = (double**)((unsigned char*)d_bd + align256(sizeof(BinDesc) * (size_t)nc));
    std::vector<PgDesc> pg(nc);
    std::vector<BigCurve> bg(nc);
    std::vector<BinDesc> bd(nc);
    std::vector<double*> pp(nc);
    EdgeCache ec;
    ec.dex = dex;
    std::vector<const std::vector<int64_t>*> edges(nc, nullptr);
    size_t off = pg_header_ws(nc);
    int32_t maxbins = 0;
    int n_lds = 0;
    for (int i = 0; i < nc; ++i) {
        const int c = order[i];
        const int64_t nn = n[c];
        memset(&pg[i], 0, sizeof(PgDesc));
        memset(&bg[i], 0, sizeof(BigCurve));
        memset(&bd[i], 0, sizeof(BinDesc));
        pp[i] = P_out + p_offset[c];
        if (pg_lds(nn)) {
            ++n_lds;
            pg[i].n = (int32_t)nn;
            pg[i].x = x + offset[c];
            pg[i].P = P_out + p_offset[c];
            const void* tw = nullptr;
            if ((rc = get_twiddles(ctx, nn, AGN_FP64, &tw))) return rc;
            pg[i].tw = tw;
            pg[i].plan = make_plan(nn / 2);
        } else {
            BigCurve& b = bg[i];
            b.n = nn;
            b.X0 = const_cast<double*>(x + offset[c]);  // read only (in_mode 1 of the first pass)
            b.sortA = base + off; off += align256((size_t)nn * 8);
            b.sortB = base + off; off += align256((size_t)nn * 8);
            b.state = (int32_t*)(base + off); off += align256(16);
        }
        if (bins_out) {
            edges[i] = &ec.get(nn);
            bd[i].P = P_out + p_offset[c];
            bd[i].out = bins_out + b_offset[c];
            bd[i].edges = (const int64_t*)(base + off);
            bd[i].nbins = (int32_t)(edges[i]->size() / 2);
            maxbins = std::max(maxbins, bd[i].nbins);
            off += align256(edges[i]->size() * sizeof(int64_t));
        }
    }
    // one upload: header, then the bin edges
    {
        std::vector<unsigned char> hdr(off, 0);
        memcpy(hdr.data(), pg.data(), sizeof(PgDesc) * (size_t)nc);
        memcpy(hdr.data() + ((unsigned char*)d_bg - base), bg.data(), sizeof(BigCurve) * (size_t)nc);
        memcpy(hdr.data() + ((unsigned char*)d_bd - base), bd.data(), sizeof(BinDesc) * (size_t)nc);
        memcpy(hdr.data() + ((unsigned char*)d_pp - base), pp.data(), sizeof(double*) * (size_t)nc);
        for (int i = 0; i < nc; ++i)
            if (bins_out && edges[i] && !edges[i]->empty())
                memcpy(hdr.data() + ((const unsigned char*)bd[i].edges - base), edges[i]->data(),
                       edges[i]->size() * sizeof(int64_t));
        if ((rc = stage_upload(ctx, ws, hdr.data(), hdr.size(), st))) return rc;
    }
    {
        ProfScope ps(ctx, "periodogram", st);
        int i = 0;
        while (i < n_lds) {
            int j = i;
            while (j < n_lds && pg[j].n == pg[i].n) ++j;
            const int64_t nn = pg[i].n;
            const int E = lds_ipt(nn) / 2, nt = (int)(nn / lds_ipt(nn));
            const size_t lds = lds_pg_layout((int)nn, nullptr);
            if (lds > ctx->lds_max) return fail(AGN_EUNSUPPORTED_N, "n=%lld: LDS too small", (long long)nn);
            switch (E) {
                case 1: launch_pg<1>(d_pg + i, j - i, nt, lds, st); break;
                case 2: launch_pg<2>(d_pg + i, j - i, nt, lds, st); break;
                case 3: launch_pg<3>(d_pg + i, j - i, nt, lds, st); break;
                case 4: launch_pg<4>(d_pg + i, j - i, nt, lds, st); break;
                case 6: launch_pg<6>(d_pg + i, j - i, nt, lds, st); break;
                case 8: launch_pg<8>(d_pg + i, j - i, nt, lds, st); break;
                default: return fail(AGN_EINVAL, "internal: no kernel for E=%d", E);
            }
            i = j;
        }
        while (i < nc) {
            int j = i;
            while (j < nc && bg[j].n == bg[i].n) ++j;
            const int64_t nn = bg[i].n, M = nn / 2;
            TwTable tb;
            std::vector<int> rad;
            if ((rc = big_group_setup(ctx, nn, AGN_FP64, &tb, &rad))) return rc;
            hipLaunchKernelGGL(k_big_init, dim3((unsigned)(j - i)), dim3(64), 0, st, d_bg + i);
            int sel = 0;
            int64_t Ns = 1;
            for (size_t p = 0; p < rad.size(); ++p) {
                FftPass P;
                memset(&P, 0, sizeof(P));
                P.M = M; P.R = rad[p]; P.cols = fft_cols(M, rad[p], Ns, AGN_FP64); P.nthreads = rad[p] * P.cols / FFT_E;
                P.Ns = Ns;
                P.in_mode = p == 0 ? 1 : 0; P.out_mode = 0; P.inverse = 0;
                P.x_sel = 0; P.with_delta = 0;
                P.src_sel = 1 - sel; P.dst_sel = sel; P.sub = make_plan(rad[p]);
                launch_fft_pass<double>(nullptr, d_bg + i, j - i, P, tb, st);
                Ns *= rad[p];
                sel = 1 - sel;
            }
            hipLaunchKernelGGL(k_big_fold_power, dim3((unsigned)((M / 2 + 1 + 255) / 256), (unsigned)(j - i)),
                               dim3(256), 0, st, d_bg + i, M, 1 - sel, tb, d_pp + i);
            i = j;
        }
    }
    HIPCHK(hipGetLastError());
    if (bins_out && maxbins > 0) {
        ProfScope ps(ctx, "log_bins", st);
        hipLaunchKernelGGL(k_log_bins, dim3((unsigned)maxbins, (unsigned)nc), dim3(256), 0, st, d_bd);
        HIPCHK(hipGetLastError());
    }
    return AGN_OK;
}

// ---------------------------------------------------------------------------
// fit of Eq. 3 to log-binned periodograms (convergence test)
// ---------------------------------------------------------------------------
static size_t fit_layout(int32_t nc, const int64_t* n, double dex, EdgeCache* ec, std::vector<size_t>* f_off) {
    size_t off = align256(sizeof(FitDesc) * (size_t)nc);
    f_off->assign((size_t)nc, 0);
    for (int32_t c = 0; c < nc; ++c) {
        (*f_off)[c] = off;
        off += align256(sizeof(double) * (ec->get(n[c]).size() / 2));
    }
    return off;
}

extern "C" int agn_psd_fit_workspace_size(int32_t n_curves, const int64_t* n, double dex, size_t* bytes) {
    if (!bytes || (n_curves > 0 && !n)) return fail(AGN_EINVAL, "NULL argument");
    if (n_curves < 0) return fail(AGN_EINVAL, "n_curves < 0");
    if (!(dex > 0.0) || !std::isfinite(dex)) return fail(AGN_EINVAL, "dex must be finite and > 0");
    for (int32_t c = 0; c < n_curves; ++c)
        if (!n_supported(n[c]) || n[c] < 4)
            return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [4, 2^27]", (long long)n[c]);
    EdgeCache ec;
    ec.dex = dex;
    std::vector<size_t> f_off;
    *bytes = fit_layout(n_curves, n, dex, &ec, &f_off);
    return AGN_OK;
}

extern "C" int agn_psd_fit_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const double* dt,
                                 const agn_psd_params* p, double dex, const int64_t* b_offset, const double* bins,
                                 double* fit_out, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    if (n_curves < 0) return fail(AGN_EINVAL, "n_curves < 0");
    if (n_curves == 0) return AGN_OK;
    if (!n || !dt || !p || !b_offset || !bins || !fit_out) return fail(AGN_EINVAL, "NULL argument");
    size_t need = 0;
    int rc = agn_psd_fit_workspace_size(n_curves, n, dex, &need);
    if (rc) return rc;
    if (!ws || ws_bytes < need)
        return fail(AGN_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    EdgeCache ec;
    ec.dex = dex;
    std::vector<size_t> f_off;
    fit_layout(n_curves, n, dex, &ec, &f_off);
    std::vector<unsigned char> hdr(need, 0);
    FitDesc* fd = (FitDesc*)hdr.data();
    unsigned char* base = (unsigned char*)ws;
    for (int32_t c = 0; c < n_curves; ++c) {
        if (!(dt[c] > 0.0) || !std::isfinite(dt[c])) return fail(AGN_EINVAL, "dt[%d] must be finite and > 0", c);
        if (!(p[c].f_br > 0.0) || !std::isfinite(p[c].f_br) || !std::isfinite(p[c].a_low) ||
            !std::isfinite(p[c].a_high))
            return fail(AGN_EINVAL, "invalid PSD parameters for curve %d", c);
        if (b_offset[c] < 0) return fail(AGN_EINVAL, "b_offset[%d] < 0", c);
        const std::vector<int64_t>& e = ec.get(n[c]);
        const int nb = (int)(e.size() / 2);
        double* fc = (double*)(hdr.data() + f_off[c]);
        int below = 0, above = 0;
        for (int b = 0; b < nb; ++b) {
            // mean of f_j = j / (n dt) over the bin's j in [lo, hi)
            fc[b] = 0.5 * (double)(e[2 * b] + e[2 * b + 1] - 1) / ((double)n[c] * dt[c]);
            below += fc[b] < p[c].f_br;
            above += fc[b] > p[c].f_br;
        }
        if (below < 1 || above < 1)
            return fail(AGN_EINVAL, "curve %d: f_br must lie inside the binned frequency range", c);
        fd[c].f = (const double*)(base + f_off[c]);
        fd[c].pbar = bins + b_offset[c];
        fd[c].out = fit_out + 4 * (int64_t)c;
        fd[c].f_br = p[c].f_br;
        fd[c].a_low0 = p[c].a_low;
        fd[c].a_high0 = p[c].a_high;
        fd[c].nb = nb;
    }
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    if ((rc = stage_upload(ctx, ws, hdr.data(), hdr.size(), st))) return rc;
    {
        ProfScope ps(ctx, "psd_fit", st);
        hipLaunchKernelGGL(k_psd_fit, dim3((unsigned)n_curves), dim3(64), 0, st, (const FitDesc*)ws, n_curves);
    }
    HIPCHK(hipGetLastError());
    return AGN_OK;
}

// ---------------------------------------------------------------------------
// lag statistics: structure function (Eq. A6), Eq. 6 mean, |dm| counts
// ---------------------------------------------------------------------------
struct LagLayout {
    size_t curves, lags, pre, part_sum, part_cnt, sf2, mag, total;
    int64_t blocks;
};

static int lag_layout(int32_t nc, const int64_t* n, int32_t K, const int64_t* lags, int32_t J, int32_t units,
                      std::vector<int64_t>* pre, std::vector<size_t>* mag_off, LagLayout* L) {
    if (nc < 0 || K < 0 || J < 0) return fail(AGN_EINVAL, "negative count");
    if (nc > 0 && !n) return fail(AGN_EINVAL, "n is NULL");
    if (K > 0 && !lags) return fail(AGN_EINVAL, "lags is NULL");
    if (J > LAG_MAX_THR) return fail(AGN_EINVAL, "at most %d thresholds", LAG_MAX_THR);
    if (units != AGN_SF_LINEAR && units != AGN_SF_MAGNITUDE) return fail(AGN_EINVAL, "unknown units");
    if ((int64_t)nc * K > (int64_t)INT32_MAX / 2) return fail(AGN_EINVAL, "too many (curve, lag) items");
    pre->assign((size_t)nc * K + 1, 0);
    int64_t g = 0;
    for (int32_t c = 0; c < nc; ++c) {
        if (n[c] < 2) return fail(AGN_EINVAL, "n[%d] = %lld < 2", c, (long long)n[c]);
        for (int32_t l = 0; l < K; ++l) {
            if (lags[l] < 1 || lags[l] >= n[c])
                return fail(AGN_EINVAL, "lag %lld outside [1, n - 1] for curve %d (n = %lld)", (long long)lags[l], c,
                            (long long)n[c]);
            (*pre)[(size_t)c * K + l] = g;
            const int64_t P = n[c] - lags[l];
            g += std::min<int64_t>((P + LAG_CHUNK - 1) / LAG_CHUNK, LAG_MAX_BLOCKS);
        }
    }
    (*pre)[(size_t)nc * K] = g;
    const size_t items = (size_t)nc * K;
    L->blocks = g;
    L->curves = 0;
    L->lags = L->curves + align256(sizeof(LagCurve) * (size_t)nc);
    L->pre = L->lags + align256(sizeof(int64_t) * (size_t)K);
    L->part_sum = L->pre + align256(sizeof(int64_t) * (items + 1));
    L->part_cnt = L->part_sum + align256(sizeof(double) * (size_t)g);
    L->sf2 = L->part_cnt + align256(sizeof(uint32_t) * (size_t)g * (size_t)(1 + J));
    L->mag = L->sf2 + align256(sizeof(double) * items);
    L->total = L->mag;
    mag_off->assign((size_t)nc, 0);
    if (units == AGN_SF_MAGNITUDE)
        for (int32_t c = 0; c < nc; ++c) {
            (*mag_off)[c] = L->total;
            L->total += align256(sizeof(double) * (size_t)n[c]);
        }
    return AGN_OK;
}

extern "C" int agn_lag_stats_workspace_size(int32_t n_curves, const int64_t* n, int32_t n_lags, const int64_t* lags,
                                            int32_t n_thr, int32_t units, size_t* bytes) {
    if (!bytes) return fail(AGN_EINVAL, "bytes is NULL");
    std::vector<int64_t> pre;
    std::vector<size_t> mag;
    LagLayout L;
    int rc = lag_layout(n_curves, n, n_lags, lags, n_thr, units, &pre, &mag, &L);
    if (rc) return rc;
    *bytes = L.total;
    return AGN_OK;
}

extern "C" int agn_lag_stats_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const int64_t* offset,
                                   const double* x, int32_t n_lags, const int64_t* lags, int32_t units,
                                   double* sf2_out, double* rep_out, int32_t n_thr, const double* dm_ref,
                                   double lam_cut, uint64_t* exceed_out, uint64_t* pairs_out, void* ws,
                                   size_t ws_bytes, void* stream) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    if (n_curves < 0 || n_lags < 0 || n_thr < 0) return fail(AGN_EINVAL, "negative count");
    if (n_curves == 0 || n_lags == 0) return AGN_OK;
    if (!n || !offset || !x || !lags) return fail(AGN_EINVAL, "NULL argument");
    if (units != AGN_SF_LINEAR && units != AGN_SF_MAGNITUDE) return fail(AGN_EINVAL, "unknown units");
    if (n_thr > 0 && (!dm_ref || !exceed_out)) return fail(AGN_EINVAL, "thresholds need dm_ref and exceed_out");
    if (!std::isfinite(lam_cut)) return fail(AGN_EINVAL, "lam_cut must be finite");
    for (int32_t j = 0; j < n_thr; ++j) {
        if (!(dm_ref[j] >= 0.0) || !std::isfinite(dm_ref[j])) return fail(AGN_EINVAL, "dm_ref[%d] must be >= 0", j);
        if (j > 0 && dm_ref[j] < dm_ref[j - 1]) return fail(AGN_EINVAL, "dm_ref must be ascending");
    }
    for (int32_t c = 0; c < n_curves; ++c)
        if (offset[c] < 0) return fail(AGN_EINVAL, "offset[%d] < 0", c);
    std::vector<int64_t> pre;
    std::vector<size_t> mag;
    LagLayout L;
    int rc = lag_layout(n_curves, n, n_lags, lags, n_thr, units, &pre, &mag, &L);
    if (rc) return rc;
    if (!ws || ws_bytes < L.total)
        return fail(AGN_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    unsigned char* base = (unsigned char*)ws;
    std::vector<unsigned char> hdr(L.part_sum, 0);
    LagCurve* hc = (LagCurve*)(hdr.data() + L.curves);
    for (int32_t c = 0; c < n_curves; ++c) {
        hc[c].x = x + offset[c];
        hc[c].m = units == AGN_SF_MAGNITUDE ? (double*)(base + mag[c]) : nullptr;
        hc[c].n = n[c];
    }
    memcpy(hdr.data() + L.lags, lags, sizeof(int64_t) * (size_t)n_lags);
    memcpy(hdr.data() + L.pre, pre.data(), sizeof(int64_t) * pre.size());
    if ((rc = stage_upload(ctx, ws, hdr.data(), hdr.size(), st))) return rc;
    LagArgs A;
    memset(&A, 0, sizeof(A));
    A.curves = (const LagCurve*)(base + L.curves);
    A.lags = (const int64_t*)(base + L.lags);
    A.pre = (const int64_t*)(base + L.pre);
    A.part_sum = (double*)(base + L.part_sum);
    A.part_cnt = (uint32_t*)(base + L.part_cnt);
    A.sf2 = sf2_out ? sf2_out : (double*)(base + L.sf2);
    A.exceed = n_thr > 0 ? exceed_out : nullptr;
    A.pairs = pairs_out;
    A.items = n_curves * n_lags;
    A.K = n_lags;
    A.J = n_thr;
    A.units = units;
    A.cut = lam_cut;
    for (int32_t j = 0; j < n_thr; ++j) A.fac[j] = std::pow(10.0, dm_ref[j] / 2.5);
    {
        ProfScope ps(ctx, "lag_stats", st);
        if (units == AGN_SF_MAGNITUDE) {
            int64_t nmax = 0;
            for (int32_t c = 0; c < n_curves; ++c) nmax = std::max(nmax, n[c]);
            hipLaunchKernelGGL(k_lag_mag, dim3((unsigned)((nmax + 1023) / 1024), (unsigned)n_curves), dim3(256), 0,
                               st, A.curves);
        }
        hipLaunchKernelGGL(k_lag_partial, dim3((unsigned)L.blocks), dim3(LAG_THREADS), 0, st, A);
        hipLaunchKernelGGL(k_lag_finish, dim3((unsigned)A.items), dim3(LAG_THREADS), 0, st, A);
        if (rep_out)
            hipLaunchKernelGGL(k_lag_rep, dim3((unsigned)((n_lags + 255) / 256)), dim3(256), 0, st,
                               (const double*)A.sf2, n_curves, n_lags, rep_out);
    }
    HIPCHK(hipGetLastError());
    return AGN_OK;
}

static int launch_pdf_closed(agn_ctx* ctx, PdfClosed& P, void* stream) {
    HIPCHK(hipSetDevice(ctx->device));
    {
        ProfScope ps(ctx, "erdf_draw", (hipStream_t)stream);
        hipLaunchKernelGGL(k_pdf_closed, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, P);
    }
    HIPCHK(hipGetLastError());
    return AGN_OK;
}

static void sharp_bpl_masses(PdfClosed& P, double u_min, double u_max, double u_star, double e1, double e2) {
    const double ln10 = std::log(10.0);
    P.kind = 0; P.u_min = u_min; P.u_max = u_max; P.u_star = u_star; P.e1 = e1; P.e2 = e2;
    P.a1 = std::pow(10.0, e1 * (u_star - u_min));
    P.m1 = (e1 == 0.0) ? u_star - u_min : (P.a1 - 1.0) / (e1 * ln10);
    P.m2 = (e2 == 0.0) ? u_max - u_star : (1.0 - std::pow(10.0, -e2 * (u_max - u_star))) / (e2 * ln10);
}

extern "C" int agn_erdf_draw(agn_ctx* ctx, const agn_erdf_params* p, int64_t n, uint64_t seed,
                             uint32_t curve_id, double* out, void* stream) {
    if (!ctx || !p || (n > 0 && !out)) return fail(AGN_EINVAL, "NULL argument");
    if (n < 0) return fail(AGN_EINVAL, "n < 0");
    if (!(p->u_min < p->u_br && p->u_br < p->u_max) || p->d1 == 0.0 || p->d2 == 0.0 ||
        !std::isfinite(p->u_min) || !std::isfinite(p->u_max) || !std::isfinite(p->d1) || !std::isfinite(p->d2))
        return fail(AGN_EINVAL, "invalid PDF parameters");
    if (n == 0) return AGN_OK;
    PdfClosed P{};
    sharp_bpl_masses(P, p->u_min, p->u_max, p->u_br, p->d1, p->d2);
    P.n = n; P.seed = seed; P.curve_id = curve_id; P.out = out;
    return launch_pdf_closed(ctx, P, stream);
}

extern "C" int agn_pdf_draw(agn_ctx* ctx, const agn_pdf_params* p, int64_t n, uint64_t seed, uint32_t curve_id,
                            double* out, void* stream) {
    if (!ctx || !p || (n > 0 && !out)) return fail(AGN_EINVAL, "NULL argument");
    if (n < 0) return fail(AGN_EINVAL, "n < 0");
    if (p->kind < AGN_PDF_SHARP_BPL || p->kind > AGN_PDF_LOGNORMAL) return fail(AGN_EINVAL, "unknown PDF kind");
    if (p->measure != AGN_PDF_PER_LOG && p->measure != AGN_PDF_PER_LINEAR) return fail(AGN_EINVAL, "unknown measure");
    if (!std::isfinite(p->u_min) || !std::isfinite(p->u_max) || !std::isfinite(p->u_star) || !(p->u_min < p->u_max))
        return fail(AGN_EINVAL, "need finite u_min < u_max and u_star");
    const double ln10 = std::log(10.0);
    const double shift = (p->measure == AGN_PDF_PER_LINEAR) ? 1.0 : 0.0;
    if (p->kind == AGN_PDF_SHARP_BPL || p->kind == AGN_PDF_EQ1) {
        if (!std::isfinite(p->d1) || !std::isfinite(p->d2)) return fail(AGN_EINVAL, "non-finite slopes");
        // exp(c x) over the support must stay finite and normal
        const double xm = std::fmax(std::fabs(p->u_min - p->u_star), std::fabs(p->u_max - p->u_star));
        if (std::fmax(std::fabs(p->d1 - shift), std::fabs(p->d2 - shift)) * ln10 * xm > 600.0)
            return fail(AGN_EINVAL, "PDF dynamic range over the support exceeds double precision");
    }
    if (p->kind == AGN_PDF_SHARP_BPL && !(p->u_min < p->u_star && p->u_star < p->u_max))
        return fail(AGN_EINVAL, "sharp broken power law needs u_min < u_star < u_max");
    if (p->kind == AGN_PDF_LOGNORMAL && !(p->sigma > 0.0 && std::isfinite(p->sigma)))
        return fail(AGN_EINVAL, "log-normal needs sigma > 0");
    if (n == 0) return AGN_OK;
    if (p->kind == AGN_PDF_SHARP_BPL) {
        PdfClosed P{};
        sharp_bpl_masses(P, p->u_min, p->u_max, p->u_star, p->d1 - shift, p->d2 - shift);
        P.n = n; P.seed = seed; P.curve_id = curve_id; P.out = out;
        return launch_pdf_closed(ctx, P, stream);
    }
    if (p->kind == AGN_PDF_LOGNORMAL) {
        PdfClosed P{};
        P.kind = 2; P.u_min = p->u_min; P.u_max = p->u_max;
        P.mu = p->u_star + shift * p->sigma * p->sigma * ln10;
        P.s = p->sigma * std::sqrt(2.0);
        const double za = (p->u_min - P.mu) / P.s, zb = (p->u_max - P.mu) / P.s;
        P.c_lo = 0.5 * std::erfc(-za);
        P.c_hi = 0.5 * std::erfc(zb);
        // the mass inside, from the tails that keep the difference exact
        if (za >= 0.0) P.tot = 0.5 * (std::erfc(za) - std::erfc(zb));
        else if (zb <= 0.0) P.tot = 0.5 * (std::erfc(-zb) - std::erfc(-za));
        else P.tot = 1.0 - P.c_lo - P.c_hi;
        if (!(P.tot > 0.0)) return fail(AGN_EINVAL, "log-normal support carries no mass in double precision");
        P.n = n; P.seed = seed; P.curve_id = curve_id; P.out = out;
        return launch_pdf_closed(ctx, P, stream);
    }
    if ((p->u_max - p->u_min) / PDF_CELLS * std::fabs(p->d2 - p->d1) * ln10 > 0.5)
        return fail(AGN_EINVAL, "Eq. 1 break sharper than two table cells: (u_max - u_min) |d2 - d1| ln 10 must "
                                "be <= %g", 0.5 * PDF_CELLS);
    PdfTable T{};
    T.u_min = p->u_min; T.u_max = p->u_max; T.u_star = p->u_star;
    T.c1 = (p->d1 - shift) * ln10; T.c2 = (p->d2 - shift) * ln10;
    T.h = (p->u_max - p->u_min) / PDF_CELLS;
    T.n = n; T.seed = seed; T.curve_id = curve_id; T.out = out;
    const int64_t want = (n + PDF_THREADS * 64 - 1) / (PDF_THREADS * 64);
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, PDF_MAX_BLOCKS));
    HIPCHK(hipSetDevice(ctx->device));
    {
        ProfScope ps(ctx, "erdf_draw", (hipStream_t)stream);
        hipLaunchKernelGGL(k_pdf_eq1, dim3(nb), dim3(PDF_THREADS), 0, (hipStream_t)stream, T);
    }
    HIPCHK(hipGetLastError());
    return AGN_OK;
}

extern "C" int agn_pdf_slice(agn_ctx* ctx, const agn_pdf_params* p, int64_t n, int32_t n_chains, int32_t burn,
                             uint64_t seed, uint32_t curve_id, double* out, void* stream) {
    if (!ctx || !p || (n > 0 && !out)) return fail(AGN_EINVAL, "NULL argument");
    if (n < 0) return fail(AGN_EINVAL, "n < 0");
    if (n_chains < 1) return fail(AGN_EINVAL, "n_chains must be >= 1");
    if (burn < 0 || burn > (1 << 24)) return fail(AGN_EINVAL, "burn must be in [0, 2^24]");
    if (p->kind < AGN_PDF_SHARP_BPL || p->kind > AGN_PDF_LOGNORMAL) return fail(AGN_EINVAL, "unknown PDF kind");
    if (p->measure != AGN_PDF_PER_LOG && p->measure != AGN_PDF_PER_LINEAR) return fail(AGN_EINVAL, "unknown measure");
    if (!std::isfinite(p->u_min) || !std::isfinite(p->u_max) || !std::isfinite(p->u_star) || !(p->u_min < p->u_max))
        return fail(AGN_EINVAL, "need finite u_min < u_max and u_star");
    if (p->kind != AGN_PDF_LOGNORMAL && (!std::isfinite(p->d1) || !std::isfinite(p->d2)))
        return fail(AGN_EINVAL, "non-finite slopes");
    if (p->kind == AGN_PDF_LOGNORMAL && !(p->sigma > 0.0 && std::isfinite(p->sigma)))
        return fail(AGN_EINVAL, "log-normal needs sigma > 0");
    if (n == 0) return AGN_OK;
    PdfSlice S;
    memset(&S, 0, sizeof(S));
    S.kind = p->kind; S.measure = p->measure;
    S.u_star = p->u_star; S.d1 = p->d1; S.d2 = p->d2;
    S.gauss = p->kind == AGN_PDF_LOGNORMAL ? 1.0 / (2.0 * p->sigma * p->sigma * std::log(10.0)) : 0.0;
    S.lo = std::pow(10.0, p->u_min);
    S.hi = std::pow(10.0, p->u_max);
    S.start = std::pow(10.0, p->u_star);
    if (!(S.start > S.lo && S.start < S.hi)) S.start = 0.5 * (S.lo + S.hi);
    if (!(S.lo > 0.0) || !std::isfinite(S.hi)) return fail(AGN_EINVAL, "support outside double range");
    S.n = n; S.n_chains = n_chains; S.burn = burn; S.seed = seed; S.curve_id = curve_id; S.out = out;
    const int64_t chains = std::min<int64_t>(n_chains, n);
    HIPCHK(hipSetDevice(ctx->device));
    {
        ProfScope ps(ctx, "erdf_draw", (hipStream_t)stream);
        hipLaunchKernelGGL(k_pdf_slice, dim3((unsigned)((chains + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           S);
    }
    HIPCHK(hipGetLastError());
    return AGN_OK;
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

// ---------------------------------------------------------------------------
// The iteration's transforms and ranking on their own (test exports)
// ---------------------------------------------------------------------------
static int test_check(int64_t n, agn_precision prec, int32_t path) {
    if (check_prec(prec)) return AGN_EINVAL;
    if (!n_supported(n)) return fail(AGN_EUNSUPPORTED_N, "n=%lld is not 2^a or 3*2^a in [2, 2^27]", (long long)n);
    if (path == AGN_TEST_PATH_LDS) {
        if (!lds_path(n, prec))
            return fail(AGN_EUNSUPPORTED_N, "n=%lld does not run on the LDS-resident path in this precision",
                        (long long)n);
    } else if (path == AGN_TEST_PATH_HBM) {
        if (n % BIG_TILE != 0)
            return fail(AGN_EUNSUPPORTED_N, "the multi-pass kernels need n to be a multiple of %d", BIG_TILE);
    } else {
        return fail(AGN_EINVAL, "path %d is neither AGN_TEST_PATH_LDS nor AGN_TEST_PATH_HBM", path);
    }
    return AGN_OK;
}

static size_t test_ws_bytes(int64_t n, agn_precision prec, int32_t path) {
    if (path == AGN_TEST_PATH_LDS) return align256(sizeof(TestLds));
    return align256(sizeof(BigCurve)) + big_curve_ws(n, prec);
}

extern "C" int agn_test_workspace_size(int64_t n, agn_precision prec, int32_t path, size_t* bytes) {
    if (!bytes) return fail(AGN_EINVAL, "bytes is NULL");
    const int rc = test_check(n, prec, path);
    if (rc) return rc;
    *bytes = test_ws_bytes(n, prec, path);
    return AGN_OK;
}

template <typename T>
static int test_run_lds(agn_ctx* ctx, int mode, int64_t n, agn_precision prec, const double* in, double* out,
                        uint32_t* rank_out, void* ws, hipStream_t st) {
    TestLds d;
    memset(&d, 0, sizeof(d));
    d.n = (int32_t)n;
    d.mode = mode;
    d.in = in;
    d.out = out;
    d.rank_out = rank_out;
    const void* tw = nullptr;
    int rc = get_twiddles(ctx, n, AGN_FP64, &tw);
    if (rc) return rc;
    d.tw = tw;
    d.plan = make_plan(n / 2);
    const int ipt = lds_ipt(n), E = ipt / 2, nt = (int)(n / ipt);
    const size_t lds = lds_iter_bytes(n, prec);
    if (lds > ctx->lds_max)
        return fail(AGN_EUNSUPPORTED_N, "n=%lld needs %zu bytes of LDS; the device allows %zu", (long long)n, lds,
                    ctx->lds_max);
    if (E >= 8 && nt % 32 != 0) return fail(AGN_EINVAL, "internal: %d-thread block for E=%d", nt, E);
    rc = stage_upload(ctx, ws, &d, sizeof(d), st);
    if (rc) return rc;
    const TestLds* dp = (const TestLds*)ws;
    switch (E) {
        case 1: hipLaunchKernelGGL((k_test_lds<T, 1>), dim3(1), dim3(nt), lds, st, dp); break;
        case 2: hipLaunchKernelGGL((k_test_lds<T, 2>), dim3(1), dim3(nt), lds, st, dp); break;
        case 3: hipLaunchKernelGGL((k_test_lds<T, 3>), dim3(1), dim3(nt), lds, st, dp); break;
        case 4: hipLaunchKernelGGL((k_test_lds<T, 4>), dim3(1), dim3(nt), lds, st, dp); break;
        case 6: hipLaunchKernelGGL((k_test_lds<T, 6>), dim3(1), dim3(nt), lds, st, dp); break;
        case 8: hipLaunchKernelGGL((k_test_lds<T, 8>), dim3(1), dim3(nt), lds, st, dp); break;
        default: return fail(AGN_EINVAL, "internal: no kernel for E=%d", E);
    }
    return AGN_OK;
}

template <typename T>
static int test_run_big(agn_ctx* ctx, int mode, int64_t n, agn_precision prec, const double* in, double* out,
                        uint32_t* rank_out, void* ws, hipStream_t st) {
    typedef typename key_of<T>::type K;
    TwTable tb;
    std::vector<int> rad;
    int rc = big_group_setup(ctx, n, prec, &tb, &rad);
    if (rc) return rc;
    const int64_t M = n / 2, ntiles = n / BIG_TILE;
    unsigned char* base = (unsigned char*)ws;
    BigCurve d;
    memset(&d, 0, sizeof(d));
    size_t off = align256(sizeof(BigCurve));
    d.n = n;
    d.iters = 1;
    d.tol = -1.0;
    d.s64 = (double*)(base + off); off += align256((size_t)n * 8);
    d.X0 = (double*)(base + off); off += align256((size_t)n * 8);
    d.X1 = (double*)(base + off); off += align256((size_t)n * 8);
    d.rankA = (uint32_t*)(base + off); off += align256((size_t)n * 4);
    d.rankB = (uint32_t*)(base + off); off += align256((size_t)n * 4);
    d.sortA = base + off; off += align256((size_t)n * 12);
    d.sortB = base + off; off += align256((size_t)n * 12);
    d.look = (uint32_t*)(base + off); off += align256((size_t)ntiles * 256 * 4);
    d.dcount = (uint32_t*)(base + off); off += align256(SORT_MAX_PASSES * 256 * 4);
    d.dstart = (uint32_t*)(base + off); off += align256(SORT_MAX_PASSES * 256 * 4);
    d.tickets = (uint32_t*)(base + off); off += align256(SORT_MAX_PASSES * 4);
    d.dpart = (double*)(base + off); off += align256((size_t)big_npart(n) * 8);
    d.cpart = (uint32_t*)(base + off); off += align256((size_t)big_npart(n) * 4);
    d.state = (int32_t*)(base + off); off += align256(16);
    if (mode == TEST_RFFT) d.X0 = const_cast<double*>(in);  // read as x_i by the first forward pass
    if (mode == TEST_RANK) {
        d.rankB = rank_out;  // the last pass writes rank[sample] = sorted position here
        d.rank_out = rank_out;
    }
    rc = stage_upload(ctx, ws, &d, sizeof(d), st);
    if (rc) return rc;
    const BigCurve* dv = (const BigCurve*)ws;
    hipLaunchKernelGGL(k_big_init, dim3(1), dim3(64), 0, st, dv);
    const int np = (int)rad.size();
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (mode == TEST_RANK) {
        hipLaunchKernelGGL((k_test_big_keys<T>), dim3(nb), dim3(256), 0, st, dv, n, in);
        int seq = 0;
        hipLaunchKernelGGL(k_sort_clear, dim3((unsigned)ntiles), dim3(BIG_THREADS), 0, st, dv);
        run_sort<K>(ctx, dv, 1, n, 0, SORT_MODE_RANK, 1, BIG_TILE, &seq, ctx->look_polls, st);
        return AGN_OK;
    }
    // The iteration's transforms: forward passes 0 .. np-2, then the middle
    // pass, whose fold writes the spectrum (rfft); or the middle pass started
    // from the given half spectrum, then the inverse passes in reverse radix
    // order (irfft).
    int sel = 0;  // region written by the next pass
    int64_t Ns = 1;
    if (mode == TEST_RFFT) {
        for (int p = 0; p < np - 1; ++p) {
            FftPass P;
            memset(&P, 0, sizeof(P));
            P.M = M; P.R = rad[p]; P.cols = fft_cols(M, rad[p], Ns, prec); P.nthreads = rad[p] * P.cols / FFT_E;
            P.Ns = Ns;
            P.in_mode = p == 0 ? 1 : 0; P.out_mode = 0; P.inverse = 0;
            P.x_sel = 0; P.with_delta = 0;
            P.src_sel = 1 - sel; P.dst_sel = sel; P.sub = make_plan(rad[p]);
            launch_fft_pass<T>(ctx, dv, 1, P, tb, st);
            Ns *= rad[p];
            sel = 1 - sel;
        }
        MidPass P = make_mid(M, rad[np - 1], 1 - sel, sel, prec);
        P.X_out = out;
        launch_fft_mid<T, MID_SPECTRUM>(ctx, dv, 1, P, tb, st);
        return AGN_OK;
    }
    MidPass Pm = make_mid(M, rad[np - 1], 1, 0, prec);
    Pm.Y_in = in;
    launch_fft_mid<T, MID_UNFOLD>(ctx, dv, 1, Pm, tb, st);
    sel = 1;
    Ns = rad[np - 1];
    for (int p = np - 2; p >= 0; --p) {
        FftPass P;
        memset(&P, 0, sizeof(P));
        P.M = M; P.R = rad[p]; P.cols = fft_cols(M, rad[p], Ns, prec); P.nthreads = rad[p] * P.cols / FFT_E;
        P.Ns = Ns;
        P.in_mode = 0; P.out_mode = 0; P.inverse = 1;
        P.src_sel = 1 - sel; P.dst_sel = sel; P.sub = make_plan(rad[p]);
        launch_fft_pass<T>(ctx, dv, 1, P, tb, st);
        Ns *= rad[p];
        sel = 1 - sel;
    }
    hipLaunchKernelGGL((k_test_big_real<T>), dim3(nb), dim3(256), 0, st, dv, n, 1 - sel, out);
    return AGN_OK;
}

static int test_dispatch(agn_ctx* ctx, int mode, const double* in, int64_t n, agn_precision prec, int32_t path,
                         double* out, uint32_t* rank_out, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(AGN_EINVAL, "ctx is NULL");
    if (!in || (mode == TEST_RANK ? !rank_out : !out)) return fail(AGN_EINVAL, "NULL input or output");
    int rc = test_check(n, prec, path);
    if (rc) return rc;
    const size_t need = test_ws_bytes(n, prec, path);
    if (!ws || ws_bytes < need)
        return fail(AGN_EINVAL, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    if (path == AGN_TEST_PATH_HBM && mode == TEST_RFFT && ((uintptr_t)in & 15) != 0)
        return fail(AGN_EINVAL, "the multi-pass transform reads x in 16-byte pairs: x must be 16-byte aligned");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (path == AGN_TEST_PATH_LDS)
        rc = prec == AGN_FP32 ? test_run_lds<float>(ctx, mode, n, prec, in, out, rank_out, ws, st)
                              : test_run_lds<double>(ctx, mode, n, prec, in, out, rank_out, ws, st);
    else
        rc = prec == AGN_FP32 ? test_run_big<float>(ctx, mode, n, prec, in, out, rank_out, ws, st)
                              : test_run_big<double>(ctx, mode, n, prec, in, out, rank_out, ws, st);
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    return AGN_OK;
}

extern "C" int agn_test_rfft(agn_ctx* ctx, const double* x, int64_t n, agn_precision prec, int32_t path,
                             double* X_out, void* ws, size_t ws_bytes, void* stream) {
    return test_dispatch(ctx, TEST_RFFT, x, n, prec, path, X_out, nullptr, ws, ws_bytes, stream);
}

extern "C" int agn_test_irfft(agn_ctx* ctx, const double* Y, int64_t n, agn_precision prec, int32_t path,
                              double* y_out, void* ws, size_t ws_bytes, void* stream) {
    return test_dispatch(ctx, TEST_IRFFT, Y, n, prec, path, y_out, nullptr, ws, ws_bytes, stream);
}

extern "C" int agn_test_argsort(agn_ctx* ctx, const double* y, int64_t n, agn_precision prec, int32_t path,
                                uint32_t* rank_out, void* ws, size_t ws_bytes, void* stream) {
    return test_dispatch(ctx, TEST_RANK, y, n, prec, path, nullptr, rank_out, ws, ws_bytes, stream);
}

extern "C" int agn_test_lds_bandwidth(int32_t blocks, int32_t reps, float* out, double* seconds, void* stream) {
    if (!out || !seconds || blocks < 1 || reps < 1) return fail(AGN_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(AGN_EDEVICE, "hipEventCreate failed");
    }
    // one untimed launch, then the timed one
    hipLaunchKernelGGL(k_lds_read_bw, dim3((unsigned)blocks), dim3(1024), 0, st, reps, out);
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_lds_read_bw, dim3((unsigned)blocks), dim3(1024), 0, st, reps, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(AGN_EDEVICE, "LDS bandwidth probe: %s", hipGetErrorString(e));
    *seconds = (double)ms * 1e-3;
    return AGN_OK;
}
