// big_path.hpp -- the light-curve iteration (Sec. 2.1, Sec. 3.2.2) for curves
// longer than one workgroup's LDS (up to 2^27 samples): every step is a
// separate pass over HBM, batched over all curves of one length.
//
// Per iteration i (x_i is kept in time order, FP64, two buffers):
//   FFT passes   the first pass reads x_i and x_{i-1} in time order, adds the
//                Eq. 4 terms log10(x_i / x_{i-1})^2 of the previous iteration to
//                per-block partials, and feeds z[m] = x[2m] + i x[2m+1]
//   middle pass  the forward transform's last pass, the real-spectrum fold
//                with the modulus replacement (pairs k, M-k), and the inverse
//                transform's first pass (k_fft_mid)
//   IFFT passes  the remaining radices in reverse order ... -> y, written as
//                order-preserving integer keys
//   sort passes  LSD radix sort of (key, sample index), 8-bit digits: one
//                histogram of every pass's digits, their starts, then per pass
//                one stable scatter staged through LDS in digit order (global
//                writes are contiguous runs), each tile finding where its runs
//                start by a decoupled look-back over the tiles before it; the
//                last pass writes x_{i+1}[sample] = s[sorted position] into the
//                other series buffer (the sorted values are read contiguously)
//
// FFT pass (self-sorting Stockham step with a large radix R): butterfly j of
// M/R reads z[j + r M/R], r < R, multiplies by W_{Ns R}^{(j mod Ns) r}, takes a
// length-R DFT and writes output q to z[(j - j mod Ns) R + j mod Ns + q Ns].  A
// workgroup takes C consecutive butterflies (C = 16..64 so that the tile of
// R x C values is 64 KB; C-element rows of 128-512 bytes) into LDS and runs the
// C length-R DFTs there as small Stockham passes.
// Inter-pass twiddles W_N^t are generated in double precision from a two-level
// table (W_N^{t_hi B} W_N^{t_lo}, B = 4096), stepped along a thread's column by
// FP64 products, and rounded once to the working precision.
#pragma once
#include "common.hpp"
#include "lds_fft.hpp"

namespace agn {

constexpr int BIG_TILE = 8192;       // sort / delta tile
constexpr int BIG_THREADS = 256;     // block of the streaming kernels (BIG_IPT elements each)
constexpr int BIG_IPT = BIG_TILE / BIG_THREADS;
// Keys per thread of the scatter kernel: 16 for 32-bit keys (512 threads per
// tile), 8 for 64-bit keys (1024 threads: the tile's staging fills most of the
// LDS, so one workgroup per CU; more threads keep more loads in flight).
template <typename K>
struct scat_ipt {
    static constexpr int value = sizeof(K) == 4 ? 16 : 8;
};
// Keys per wave whose digit peer masks are formed together in the scatter's
// ranking (it divides both key counts per thread).
constexpr int RANK_GROUP = 4;
// Larger sort tile for 32-bit keys (curves whose length it divides): digit
// runs twice as long, 146 KB of LDS, one 1024-thread workgroup per CU.  Its
// staging does not fit for 64-bit keys.  Exact either way; the batch-plan
// autotuner chooses.
constexpr int SORT_TILE_BIG = 16384;
constexpr int FFT_COLS_MIN = 16;     // fewest butterflies per FFT workgroup
constexpr int FFT_COLS_MAX = 64;     // most butterflies per FFT workgroup
constexpr int TW_LO_BITS = 12;       // two-level twiddle split

struct BigCurve {
    int64_t n;
    int32_t iters;
    int32_t is_big;        // unused by kernels, kept for alignment
    double tol;
    const void* amp;       // T[M + 1]
    const double* x0;      // [N] draw order
    double* s64;           // [N] sorted draw
    double* X0;            // [N] x_i for even i (time order)
    double* X1;            // [N] x_i for odd i
    uint32_t* rankA;       // [N] ranks of x_i, even i (kept only if rank_out)
    uint32_t* rankB;       // [N] ranks of x_i, odd i
    unsigned char* sortA;  // N * 12 bytes: 64-bit keys then 32-bit values, or 8-byte key/index records
    unsigned char* sortB;
    uint32_t* look;        // ntiles * 256 look-back words of the sort scatter
    uint32_t* dcount;      // [SORT_MAX_PASSES][256] digit totals of one sort (accumulated)
    uint32_t* dstart;      // [SORT_MAX_PASSES][256] digit starts of one sort
    uint32_t* tickets;     // [SORT_MAX_PASSES] tile tickets of the scatter passes
    double* dpart;         // [npart] delta partial sums
    uint32_t* cpart;       // [npart] changed-sample counts
    int32_t* state;        // [0] valid, [1] active, [2] iterations done, [3] a look-back wait gave up
    double* x_out;
    double* delta_out;     // [iters] or null
    int32_t* iters_done;   // or null
    uint32_t* rank_out;    // or null
};

// Two-level FP64 twiddle table for one length N: lo[u] = W_N^u, u < B;
// hi[v] = W_N^{v B}, v < N / B (+1).
struct TwTable {
    const cplx<double>* lo;
    const cplx<double>* hi;
};

// W_N^t (forward sign) in double precision, 0 <= t < N.
AGN_DEV cplx<double> tw64(const TwTable& tb, int64_t t) {
    const cplx<double> a = tb.hi[t >> TW_LO_BITS];
    const cplx<double> b = tb.lo[t & ((1 << TW_LO_BITS) - 1)];
    return cmul(a, b);
}

// ----------------------------------------------------------------------------
// FFT pass over HBM
// ----------------------------------------------------------------------------
struct FftPass {
    int64_t M;           // complex length
    int32_t R;           // radix of this pass (<= 512)
    int32_t nthreads;    // R * cols / E
    int32_t cols;        // butterflies per workgroup (power of two, 16..64)
    int64_t Ns;          // product of the previous radices
    int32_t in_mode;     // 0: complex buffer, 1: series x_i (FP64, time order)
    int32_t out_mode;    // 0: complex buffer, 1: keys of y (real view), 2: none (Eq. 4 partials only)
    int32_t inverse;
    int32_t x_sel;       // in_mode 1: x_i in X0 (0) or X1 (1)
    int32_t with_delta;  // in_mode 1: add Eq. 4 terms of x_i against x_{i-1}
    int32_t src_sel;     // 0: sortA, 1: sortB (complex input)
    int32_t dst_sel;     // 0: sortA, 1: sortB (complex or key output)
    FftPlan sub;         // radices of the in-LDS length-R DFT
};

template <typename T>
AGN_DEV int tpad(int e) { return e + (e >> (sizeof(T) == 4 ? 5 : 4)); }

// In-LDS Stockham pass over C independent columns: element (r, c) at
// tpad(r * C + c).  Sub-twiddles come from the LDS table of R-th roots.
template <typename T, int RR, int BMAX, bool INV, int C>
AGN_DEV void col_pass(cplx<T>* buf, const cplx<T>* wr, int R, int Ns, int tid, int nt) {
    const int nb = (R / RR) * C;  // butterflies
    const int RB = R / RR;
    const bool pow2 = (Ns & (Ns - 1)) == 0;
    cplx<T> v[BMAX][RR];
    cplx<T> w[BMAX][RR];
    tid = opaque(tid);
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int q = tid + b * nt;
        if (q < nb) {
            const int j = q / C, c = q % C;
#pragma unroll
            for (int r = 0; r < RR; ++r) v[b][r] = buf[tpad<T>((j + r * RB) * C + c)];
            if (Ns > 1) {
                const int jm = pow2 ? (j & (Ns - 1)) : (j % Ns);
                const int step = R / (Ns * RR);
                // jm * r * step < Ns * RR * R / (Ns * RR) = R
#pragma unroll
                for (int r = 1; r < RR; ++r) {
                    cplx<T> t = wr[jm * r * step];
                    w[b][r] = INV ? cconj(t) : t;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int q = tid + b * nt;
        if (q < nb) {
            const int j = q / C, c = q % C;
            const int jm = pow2 ? (j & (Ns - 1)) : (j % Ns);
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < RR; ++r) v[b][r] = cmul(v[b][r], w[b][r]);
            }
            dftR<T, RR, INV>(v[b]);
            const int d = (j - jm) * RR + jm;
#pragma unroll
            for (int r = 0; r < RR; ++r) buf[tpad<T>((d + r * Ns) * C + c)] = v[b][r];
        }
    }
    __syncthreads();
}

template <typename T, int E, bool INV, int C>
AGN_DEV void col_fft(cplx<T>* buf, const cplx<T>* wr, int R, const FftPlan& plan, int tid, int nt) {
    int Ns = 1;
    for (int p = 0; p < plan.npass; ++p) {
        const int RR = plan.radix[p];
        if (RR == 8) col_pass<T, 8, (E + 7) / 8, INV, C>(buf, wr, R, Ns, tid, nt);
        else if (RR == 4) col_pass<T, 4, (E + 3) / 4, INV, C>(buf, wr, R, Ns, tid, nt);
        else if (RR == 3) col_pass<T, 3, (E + 2) / 3, INV, C>(buf, wr, R, Ns, tid, nt);
        else col_pass<T, 2, (E + 1) / 2, INV, C>(buf, wr, R, Ns, tid, nt);
        Ns *= RR;
    }
}

// ---- The same in-LDS transform for R = 2^LR known at compile time ----
// Power-of-two radices are the common case; with R, the thread count (R C / 8,
// eight values per thread) and the sub-radices fixed, every butterfly index is
// a shift or a mask and the eight LDS offsets of a butterfly are immediates.
// Each butterfly does the arithmetic of col_pass (same elements, same
// sub-twiddles, same dftR); the two can differ in the last bit only where the
// compiler fuses a different product of a butterfly into a multiply-add.
//
// Padded LDS index of (row, column): tpad(row C + c) = row_off(row) + col_off(c).
// With C a multiple of the padding period (32 FP32 values, 16 FP64) both parts
// are linear; for FP32 and C = 16 a pad word follows every two rows, so
// row_off(row) = 16 row + row / 2, which is additive over a step of k rows
// from an even row, or of an even k from any row.
constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

template <typename T, int C>
struct lds_lay {
    static constexpr int SH = sizeof(T) == 4 ? 5 : 4;
    static constexpr bool WIDE = C >= (1 << SH);
    static_assert(WIDE || 2 * C == (1 << SH), "column count without a linear padded layout");
    AGN_DEV static uint32_t row_off(uint32_t r) { return WIDE ? r * (C + (C >> SH)) : r * C + (r >> 1); }
    AGN_DEV static uint32_t col_off(uint32_t c) { return WIDE ? c + (c >> SH) : c; }
    static constexpr uint32_t step(uint32_t k) { return WIDE ? k * (C + (C >> SH)) : k * C + (k >> 1); }
};

template <typename T, int RR, bool INV, int C, int R, int NS>
AGN_DEV void col_pass_fx(cplx<T>* buf, const cplx<T>* wr, uint32_t tid) {
    typedef lds_lay<T, C> L;
    constexpr int RB = R / RR;         // butterflies per column
    constexpr int NT = R * C / 8;      // threads
    constexpr int BPT = 8 / RR;        // butterflies per thread
    constexpr int LC = ilog2c(C);
    static_assert(RB % 2 == 0 && (NS == 1 || NS % 2 == 0), "row steps must be even");
    cplx<T> v[BPT][RR];
    cplx<T> w[BPT][RR];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const uint32_t q = tid + b * NT;
        const uint32_t j = q >> LC, c = q & (C - 1);
        const uint32_t base = L::row_off(j) + L::col_off(c);
#pragma unroll
        for (int r = 0; r < RR; ++r) v[b][r] = buf[base + L::step(r * RB)];
        if constexpr (NS > 1) {
            constexpr uint32_t STEP = R / (NS * RR);
            const uint32_t t = (j & (NS - 1)) * STEP;
#pragma unroll
            for (int r = 1; r < RR; ++r) {
                const cplx<T> tw = wr[t * r];
                w[b][r] = INV ? cconj(tw) : tw;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const uint32_t q = tid + b * NT;
        const uint32_t j = q >> LC, c = q & (C - 1);
        const uint32_t jm = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < RR; ++r) v[b][r] = cmul(v[b][r], w[b][r]);
        }
        dftR<T, RR, INV>(v[b]);
        // first sub-pass: rows j RR + r from the even row j RR; later: rows d + r NS, NS even
        const uint32_t base = L::row_off((j - jm) * RR + jm) + L::col_off(c);
#pragma unroll
        for (int r = 0; r < RR; ++r) buf[base + L::step(NS == 1 ? r : r * NS)] = v[b][r];
    }
    __syncthreads();
}

// Sub-radices in make_plan's order for a power of two: 8 while 8 divides what
// is left, then 4 or 2.
template <typename T, bool INV, int C, int R, int NS = 1>
AGN_DEV void col_fft_fx(cplx<T>* buf, const cplx<T>* wr, uint32_t tid) {
    if constexpr (NS < R) {
        constexpr int LEFT = R / NS;
        constexpr int RR = LEFT % 8 == 0 ? 8 : (LEFT % 4 == 0 ? 4 : 2);
        col_pass_fx<T, RR, INV, C, R, NS>(buf, wr, tid);
        col_fft_fx<T, INV, C, R, NS * RR>(buf, wr, tid);
    }
}

template <typename T>
AGN_DEV cplx<T> to_T(cplx<double> a) { return cmk((T)a.re, (T)a.im); }

// One term of Eq. 4, log10(a / b), for a sample whose value changed from b to
// a.  FP64: the exact ratio and log10.  FP32 form: the ratio of the values
// rounded to float and the hardware log2 (a few 2^-24 relative in the ratio,
// so about 1e-7 absolute in the term), scaled to log10; the sum over the
// terms stays in FP64.
template <typename T>
AGN_DEV double eq4_term(double a, double b) {
    if constexpr (sizeof(T) == 4) {
        const float r = (float)a / (float)b;
        return (double)__log2f(r) * 0.30102999566398119521;  // log10(2)
    } else {
        return log10(a / b);
    }
}

// grid: (M / R / C, curves), block: P.nthreads (E = R * C / nthreads, nthreads a
// multiple of C and at most 1024, so each thread stays in one column
// c = tid mod C).
template <typename T, int E, bool INV, int C, int LR>
__global__ __launch_bounds__(1024) void k_fft_pass(const BigCurve* __restrict__ cv, FftPass P, TwTable tb) {
    typedef typename key_of<T>::type K;
    typedef lds_lay<T, C> L;
    // LR > 0: R = 2^LR and E = 8 fixed at compile time (col_fft_fx); 0: any R
    constexpr bool FX = LR > 0;
    static_assert(!FX || E == 8, "the compile-time transform takes 8 values per thread");
    extern __shared__ __align__(16) unsigned char smem[];
    const BigCurve& d = cv[blockIdx.y];
    if (d.state[1] == 0) return;
    const int tid = threadIdx.x;
    const int R = FX ? (1 << LR) : P.R;
    const int nt = FX ? (1 << LR) * C / E : (int)blockDim.x;
    const int64_t M = P.M, N = 2 * M, MR = M / R, Ns = P.Ns;
    const int64_t j0 = (int64_t)blockIdx.x * C;
    // Ns is 1 or a multiple of C, so (j0 + c) mod Ns = j0m + c.
    const int64_t j0m = (Ns > 1) ? (j0 % Ns) : 0;
    cplx<T>* buf = (cplx<T>*)smem;
    cplx<T>* wr = (cplx<T>*)(smem + (size_t)tpad<T>(R * C + 1) * sizeof(cplx<T>) + 16);
    double* red = (double*)(wr + R);          // one double per wave (<= 16 waves)
    uint32_t* redc = (uint32_t*)(red + 16);   // one word per wave


    // R-th roots for the in-LDS passes: W_R^u = W_N^{u N / R}.
    for (int u = tid; u < R; u += nt) wr[u] = to_T<T>(tw64(tb, (int64_t)u * (N / R)));

    // Load R rows of C consecutive butterflies; apply inter-pass twiddles.
    // Element e = tid + k nt sits in column c = tid mod C and row
    // r_k = tid / C + k (nt / C); its twiddle W_N^{b r_k}, b = (j0m + c) N / (Ns R),
    // is W_N^{b r_0} (W_N^{b nt / C})^k, formed by FP64 products (at most
    // E - 1 of them, a few ulp of FP64) and rounded once to T.
    const gmem<cplx<T>>* src = as_global((const cplx<T>*)(P.src_sel ? d.sortB : d.sortA));
    const gmem<cplx<double>>* xc = as_global((const cplx<double>*)(P.x_sel ? d.X1 : d.X0));
    const gmem<cplx<double>>* xp = as_global((const cplx<double>*)(P.x_sel ? d.X0 : d.X1));
    double acc = 0.0;
    uint32_t chg = 0;
    const int c_t = tid % C, r_t = tid / C, dr = nt / C;
    // (compile-time form: element e's padded LDS index from the thread's own)
    const uint32_t e_lds = L::row_off((uint32_t)r_t) + L::col_off((uint32_t)c_t);
    const bool twid = Ns > 1;
    cplx<double> wk = cmk(1.0, 0.0), wstep = cmk(1.0, 0.0);
    if (twid) {
        const int64_t b = (j0m + c_t) * (N / (Ns * R));
        wk = tw64(tb, b * r_t);
        wstep = tw64(tb, b * dr);
    }
    // E elements per thread, loaded in two unrolled halves so that the data
    // loads of a half are all in flight together.
    static_assert(E % 2 == 0, "E must be even");
    const int64_t m_t = j0 + c_t + (int64_t)r_t * MR;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cplx<T> v[E / 2];
#pragma unroll
        for (int u = 0; u < E / 2; ++u) {
            const int64_t m = m_t + (int64_t)((h * (E / 2) + u) * dr) * MR;
            if (P.in_mode == 1) {
                const cplx<double> a = gload(xc + m);  // x[2m], x[2m + 1]
                if (P.with_delta) {
                    const cplx<double> b = gload(xp + m);
                    if (a.re != b.re) { const double l = eq4_term<T>(a.re, b.re); acc += l * l; ++chg; }
                    if (a.im != b.im) { const double l = eq4_term<T>(a.im, b.im); acc += l * l; ++chg; }
                }
                v[u] = cmk((T)a.re, (T)a.im);
            } else {
                v[u] = gload(src + m);
            }
        }
#pragma unroll
        for (int u = 0; u < E / 2; ++u) {
            const int k = h * (E / 2) + u;
            cplx<T> x = v[u];
            if (twid) {
                cplx<T> w = to_T<T>(wk);
                if (INV) w = cconj(w);
                x = cmul(x, w);
                wk = cmul(wk, wstep);
            }
            if constexpr (FX) buf[e_lds + L::step(k * ((1 << LR) / 8))] = x;  // row r_t + k R / 8
            else buf[tpad<T>(tid + k * nt)] = x;
        }
    }
    if (P.in_mode == 1 && P.with_delta) {
        // per-block Eq. 4 partials, fixed reduction order (blocks are >= 64 threads)
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int s2 = 32; s2 >= 1; s2 >>= 1) {
            acc += __shfl_xor(acc, s2, 64);
            chg += __shfl_xor(chg, s2, 64);
        }
        if (lane == 0) { red[wave] = acc; redc[wave] = chg; }
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            uint32_t cc = 0;
            for (int w = 0; w < nt / 64; ++w) { t += red[w]; cc += redc[w]; }
            d.dpart[blockIdx.x] = t;
            d.cpart[blockIdx.x] = cc;
        }
    }
    // Eq. 4 of the last iteration of a call: the same loads and partition as
    // the first pass of an iteration, so every delta has one summation order
    if (P.out_mode == 2) return;
    __syncthreads();
    if constexpr (FX) col_fft_fx<T, INV, C, (1 << LR)>(buf, wr, (uint32_t)tid);
    else col_fft<T, E, INV, C>(buf, wr, R, P.sub, tid, nt);

    // Write outputs: butterfly j = j0 + c, output q goes to (j - jm) R + jm + q Ns.
    gmem<typename vec2_of<K>::type>* keys = as_global((typename vec2_of<K>::type*)(P.dst_sel ? d.sortB : d.sortA));
    gmem<cplx<T>>* dst = as_global((cplx<T>*)(P.dst_sel ? d.sortB : d.sortA));
    auto put = [&](int64_t m, const cplx<T>& v) {
        if (P.out_mode == 1) {
            typename vec2_of<K>::type kv;
            kv.x = ord_key(v.re);
            kv.y = ord_key(v.im);
            keys[m] = kv;  // keys 2m, 2m + 1
        } else {
            gstore(dst + m, v);
        }
    };
    if constexpr (FX) {
        constexpr uint32_t RF = 1u << LR;
        if (Ns == 1) {
            // e = tid + k nt: column c = tid / R + k C / 8, row q = tid mod R;
            // column c's outputs are z[(j0 + c) R + q]
            const uint32_t q = (uint32_t)tid & (RF - 1), c1 = (uint32_t)tid >> LR;
            const int64_t mb = (j0 + c1) * (int64_t)RF + q;
            const uint32_t lq = L::row_off(q);
#pragma unroll
            for (int k = 0; k < E; ++k)
                put(mb + (int64_t)k * (C / 8) * RF, buf[lq + L::col_off(c1 + k * (C / 8))]);
        } else {
            // e = tid + k nt: row q = r_t + k R / 8, column c_t
            const int64_t mb = (j0 - j0m) * (int64_t)RF + j0m + c_t + (int64_t)r_t * Ns;
#pragma unroll
            for (int k = 0; k < E; ++k)
                put(mb + (int64_t)k * (RF / 8) * Ns, buf[e_lds + L::step(k * (RF / 8))]);
        }
    } else {
        for (int e = tid; e < R * C; e += nt) {
            int q, c;
            if (Ns == 1) { c = e / R; q = e % R; } else { q = e / C; c = e % C; }
            const int64_t jm = (Ns > 1) ? j0m + c : 0;
            const int64_t m = (j0 + c - jm) * R + jm + (int64_t)q * Ns;
            put(m, buf[tpad<T>(q * C + c)]);
        }
    }
}

// ----------------------------------------------------------------------------
// Middle pass: the forward transform's last radix-R pass, the real-spectrum
// fold with the modulus replacement, and the inverse transform's first
// radix-R pass, in one trip through HBM.
//
// The last forward pass (stride Ns = M/R) maps column j -- the R values
// z[j + r M/R] -- onto itself: output q is Z[j + q M/R].  The Hermitian
// partner of Z[j + q M/R] is Z[(M/R - j) + (R - 1 - q) M/R] for j >= 1, i.e.
// in the mirror column M/R - j; columns 0 and M/R/2 pair with themselves.
// The inverse transform runs its radices in the reverse order, so its first
// pass (radix R, stride 1) again reads whole columns and writes column j's
// outputs to z[j R .. j R + R).  A workgroup therefore takes C columns
// j0 .. j0+C-1 and their C mirrors (slot C + m holds column M/R - j0 - m;
// in block 0, slot C holds the self-paired column M/R/2, as column M/R does
// not exist), and needs no data from any other workgroup.
// Modes (compile time): MID_REPLACE is the iteration; MID_SPECTRUM writes the
// real-input spectrum X (double) instead of continuing; MID_UNFOLD starts from
// a given half spectrum Y (double) instead of the forward pass.  The last two
// serve the test exports.
// ----------------------------------------------------------------------------
enum { MID_REPLACE = 0, MID_SPECTRUM = 1, MID_UNFOLD = 2 };

struct MidPass {
    int64_t M;           // complex length
    int32_t R;           // radix of the last forward / first inverse pass (<= 512)
    int32_t nthreads;    // R * 2 * cols / E
    int32_t cols;        // column pairs per workgroup (C)
    int32_t src_sel;     // complex input region (sortA 0 / sortB 1)
    int32_t dst_sel;     // complex output region
    FftPlan sub;         // radices of the in-LDS length-R DFT
    double* X_out;       // MID_SPECTRUM: n/2 + 1 complex doubles
    const double* Y_in;  // MID_UNFOLD: n/2 + 1 complex doubles
};

// Workgroups are dealt to the 8 XCDs in turn (workgroup x of a launch whose
// row count is a multiple of 8 runs on XCD x mod 8).  xcd_order numbers the
// rows so that consecutive numbers run on one XCD, one after another.
AGN_DEV int64_t xcd_order(int64_t x, int64_t rows) {
    return (rows & 7) ? x : (x & 7) * (rows >> 3) + (x >> 3);
}

// grid: (M / R / (2 C), curves), block P.nthreads (E = 2 R C / nthreads).
// Column block b = xcd_order(x): a row of 8 columns is 64 bytes (FP32) and
// its 8 target moduli 32 bytes, so two and four neighbouring blocks share
// each cache line; numbered this way, they run on one XCD at about the same
// time and find the line in its L2 instead of each fetching it.
template <typename T, int E, int C, int MODE, int LR>
__global__ __launch_bounds__(1024) void k_fft_mid(const BigCurve* __restrict__ cv, MidPass P, TwTable tb) {
    constexpr int C2 = 2 * C;
    typedef lds_lay<T, C2> L;
    // LR > 0: R = 2^LR and E = 8 fixed at compile time (col_fft_fx); 0: any R
    constexpr bool FX = LR > 0;
    static_assert(!FX || E == 8, "the compile-time transform takes 8 values per thread");
    extern __shared__ __align__(16) unsigned char smem[];
    const BigCurve& d = cv[blockIdx.y];
    if (d.state[1] == 0) return;
    const int tid = threadIdx.x;
    const int R = FX ? (1 << LR) : P.R;
    const int nt = FX ? (1 << LR) * C2 / E : (int)blockDim.x;
    const int64_t M = P.M, N = 2 * M, MR = M / R;
    const int64_t j0 = xcd_order(blockIdx.x, gridDim.x) * C;
    cplx<T>* buf = (cplx<T>*)smem;
    cplx<T>* wr = (cplx<T>*)(smem + (size_t)tpad<T>(R * C2 + 1) * sizeof(cplx<T>) + 16);
    for (int u = tid; u < R; u += nt) wr[u] = to_T<T>(tw64(tb, (int64_t)u * (N / R)));
    // column of slot sl
    auto col_of = [&](int sl) -> int64_t {
        if (sl < C) return j0 + sl;
        const int m = sl - C;
        return (j0 == 0 && m == 0) ? MR / 2 : MR - j0 - m;
    };

    if constexpr (MODE != MID_UNFOLD) {
        // Load the columns; element (r, slot) takes the last forward pass's
        // twiddle W_M^{j r} = W_N^{2 j r}, formed in FP64 as in k_fft_pass.
        const gmem<cplx<T>>* src = as_global((const cplx<T>*)(P.src_sel ? d.sortB : d.sortA));
        const int c_t = tid % C2, r_t = tid / C2, dr = nt / C2;
        const uint32_t e_lds = L::row_off((uint32_t)r_t) + L::col_off((uint32_t)c_t);
        const int64_t jc = col_of(c_t);
        cplx<double> wk = tw64(tb, 2 * jc * r_t);
        const cplx<double> wstep = tw64(tb, 2 * jc * dr);
        static_assert(E % 2 == 0, "E must be even");
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            cplx<T> v[E / 2];
#pragma unroll
            for (int u = 0; u < E / 2; ++u) {
                const int r = r_t + (h * (E / 2) + u) * dr;
                v[u] = gload(src + jc + (int64_t)r * MR);
            }
#pragma unroll
            for (int u = 0; u < E / 2; ++u) {
                const int k = h * (E / 2) + u;
                const cplx<T> x = cmul(v[u], to_T<T>(wk));
                if constexpr (FX) buf[e_lds + L::step(k * ((1 << LR) / 8))] = x;  // row r_t + k R / 8
                else buf[tpad<T>(tid + k * nt)] = x;
                wk = cmul(wk, wstep);
            }
        }
        __syncthreads();
        if constexpr (FX) col_fft_fx<T, false, C2, (1 << LR)>(buf, wr, (uint32_t)tid);
        else col_fft<T, E, false, C2>(buf, wr, R, P.sub, tid, nt);
    }

    // Hermitian pairs.  Item e < R C: primary element (q, s); block 0 adds
    // R/2 items for the self-paired column M/R/2 in slot C.  Each pair is
    // taken once, with ka = its index <= M/2 (the fold's convention).
    const gmem<T>* amp = as_global((const T*)d.amp);
    const int items = R * C + (j0 == 0 ? R / 2 : 0);
    for (int e = tid; e < items; e += nt) {
        int qa, sa, qb, sb;
        int64_t ka;
        bool dc = false, self = false;
        if (e < R * C) {
            const int sl = (int)((uint32_t)e % C), q = (int)((uint32_t)e / C);
            const int64_t j = j0 + sl, k = j + (int64_t)q * MR;
            if (j == 0) {
                if (2 * q > R) continue;  // taken as the partner of row R - q
                dc = q == 0;
                self = 2 * q == R;
                ka = k; qa = q; sa = 0; qb = (R - q) % R; sb = 0;
            } else if (2 * k <= M) {
                ka = k; qa = q; sa = sl; qb = R - 1 - q; sb = C + sl;
            } else {
                ka = M - k; qa = R - 1 - q; sa = C + sl; qb = q; sb = sl;
            }
        } else {
            const int q = e - R * C;
            ka = MR / 2 + (int64_t)q * MR; qa = q; sa = C; qb = R - 1 - q; sb = C;
        }
        const cplx<T> w = to_T<T>(tw64(tb, ka));
        cplx<T>& za = buf[tpad<T>(qa * C2 + sa)];
        cplx<T>& zb = buf[tpad<T>(qb * C2 + sb)];
        if constexpr (MODE == MID_REPLACE) {
            if (dc) {
                za = fold_dc(za, w, amp[M]);
            } else if (self) {
                cplx<T> ya, unused;
                fold_pair(za, za, w, amp[ka], amp[ka], &ya, &unused);
                za = ya;
            } else {
                cplx<T> ya, yb;
                fold_pair(za, zb, w, amp[ka], amp[M - ka], &ya, &yb);
                za = ya;
                zb = yb;
            }
        } else if constexpr (MODE == MID_SPECTRUM) {
            cplx<T> Xa, Xb;
            fold_spectrum(za, (dc || self) ? za : zb, w, &Xa, &Xb);
            P.X_out[2 * ka] = (double)Xa.re;
            P.X_out[2 * ka + 1] = (double)Xa.im;
            if (!self) {
                P.X_out[2 * (M - ka)] = (double)Xb.re;
                P.X_out[2 * (M - ka) + 1] = (double)Xb.im;
            }
        } else {
            const double* Y = P.Y_in;
            if (dc) {
                const T y0 = (T)Y[0], yM = (T)Y[2 * M];
                za = cmk(y0 + yM, y0 - yM);
            } else {
                const cplx<T> Ya = cmk((T)Y[2 * ka], (T)Y[2 * ka + 1]);
                const cplx<T> Yb = cmk((T)Y[2 * (M - ka)], (T)Y[2 * (M - ka) + 1]);
                cplx<T> ya, yb;
                unfold_pair(Ya, Yb, w, &ya, &yb);
                za = ya;
                if (!self) zb = yb;
            }
        }
    }
    if constexpr (MODE == MID_SPECTRUM) return;
    __syncthreads();
    // The inverse transform's first pass: length-R DFTs of the columns (no
    // twiddles), column j's outputs to z[j R + q].
    gmem<cplx<T>>* dst = as_global((cplx<T>*)(P.dst_sel ? d.sortB : d.sortA));
    if constexpr (FX) {
        col_fft_fx<T, true, C2, (1 << LR)>(buf, wr, (uint32_t)tid);
        // e = tid + k nt: slot tid / R + 2 k (nt = 2 R), row q = tid mod R
        constexpr uint32_t RF = 1u << LR;
        const uint32_t q = (uint32_t)tid & (RF - 1), s1 = (uint32_t)tid >> LR;
        const uint32_t lq = L::row_off(q);
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int sl = (int)(s1 + k * (C2 / E));
            gstore(dst + col_of(sl) * (int64_t)RF + q, buf[lq + L::col_off((uint32_t)sl)]);
        }
    } else {
        col_fft<T, E, true, C2>(buf, wr, R, P.sub, tid, nt);
        for (int e = tid; e < R * C2; e += nt) {
            const int sl = e / R, q = e % R;
            gstore(dst + col_of(sl) * R + q, buf[tpad<T>(q * C2 + sl)]);
        }
    }
}

// ----------------------------------------------------------------------------
// LSD radix sort, 8-bit digits, tiles of BIG_TILE elements
// ----------------------------------------------------------------------------
// Element position p of a tile is held by wave p / (64 IPT), item (p mod 64 IPT)
// / 64, lane p mod 64 (striped inside a wave, so loads are coalesced and the
// wave ranks its items in position order).
enum { SORT_MODE_MOVE = 0, SORT_MODE_RANK = 1, SORT_MODE_PREP = 2 };
constexpr int SORT_MAX_PASSES = 8;
// Between passes, keys travel with their sample index as one record: 8 bytes
// (key << 32 | index) for 32-bit keys, 12 bytes (key low word, key high word,
// index; 4-byte aligned) for 64-bit keys, so that a digit run is one
// contiguous run of records rather than one run in each of two arrays.  The
// first pass reads bare keys (index implicit).
template <typename K> constexpr bool SORT_AOS = sizeof(K) == 4;

struct SortPass {
    int32_t shift;     // digit = (key >> shift) & 255
    int32_t first;     // 1: values are implicit (sample index)
    int32_t src_sel;   // 0: sortA, 1: sortB
    int32_t mode;      // SORT_MODE_*
    int32_t rank_sel;  // MODE_RANK: x_{i+1} and its ranks go to X1/rankB (1) or X0/rankA (0)
    int32_t pass;      // index of the pass within its sort (digit starts, tickets)
    int32_t epoch;     // 1..3, different for consecutive passes (look-back words)
    int32_t spin_max;  // polls before a look-back wait gives up; < 0: give up at once (tests)
};

// Look-back word of (tile, digit): bits 31-30 the pass's epoch, bits 29-28
// the state (AGG: the tile's own count; PREFIX: the count of the digit in all
// tiles up to and including this one), bits 27-0 the count (n <= 2^27).  A
// word of another epoch (the previous pass, or zero from k_sort_clear) is not
// ready.
constexpr uint32_t LOOK_AGG = 1u << 28;
constexpr uint32_t LOOK_PREFIX = 2u << 28;
constexpr uint32_t LOOK_COUNT = (1u << 28) - 1;
// A look-back wait that exceeds this many polls gives up (state[3] = 1) rather
// than spin on; the waited-for tile has a ticket, so it is running and
// publishes within microseconds.  (The context can lower the limit, or make
// every wait give up at once, to exercise that path.)
constexpr int LOOK_SPIN_MAX = 1 << 18;

AGN_DEV uint32_t look_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
AGN_DEV void look_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Zero the look-back words, digit totals and tickets of every curve (once
// per call, before its first sort).  grid: (ntiles, curves), block 256.
__global__ __launch_bounds__(BIG_THREADS) void k_sort_clear(const BigCurve* __restrict__ cv) {
    const BigCurve& d = cv[blockIdx.y];
    const int tid = threadIdx.x;
    d.look[(int64_t)blockIdx.x * 256 + tid] = 0u;
    if (blockIdx.x == 0) {
        for (int i = tid; i < SORT_MAX_PASSES * 256; i += BIG_THREADS) d.dcount[i] = 0u;
        if (tid < SORT_MAX_PASSES) d.tickets[tid] = 0u;
    }
}

// Digit totals of every pass of one sort, from its input keys (a pass only
// permutes the keys, so each pass's digit counts are those of the input).
// grid: (workgroups per curve, curves), block 256; workgroup x takes tiles
// x, x + gridDim.x, ...  Each wave counts into its own LDS histogram per
// pass; for the exponent bytes (the top byte of 32-bit keys, the top two of
// 64-bit keys), where a few digits dominate, into CT copies, lane l into copy
// l mod CT, rows padded to 257 words, so that fewer lanes of one atomic hit
// the same counter.  Totals go to dcount by one global atomic add per
// (pass, digit) and workgroup.
template <typename K>
struct count_layout {
    static constexpr int NP = (int)sizeof(K);
    static constexpr int NTOP = NP == 4 ? 1 : 2;  // exponent bytes
    static constexpr int CT = NP == 4 ? 16 : 8;   // their copies per wave
    static constexpr int WAVES = BIG_THREADS / 64;
    static constexpr int NLO = NP - NTOP;
    static constexpr int WORDS = (NLO * WAVES + NTOP * WAVES * CT) * 257;
    static constexpr int off(int p) {
        return p < NLO ? p * WAVES * 257 : (NLO * WAVES + (p - NLO) * WAVES * CT) * 257;
    }
};

template <typename K, int TILE>
__global__ __launch_bounds__(BIG_THREADS) void k_sort_count(const BigCurve* __restrict__ cv, int src_sel,
                                                            int64_t ntiles) {
    typedef count_layout<K> CL;
    constexpr int IPT = TILE / BIG_THREADS;
    __shared__ uint32_t h[CL::WORDS];
    const BigCurve& d = cv[blockIdx.y];
    if (d.state[1] == 0) return;
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < CL::WORDS; i += BIG_THREADS) h[i] = 0u;
    __syncthreads();
    const gmem<K>* keys = as_global((const K*)(src_sel ? d.sortB : d.sortA));
    const int row_lo = wave * 257, row_hi = (wave * CL::CT + (tid % CL::CT)) * 257;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t base = t * TILE + tid;
        K k[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i) k[i] = keys[base + i * BIG_THREADS];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
#pragma unroll
            for (int p = 0; p < CL::NP; ++p) {
                const int row = p < CL::NLO ? row_lo : row_hi;
                atomicAdd(&h[CL::off(p) + row + ((uint32_t)(k[i] >> (8 * p)) & 255u)], 1u);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < CL::NP; ++p) {
        const int rows = p < CL::NLO ? CL::WAVES : CL::WAVES * CL::CT;
        uint32_t c = 0;
        for (int r = 0; r < rows; ++r) c += h[CL::off(p) + r * 257 + tid];
        if (c) atomicAdd(&d.dcount[p * 256 + tid], c);
    }
}

// Digit starts of every pass (exclusive scans of the totals); clears the
// totals and the tickets for the next sort.  grid: (curves), block 256.
__global__ __launch_bounds__(BIG_THREADS) void k_sort_starts(const BigCurve* __restrict__ cv, int npass) {
    __shared__ uint32_t sh[4];
    const BigCurve& d = cv[blockIdx.x];
    if (d.state[1] == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int p = 0; p < npass; ++p) {
        const uint32_t v = d.dcount[p * 256 + tid];
        uint32_t inc = v;
#pragma unroll
        for (int s2 = 1; s2 < 64; s2 <<= 1) {
            const uint32_t o = __shfl_up(inc, s2, 64);
            if (lane >= s2) inc += o;
        }
        if (lane == 63) sh[wave] = inc;
        __syncthreads();
        uint32_t wpre = 0;
        for (int w = 0; w < wave; ++w) wpre += sh[w];
        d.dstart[p * 256 + tid] = wpre + inc - v;
        d.dcount[p * 256 + tid] = 0u;
        __syncthreads();
    }
    if (tid < SORT_MAX_PASSES) d.tickets[tid] = 0u;
}

// grid: (ntiles, curves), block TILE / scat_ipt<K>.  Stable scatter of one
// 8-bit digit.  A workgroup takes the next tile of its curve in ticket order
// (so every tile it may wait for is already running).  Each wave ranks its
// 64 x SCAT_IPT keys with ballots and per-wave running digit counters; the
// tile publishes its digit counts (AGG), then thread d walks back over the
// look-back words of digit d of the tiles before it, adding AGG counts until
// it meets a PREFIX, and publishes its own PREFIX.  The tile is then
// rearranged in LDS into digit order, and thread q takes tile positions q,
// q + SCAT_THREADS, ... so that consecutive threads write consecutive global
// positions inside each digit's run (runs of TILE / 256 keys on average).
template <typename K, int TILE>
__global__ __launch_bounds__(TILE / scat_ipt<K>::value) void k_sort_scatter(const BigCurve* __restrict__ cv,
                                                                            SortPass P, int64_t ntiles) {
    constexpr int SCAT_IPT = scat_ipt<K>::value;
    constexpr int SCAT_THREADS = TILE / SCAT_IPT;
    static_assert(SCAT_THREADS <= 1024, "tile too large for one workgroup");
    constexpr int SCAT_WAVES = SCAT_THREADS / 64;
    __shared__ uint16_t wcnt[SCAT_WAVES][256];  // per-wave running digit counters (<= 64 * SCAT_IPT),
                                                // then their exclusive prefix over waves
    __shared__ uint32_t tstart[256];            // digit start inside the tile
    __shared__ uint32_t gbase[256];             // global start of the tile's digit run
    __shared__ uint32_t wtot[4];                // digit-scan totals of the first four waves
    __shared__ uint32_t s_tile;                 // ticket
    __shared__ K skey[TILE];
    __shared__ uint32_t sval[TILE];
    static_assert(64 * SCAT_IPT * (SCAT_WAVES - 1) < 65536, "wave prefix must fit 16 bits");
    static_assert(SCAT_THREADS >= 256 && SCAT_WAVES >= 4, "the digit phase takes the first 256 threads");
    const BigCurve& d = cv[blockIdx.y];
    if (d.state[1] == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = d.n;
    if (tid == 0) s_tile = atomicAdd(&d.tickets[P.pass], 1u);
    for (int q = lane; q < 256; q += 64) wcnt[wave][q] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile >= ntiles) return;  // (never: one ticket per workgroup)
    const int64_t base = tile * TILE + (int64_t)wave * 64 * SCAT_IPT;
    const unsigned char* srcb = P.src_sel ? d.sortB : d.sortA;
    const gmem<K>* skeys = as_global((const K*)srcb);

    K key[SCAT_IPT];
    uint32_t val[SCAT_IPT];
    uint32_t loc[SCAT_IPT];
    if (P.first) {
#pragma unroll
        for (int i = 0; i < SCAT_IPT; ++i) {
            const int64_t p = base + i * 64 + lane;
            key[i] = skeys[p];
            val[i] = (uint32_t)p;
        }
    } else if constexpr (SORT_AOS<K>) {
        const gmem<uint64_t>* srec = as_global((const uint64_t*)srcb);
#pragma unroll
        for (int i = 0; i < SCAT_IPT; ++i) {
            const uint64_t r = srec[base + i * 64 + lane];
            key[i] = (K)(r >> 32);
            val[i] = (uint32_t)r;
        }
    } else {
        // 12-byte records: key low word, key high word, index
        const gmem<uint32_t>* sw = as_global((const uint32_t*)srcb);
#pragma unroll
        for (int i = 0; i < SCAT_IPT; ++i) {
            const int64_t p = 3 * (base + i * 64 + lane);
            key[i] = ((uint64_t)sw[p + 1] << 32) | sw[p];
            val[i] = sw[p + 2];
        }
    }
    // LDS-typed, so that the counter traffic compiles to ds_ instructions
    // (a volatile generic pointer becomes coherent flat loads and stores)
    volatile __attribute__((address_space(3))) uint16_t* vc =
        (volatile __attribute__((address_space(3))) uint16_t*)wcnt[wave];
    // Keys are ranked RANK_GROUP at a time: their peer masks first (independent
    // chains the compiler can interleave), then the counter updates in key order.
#pragma unroll
    for (int i0 = 0; i0 < SCAT_IPT; i0 += RANK_GROUP) {
        uint32_t plo[RANK_GROUP], phi[RANK_GROUP];
#pragma unroll
        for (int g = 0; g < RANK_GROUP; ++g) {
            const uint32_t dg = (uint32_t)(key[i0 + g] >> P.shift) & 255u;
            // lanes whose digit differs from this lane's in some bit b: the
            // ballot of bit b, XOR this lane's bit b spread over a word, ORed
            // over the bits; peers = the lanes that differ in none
            uint32_t dlo = 0u, dhi = 0u;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                // (opaque: the ballot then tests m itself instead of re-deriving the bit)
                const uint32_t m = (uint32_t)opaque(__builtin_amdgcn_sbfe((int)dg, (unsigned)b, 1u));  // 0 or ~0
                const uint64_t bal = __ballot(m != 0u);
                // d | (bal ^ m) in one three-input bitwise operation (truth table
                // indexed by d * 4 + bal * 2 + m)
                dlo = __builtin_amdgcn_bitop3_b32(dlo, (uint32_t)bal, m, 0xF6);
                dhi = __builtin_amdgcn_bitop3_b32(dhi, (uint32_t)(bal >> 32), m, 0xF6);
            }
            plo[g] = ~dlo;
            phi[g] = ~dhi;
        }
#pragma unroll
        for (int g = 0; g < RANK_GROUP; ++g) {
            const uint32_t dg = (uint32_t)(key[i0 + g] >> P.shift) & 255u;
            // peers in lower lanes
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi[g], __builtin_amdgcn_mbcnt_lo(plo[g], 0u));
            const uint32_t cur = vc[dg];
            __builtin_amdgcn_wave_barrier();
            if (below == 0) vc[dg] = (uint16_t)(cur + (uint32_t)__popc(plo[g]) + (uint32_t)__popc(phi[g]));
            __builtin_amdgcn_wave_barrier();
            loc[i0 + g] = cur + below;
        }
    }
    __syncthreads();
    // per digit (threads 0..255): prefix over waves, tile total, scan over digits
    uint32_t tot = 0, inc = 0;
    if (tid < 256) {
        const int q = tid;
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < SCAT_WAVES; ++w) {
            const uint32_t c = wcnt[w][q];
            wcnt[w][q] = (uint16_t)run;
            run += c;
        }
        tot = run;
        // publish this tile's count of digit q (tile 0: its prefix)
        look_store(&d.look[tile * 256 + q], ((uint32_t)P.epoch << 30) | (tile == 0 ? LOOK_PREFIX : LOOK_AGG) | tot);
        inc = tot;
#pragma unroll
        for (int s2 = 1; s2 < 64; s2 <<= 1) {
            const uint32_t o = __shfl_up(inc, s2, 64);
            if (lane >= s2) inc += o;
        }
        if (lane == 63) wtot[wave] = inc;
    }
    __syncthreads();
    if (tid < 256) {
        const int q = tid;
        uint32_t pre = 0;
        for (int w = 0; w < wave; ++w) pre += wtot[w];
        tstart[q] = pre + inc - tot;
        // decoupled look-back: count of digit q in the tiles before this one
        const uint32_t ep = (uint32_t)P.epoch << 30;
        uint32_t excl = 0;
        if (tile > 0 && P.spin_max < 0) {
            d.state[3] = 1;  // forced give-up (failure-handling tests): excl stays 0
            look_store(&d.look[tile * 256 + q], ep | LOOK_PREFIX | tot);
        } else if (tile > 0) {
            int64_t j = tile - 1;
            int polls = 0;
            while (j >= 0) {
                const uint32_t w = look_load(&d.look[j * 256 + q]);
                if ((w & 0xC0000000u) == ep && (w & (LOOK_AGG | LOOK_PREFIX))) {
                    excl += w & LOOK_COUNT;
                    if (w & LOOK_PREFIX) break;
                    --j;
                } else if (++polls > P.spin_max) {
                    d.state[3] = 1;
                    break;
                } else {
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            look_store(&d.look[tile * 256 + q], ep | LOOK_PREFIX | (excl + tot));
        }
        gbase[q] = d.dstart[P.pass * 256 + q] + excl;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SCAT_IPT; ++i) {
        const uint32_t dg = (uint32_t)(key[i] >> P.shift) & 255u;
        const uint32_t pl = tstart[dg] + wcnt[wave][dg] + loc[i];
        skey[pl] = key[i];
        sval[pl] = val[i];
    }
    __syncthreads();
    unsigned char* dstb = P.src_sel ? d.sortA : d.sortB;
    gmem<uint64_t>* drec = as_global((uint64_t*)dstb);
    gmem<uint32_t>* dw = as_global((uint32_t*)dstb);
    gmem<uint32_t>* rnk = as_global(P.rank_sel ? d.rankB : d.rankA);
    gmem<double>* xn = as_global(P.rank_sel ? d.X1 : d.X0);
    gmem<double>* s64 = as_global(d.s64);
    const gmem<double>* x0 = as_global(d.x0);
#pragma unroll 4
    for (int q = tid; q < TILE; q += SCAT_THREADS) {
        const K k = skey[q];
        const uint32_t v = sval[q];
        const uint32_t dg = (uint32_t)(k >> P.shift) & 255u;
        const uint32_t dest = gbase[dg] + (uint32_t)q - tstart[dg];
        if (dest >= (uint32_t)n) continue;  // (never, unless a look-back wait gave up)
        if (P.mode == SORT_MODE_MOVE) {
            if constexpr (SORT_AOS<K>) {
                drec[dest] = ((uint64_t)k << 32) | v;
            } else {
                dw[3 * (size_t)dest] = (uint32_t)k;
                dw[3 * (size_t)dest + 1] = (uint32_t)((uint64_t)k >> 32);
                dw[3 * (size_t)dest + 2] = v;
            }
        } else if (v < (uint32_t)n) {  // (always, unless a look-back wait gave up in an earlier pass)
            if (P.mode == SORT_MODE_RANK) {
                xn[v] = s64[dest];
                if (d.rank_out) rnk[v] = dest;
            } else {
                s64[dest] = x0[v];
                rnk[v] = dest;
            }
        }
    }
}

// Order-preserving keys of the draw, its validity, and x_0 = draw (prep, once
// per call).  grid: (ntiles, curves), block 256.
__global__ __launch_bounds__(BIG_THREADS) void k_big_prep_keys(const BigCurve* __restrict__ cv) {
    const BigCurve& d = cv[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * BIG_TILE;
    uint64_t* keys = (uint64_t*)d.sortA;
    int bad = 0;
    for (int i = 0; i < BIG_IPT; ++i) {
        const int64_t p = base + i * BIG_THREADS + threadIdx.x;
        const double x = d.x0[p];
        bad |= !(x > 0.0 && x <= 1.7976931348623157e308);
        keys[p] = ord_key(x);
        d.X0[p] = x;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicAnd(&d.state[0], 0);
}

// State init: valid = 1, active = 1, done = 0, no look-back wait given up.  grid: (curves), block 64.
__global__ void k_big_init(const BigCurve* __restrict__ cv) {
    const BigCurve& d = cv[blockIdx.x];
    if (threadIdx.x == 0) {
        d.state[0] = 1;
        d.state[1] = 1;
        d.state[2] = 0;
        d.state[3] = 0;
    }
}

// After prep: deactivate invalid curves and curves with nothing to do.
__global__ void k_big_after_prep(const BigCurve* __restrict__ cv) {
    const BigCurve& d = cv[blockIdx.x];
    if (threadIdx.x == 0) {
        if (d.state[0] == 0 || d.iters <= 0) d.state[1] = 0;
    }
}

// One block per curve: delta of iteration `it` from `npart` partials,
// iteration count, stopping rule.
__global__ __launch_bounds__(BIG_THREADS) void k_big_delta_final(const BigCurve* __restrict__ cv, int it,
                                                                 int64_t npart) {
    __shared__ double shd[4];
    __shared__ uint32_t shc[4];
    const BigCurve& d = cv[blockIdx.x];
    if (d.state[1] == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double acc = 0.0;
    uint32_t chg = 0;
    for (int64_t t = tid; t < npart; t += BIG_THREADS) {
        acc += d.dpart[t];
        chg += d.cpart[t];
    }
#pragma unroll
    for (int s2 = 32; s2 >= 1; s2 >>= 1) {
        acc += __shfl_xor(acc, s2, 64);
        chg += __shfl_xor(chg, s2, 64);
    }
    if (lane == 0) { shd[wave] = acc; shc[wave] = chg; }
    __syncthreads();
    if (tid == 0) {
        const double a = (shd[0] + shd[1]) + (shd[2] + shd[3]);
        const uint32_t c = shc[0] + shc[1] + shc[2] + shc[3];
        const double delta = sqrt(a / (double)d.n);
        if (d.delta_out) d.delta_out[it] = delta;
        d.state[2] = it + 1;
        if (it + 1 >= d.iters || (d.tol >= 0.0 && (c == 0u || (d.tol > 0.0 && delta <= d.tol))))
            d.state[1] = 0;
    }
}

// x_out = x_done, rank_out, iters_done, zero-fill of unused delta entries.
// grid: (ntiles, curves), block 256.
__global__ __launch_bounds__(BIG_THREADS) void k_big_output(const BigCurve* __restrict__ cv) {
    const BigCurve& d = cv[blockIdx.y];
    const int done = d.state[2];
    const double* x = (done & 1) ? d.X1 : d.X0;
    const uint32_t* r = (done & 1) ? d.rankB : d.rankA;
    const int64_t base = (int64_t)blockIdx.x * BIG_TILE;
    for (int i = 0; i < BIG_IPT; ++i) {
        const int64_t p = base + i * BIG_THREADS + threadIdx.x;
        d.x_out[p] = x[p];
        if (d.rank_out) d.rank_out[p] = r[p];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (d.iters_done) *d.iters_done = d.state[3] ? -2 : (d.state[0] ? done : -1);
        if (d.delta_out)
            for (int j = done; j < d.iters; ++j) d.delta_out[j] = 0.0;
    }
}

}  // namespace agn
