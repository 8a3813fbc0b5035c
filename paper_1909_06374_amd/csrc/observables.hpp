// observables.hpp -- what is measured on the generator's output (App. A,
// Sec. 3.2.10, Sec. 4.2): the periodogram of Eq. A2 for a batch of real
// series and its means over logarithmic frequency bins,
// P_j = 2 / N^2 |X_j|^2, X_j = sum_t x[t] exp(-2 pi i j t / N), j = 0..N/2,
// in double precision; and lag statistics (structure function, |dm| counts).
//
// Curves that fit one workgroup's LDS transform there (Stockham passes of the
// half-length complex FFT of z[m] = x[2m] + i x[2m+1], then the real-spectrum
// fold); longer curves use the multi-pass FFT kernels and a fold kernel here.
#pragma once
#include "big_path.hpp"
#include "lds_fft.hpp"

namespace agn {

struct PgDesc {
    int32_t n;
    int32_t pad_;
    const double* x;       // [N]
    double* P;             // [N/2 + 1]
    const void* tw;        // cplx<double>[N/2 + 1], W_N^t
    FftPlan plan;          // radices of the length-N/2 complex FFT
};

// LDS bytes of the periodogram kernel: FFT buffer + two-level twiddle table.
__host__ __device__ inline size_t lds_pg_layout(int N, size_t* tw_off) {
    const size_t fft = (size_t)cpad_size<double>(N / 2) * sizeof(cplx<double>);
    const size_t tw = (fft + 15) & ~(size_t)15;
    if (tw_off) *tw_off = tw;
    return tw + (size_t)tw_lds_entries(N) * sizeof(cplx<double>);
}

// P[k] and P[M - k] from the half-length spectrum Z (k = 0: P[0] and P[M]).
AGN_DEV void fold_power(cplx<double> zk, cplx<double> zm, cplx<double> w, int64_t k, int64_t M, double scale,
                        double* P) {
    const cplx<double> Ev = cmk((zk.re + zm.re) * 0.5, (zk.im - zm.im) * 0.5);
    const cplx<double> Ov = cmk((zk.im + zm.im) * 0.5, (zm.re - zk.re) * 0.5);
    const cplx<double> wO = cmul(w, Ov);
    if (k == 0) {
        const double x0 = Ev.re + wO.re, xn = Ev.re - wO.re;
        P[0] = scale * x0 * x0;
        P[M] = scale * xn * xn;
        return;
    }
    const cplx<double> Xk = cadd(Ev, wO);
    const cplx<double> Xm = csub(Ev, wO);  // conj(X_{M-k}); same modulus
    P[k] = scale * (Xk.re * Xk.re + Xk.im * Xk.im);
    if (M - k != k) P[M - k] = scale * (Xm.re * Xm.re + Xm.im * Xm.im);
}

// One workgroup per curve; block N / IPT threads (E = IPT / 2 values per thread).
template <int E>
__global__ __launch_bounds__(1024) void k_lds_periodogram(const PgDesc* __restrict__ descs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PgDesc& d = descs[blockIdx.x];
    const int N = d.n, M = N / 2;
    const int tid = threadIdx.x, nt = blockDim.x;
    size_t tw_off;
    lds_pg_layout(N, &tw_off);
    cplx<double>* Zc = (cplx<double>*)smem;
    double* Zf = (double*)smem;
    TwLds tw;
    tw.bits = tw_lds_bits(N);
    {
        cplx<double>* lo = (cplx<double>*)(smem + tw_off);
        cplx<double>* hi = lo + (1 << tw.bits);
        const cplx<double>* __restrict__ tg = (const cplx<double>*)d.tw;
        const int nlo = 1 << tw.bits, nhi = (N + nlo - 1) / nlo;
        for (int u = tid; u < nlo + nhi; u += nt) {
            const int t = u < nlo ? u : (u - nlo) * nlo;
            cplx<double> w;
            if (t <= M) {
                w = tg[t];
            } else {
                const cplx<double> v = tg[t - M];
                w = cmk(-v.re, -v.im);
            }
            if (u < nlo) lo[u] = w;
            else hi[u - nlo] = w;
        }
        tw.lo = lo;
        tw.hi = hi;
    }
    for (int p = tid; p < N; p += nt) Zf[rpad<double>(p)] = d.x[p];
    __syncthreads();
    lds_fft<double, E, false>(Zc, M, d.plan, tid, nt, tw);
    const double scale = 2.0 / ((double)N * (double)N);
    for (int k = tid; k <= M / 2; k += nt) {
        const int mk = (k == 0) ? 0 : M - k;
        fold_power(Zc[cpad<double>(k)], Zc[cpad<double>(mk)], twiddle<double, false>(tw, k), k, M, scale, d.P);
    }
}

// Multi-pass curves: fold of the transformed half-length spectrum (in the
// curve's sort region `sel`) into P.  grid: (ceil((M/2 + 1) / 256), curves).
__global__ __launch_bounds__(256) void k_big_fold_power(const BigCurve* __restrict__ cv, int64_t M, int sel,
                                                        TwTable tb, double* const* __restrict__ Pout) {
    const BigCurve& d = cv[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > M / 2) return;
    const cplx<double>* Z = (const cplx<double>*)(sel ? d.sortB : d.sortA);
    const int64_t mk = (k == 0) ? 0 : M - k;
    const double n = 2.0 * (double)M;
    fold_power(Z[k], Z[mk], tw64(tb, k), k, M, 2.0 / (n * n), Pout[blockIdx.y]);
}

// Mean of P over bins [lo, hi) of j.  grid: (bins, curves), block 256; the
// bin table holds, per curve, its P pointer, bin count and (lo, hi) pairs.
struct BinDesc {
    const double* P;
    double* out;
    const int64_t* edges;  // 2 * nbins
    int32_t nbins;
    int32_t pad_;
};

__global__ __launch_bounds__(256) void k_log_bins(const BinDesc* __restrict__ bd) {
    __shared__ double sh[4];
    const BinDesc& b = bd[blockIdx.y];
    const int bin = blockIdx.x;
    if (bin >= b.nbins) return;
    const int64_t lo = b.edges[2 * bin], hi = b.edges[2 * bin + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double acc = 0.0;
    for (int64_t j = lo + tid; j < hi; j += 256) acc += b.P[j];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) acc += __shfl_xor(acc, s, 64);
    if (lane == 0) sh[wave] = acc;
    __syncthreads();
    if (tid == 0) b.out[bin] = ((sh[0] + sh[1]) + (sh[2] + sh[3])) / (double)(hi - lo);
}

// ---------------------------------------------------------------------------
// Lag statistics (Eq. A6; Sec. 3.2.10; Figs. 16-17) of a batch of positive
// series at caller-chosen lags.  Work item = (curve, lag); each item is split
// over up to LAG_MAX_BLOCKS workgroups, each of which strides over chunks of
// LAG_CHUNK pairs, reading x[i] and x[i + k] coalesced.  In magnitudes, a first
// pass writes m = -2.5 log10 x once per sample, so the pair loop takes no
// logarithms.  Every workgroup writes its partial sum (FP64) and counts (u32)
// to the workspace; a second kernel adds them per item in a fixed order, so
// results do not depend on timing.  No atomics.
// ---------------------------------------------------------------------------
constexpr int LAG_THREADS = 256;
constexpr int LAG_IPT = 8;
constexpr int64_t LAG_CHUNK = (int64_t)LAG_THREADS * LAG_IPT;
constexpr int LAG_MAX_BLOCKS = 64;
constexpr int LAG_MAX_THR = 16;

struct LagCurve {
    const double* x;
    double* m;        // -2.5 log10 x (magnitude units), workspace
    int64_t n;
};

// m = -2.5 log10 x for every curve.  grid: (ceil(max n / 1024), curves).
__global__ __launch_bounds__(256) void k_lag_mag(const LagCurve* __restrict__ cv) {
    const LagCurve& c = cv[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < c.n && i < (int64_t)(blockIdx.x + 1) * 1024;
         i += 256)
        c.m[i] = -2.5 * log10(c.x[i]);
}

struct LagArgs {
    const LagCurve* curves;
    const int64_t* lags;     // [K]
    const int64_t* pre;      // [items + 1], first workgroup of each item
    double* part_sum;        // [workgroups]
    uint32_t* part_cnt;      // [workgroups][1 + J]: counted pairs, then one per threshold
    double* sf2;             // [items]
    uint64_t* exceed;        // [items][J] or null
    uint64_t* pairs;         // [items] or null
    int32_t items, K, J, units;
    double cut;              // <= 0: no detection cut
    double fac[LAG_MAX_THR]; // 10^(dm_ref / 2.5), ascending
};

AGN_DEV int lag_item_of(const int64_t* pre, int items, int64_t g) {
    int lo = 0, hi = items;  // pre[lo] <= g < pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(LAG_THREADS) void k_lag_partial(LagArgs A) {
    __shared__ double wsum[LAG_THREADS / 64];
    __shared__ uint32_t wcnt[LAG_THREADS / 64][1 + LAG_MAX_THR];
    const int64_t g = blockIdx.x;
    const int item = lag_item_of(A.pre, A.items, g);
    const int64_t b = g - A.pre[item], nb = A.pre[item + 1] - A.pre[item];
    const int c = item / A.K;
    const int64_t k = A.lags[item - c * A.K];
    const double* __restrict__ x = A.curves[c].x;
    const double* __restrict__ mg = A.curves[c].m;
    const int64_t P = A.curves[c].n - k;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int J = A.J;
    double acc = 0.0;
    uint32_t npairs = 0;
    uint32_t cnt[LAG_MAX_THR];
#pragma unroll
    for (int j = 0; j < LAG_MAX_THR; ++j) cnt[j] = 0;
    for (int64_t q = b; q * LAG_CHUNK < P; q += nb) {
        const int64_t base = q * LAG_CHUNK + tid;
        double va[LAG_IPT], vb[LAG_IPT], d[LAG_IPT];
#pragma unroll
        for (int e = 0; e < LAG_IPT; ++e) {
            const int64_t i = base + (int64_t)e * LAG_THREADS;
            va[e] = i < P ? x[i] : 1.0;
            vb[e] = i < P ? x[i + k] : 1.0;
        }
        if (A.units) {
#pragma unroll
            for (int e = 0; e < LAG_IPT; ++e) {
                const int64_t i = base + (int64_t)e * LAG_THREADS;
                d[e] = i < P ? mg[i + k] - mg[i] : 0.0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < LAG_IPT; ++e) d[e] = vb[e] - va[e];
        }
#pragma unroll
        for (int e = 0; e < LAG_IPT; ++e) {
            if (base + (int64_t)e * LAG_THREADS >= P) break;
            double a = va[e], bb = vb[e];
            acc += d[e] * d[e];
            if (A.cut > 0.0) {
                if (a < A.cut && bb < A.cut) continue;
                a = fmax(a, A.cut);
                bb = fmax(bb, A.cut);
            }
            ++npairs;
            const double hi = fmax(a, bb), lo = fmin(a, bb);
#pragma unroll
            for (int j = 0; j < LAG_MAX_THR; ++j)
                if (j < J && hi > lo * A.fac[j]) ++cnt[j];
        }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        acc += __shfl_xor(acc, s, 64);
        npairs += __shfl_xor(npairs, s, 64);
    }
#pragma unroll
    for (int j = 0; j < LAG_MAX_THR; ++j) {
        if (j < J) {  // uniform
            uint32_t v = cnt[j];
#pragma unroll
            for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, 64);
            if (lane == 0) wcnt[wv][1 + j] = v;
        }
    }
    if (lane == 0) {
        wsum[wv] = acc;
        wcnt[wv][0] = npairs;
    }
    __syncthreads();
    if (tid == 0) A.part_sum[g] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    if (tid <= J) A.part_cnt[g * (1 + J) + tid] = wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
}

// One workgroup per item: the item's partials in a fixed order.
__global__ __launch_bounds__(LAG_THREADS) void k_lag_finish(LagArgs A) {
    __shared__ double ssum[LAG_THREADS];
    __shared__ uint64_t scnt[LAG_THREADS];
    const int item = blockIdx.x, tid = threadIdx.x;
    const int64_t g0 = A.pre[item], g1 = A.pre[item + 1];
    const int c = item / A.K;
    const int64_t P = A.curves[c].n - A.lags[item - c * A.K];
    const int J = A.J;
    double acc = 0.0;
    for (int64_t g = g0 + tid; g < g1; g += LAG_THREADS) acc += A.part_sum[g];
    ssum[tid] = acc;
    __syncthreads();
    for (int s = LAG_THREADS / 2; s >= 1; s >>= 1) {
        if (tid < s) ssum[tid] += ssum[tid + s];
        __syncthreads();
    }
    if (tid == 0) A.sf2[item] = ssum[0] / (double)P;
    for (int j = 0; j <= J; ++j) {
        uint64_t v = 0;
        for (int64_t g = g0 + tid; g < g1; g += LAG_THREADS) v += A.part_cnt[g * (1 + J) + j];
        scnt[tid] = v;
        __syncthreads();
        for (int s = LAG_THREADS / 2; s >= 1; s >>= 1) {
            if (tid < s) scnt[tid] += scnt[tid + s];
            __syncthreads();
        }
        if (tid == 0) {
            if (j == 0 && A.pairs) A.pairs[item] = scnt[0];
            if (j > 0 && A.exceed) A.exceed[(int64_t)item * J + (j - 1)] = scnt[0];
        }
        __syncthreads();
    }
}

// Eq. 6: mean of SF^2 over the curves at each lag.  grid: ceil(K / 256).
__global__ __launch_bounds__(256) void k_lag_rep(const double* __restrict__ sf2, int32_t n_curves, int32_t K,
                                                 double* __restrict__ rep) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= K) return;
    double acc = 0.0;
    for (int c = 0; c < n_curves; ++c) acc += sf2[(int64_t)c * K + l];
    rep[l] = acc / (double)n_curves;
}

// ---------------------------------------------------------------------------
// Fit of Eq. 3 to each curve's log-binned periodogram (the convergence test
// of Sec. 3.2.2): least squares in log10 P, the break held at the input f_br,
// (a = log10 A, a_low, a_high) free; Levenberg-Marquardt from the input
// slopes, one wave per curve (its bins spread over the lanes).
// ---------------------------------------------------------------------------
struct FitDesc {
    const double* f;     // bin frequencies (mean f_j of the bin)
    const double* pbar;  // bin means of the periodogram
    double* out;         // {a, a_low, a_high, rms}
    double f_br, a_low0, a_high0;
    int32_t nb;
    int32_t pad_;
};

struct FitEval {
    double sse;
    double A[3][3];
    double g[3];
};

// Wave sum by an xor butterfly: every lane ends with the same bits (each
// stage adds two partial sums that are equal up to commutation).
AGN_DEV double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of squares, and if jac the normal equations, over the bins; the 64
// lanes of the wave take bins lane, lane + 64, ...
AGN_DEV void fit_eval(const FitDesc& d, const double th[3], bool jac, FitEval* e, int lane) {
    const double inv_ln10 = 0.43429448190325182765;
    double sse = 0.0, a00 = 0.0, a01 = 0.0, a02 = 0.0, a11 = 0.0, a12 = 0.0, a22 = 0.0, g0 = 0.0, g1 = 0.0,
           g2 = 0.0;
    for (int b = lane; b < d.nb; b += 64) {
        const double pb = d.pbar[b];
        if (!(pb > 0.0)) continue;
        const double lu = log(d.f[b] / d.f_br);
        const double tl = exp(th[1] * lu), tH = exp(th[2] * lu), S = tl + tH;
        const double r = log10(pb) - (th[0] - log10(S));
        sse += r * r;
        if (jac) {
            const double L = lu * inv_ln10;
            const double j1 = -tl / S * L, j2 = -tH / S * L;  // d model / d(a, a_low, a_high) = (1, j1, j2)
            a00 += 1.0;
            a01 += j1;
            a02 += j2;
            a11 += j1 * j1;
            a12 += j1 * j2;
            a22 += j2 * j2;
            g0 += r;
            g1 += j1 * r;
            g2 += j2 * r;
        }
    }
    e->sse = wave_sum(sse);
    if (jac) {
        e->A[0][0] = wave_sum(a00);
        e->A[0][1] = e->A[1][0] = wave_sum(a01);
        e->A[0][2] = e->A[2][0] = wave_sum(a02);
        e->A[1][1] = wave_sum(a11);
        e->A[1][2] = e->A[2][1] = wave_sum(a12);
        e->A[2][2] = wave_sum(a22);
        e->g[0] = wave_sum(g0);
        e->g[1] = wave_sum(g1);
        e->g[2] = wave_sum(g2);
    }
}

// Solves the symmetric positive definite 3x3 system M x = y by Cholesky.
AGN_DEV bool chol3(const double M[3][3], const double y[3], double x[3]) {
    const double l00 = M[0][0];
    if (!(l00 > 0.0)) return false;
    const double L00 = sqrt(l00), L10 = M[1][0] / L00, L20 = M[2][0] / L00;
    const double l11 = M[1][1] - L10 * L10;
    if (!(l11 > 0.0)) return false;
    const double L11 = sqrt(l11), L21 = (M[2][1] - L20 * L10) / L11;
    const double l22 = M[2][2] - L20 * L20 - L21 * L21;
    if (!(l22 > 0.0)) return false;
    const double L22 = sqrt(l22);
    const double z0 = y[0] / L00, z1 = (y[1] - L10 * z0) / L11, z2 = (y[2] - L20 * z0 - L21 * z1) / L22;
    x[2] = z2 / L22;
    x[1] = (z1 - L21 * x[2]) / L11;
    x[0] = (z0 - L10 * x[1] - L20 * x[2]) / L00;
    return true;
}

// grid: n_curves workgroups of one wave; all lanes run the same damping
// steps on the same (bit-identical) sums, lane 0 writes the result.
__global__ __launch_bounds__(64) void k_psd_fit(const FitDesc* __restrict__ descs, int32_t n_curves) {
    const int c = blockIdx.x, lane = threadIdx.x;
    if (c >= n_curves) return;
    const FitDesc d = descs[c];
    double cu = 0.0, cb = 0.0, ca = 0.0, s0 = 0.0;
    for (int b = lane; b < d.nb; b += 64)
        if (d.pbar[b] > 0.0) {
            cu += 1.0;
            cb += d.f[b] < d.f_br ? 1.0 : 0.0;
            ca += d.f[b] > d.f_br ? 1.0 : 0.0;
            const double lu = log(d.f[b] / d.f_br);
            s0 += log10(d.pbar[b]) + log10(exp(d.a_low0 * lu) + exp(d.a_high0 * lu));
        }
    const double used = wave_sum(cu), below = wave_sum(cb), above = wave_sum(ca);
    s0 = wave_sum(s0);
    if (used < 3.0 || below < 1.0 || above < 1.0) {
        if (lane < 4) d.out[lane] = __builtin_nan("");
        return;
    }
    double th[3] = {s0 / used, d.a_low0, d.a_high0};
    FitEval e;
    fit_eval(d, th, true, &e, lane);
    double lambda = 1e-3;
    for (int it = 0; it < 200; ++it) {
        bool moved = false;
        double rel = 0.0;
        while (lambda < 1e16) {
            double M[3][3], dx[3];
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) M[i][k] = e.A[i][k] + (i == k ? lambda * e.A[i][i] : 0.0);
            if (chol3(M, e.g, dx)) {
                const double tn[3] = {th[0] + dx[0], th[1] + dx[1], th[2] + dx[2]};
                FitEval en;
                fit_eval(d, tn, false, &en, lane);
                if (en.sse < e.sse) {
                    rel = 0.0;
                    for (int i = 0; i < 3; ++i) {
                        rel = fmax(rel, fabs(dx[i]) / (1.0 + fabs(th[i])));
                        th[i] = tn[i];
                    }
                    lambda = fmax(lambda / 3.0, 1e-15);
                    moved = true;
                    break;
                }
            }
            lambda *= 4.0;
        }
        if (!moved) break;  // no descent at any damping: at the minimum
        fit_eval(d, th, true, &e, lane);
        if (rel < 1e-15) break;
    }
    if (lane == 0) {
        // Eq. 3 is symmetric in its two slopes; the smaller one is the low-frequency slope
        d.out[0] = th[0];
        d.out[1] = fmin(th[1], th[2]);
        d.out[2] = fmax(th[1], th[2]);
        d.out[3] = sqrt(e.sse / used);
    }
}

}  // namespace agn
