// observables.hpp -- the periodogram of App. A (Eq. A2) for a batch of real
// series, e.g. the generator's output, and its means over logarithmic
// frequency bins: P_j = 2 / N^2 |X_j|^2, X_j = sum_t x[t] exp(-2 pi i j t / N),
// j = 0..N/2, in double precision.
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

}  // namespace agn
