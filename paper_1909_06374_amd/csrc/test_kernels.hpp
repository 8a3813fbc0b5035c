// test_kernels.hpp -- the iteration's FFT and ranking kernels run on their own
// (the test exports of the C ABI), so that each step can be compared with a
// plain implementation of its definition: the real DFT of App. A (forward
// sign exp(-2 pi i jk/N)), its unnormalised inverse, and the stable argsort of
// Sec. 2.1.  The transforms and the sort are the path's own device code (the
// Stockham passes, the real-spectrum fold, the radix sorts); only the loads
// and stores at the ends differ, because the path never materialises the
// spectrum it replaces (on the multi-pass path the middle pass's spectrum and
// unfold modes, k_fft_mid, take the place of its replacement).
#pragma once
#include "common.hpp"
#include "lds_fft.hpp"
#include "lds_sort.hpp"
#include "lds_iterate.hpp"
#include "big_path.hpp"

namespace agn {

enum { TEST_RFFT = 0, TEST_IRFFT = 1, TEST_RANK = 2 };

struct TestLds {
    int32_t n;
    int32_t mode;          // TEST_*
    const double* in;      // RFFT / RANK: n reals; IRFFT: n/2 + 1 complex (re, im)
    double* out;           // RFFT: n/2 + 1 complex; IRFFT: n reals
    uint32_t* rank_out;    // RANK: rank_out[t] = sorted position of sample t
    const void* tw;        // cplx<double>[n/2 + 1], W_N^t
    FftPlan plan;          // radices of the length-n/2 complex FFT
};

// One workgroup, the LDS layout and block shape of the iteration kernel.
// RFFT: the forward passes, then the spectrum half of the fold for every
// Hermitian pair.  IRFFT: the unfold half for every pair (the DC and Nyquist
// values, real, enter as Z_0 = (Y_0 + Y_M) + i (Y_0 - Y_M)), then the inverse
// passes.  RANK: the iteration's ranking of y (lds_rank_series).
template <typename T, int E>
__global__ __launch_bounds__(1024) void k_test_lds(const TestLds* __restrict__ dp) {
    constexpr int IPT = 2 * E;
    extern __shared__ __align__(16) unsigned char smem[];
    const TestLds& d = *dp;
    const int N = d.n, M = N / 2;
    const int tid = threadIdx.x, nt = blockDim.x;
    size_t ib_off, rk_off, sc_off, tw_off;
    lds_iter_layout<T>(N, nt, &ib_off, &rk_off, &sc_off, &tw_off);
    cplx<T>* Zc = (cplx<T>*)smem;
    T* Zf = (T*)smem;
    uint16_t* ibuf = (uint16_t*)(smem + ib_off);
    uint32_t* scratch = (uint32_t*)(smem + sc_off);
    const TwLds tw = lds_load_twiddles(smem + tw_off, (const cplx<double>*)d.tw, N, tid, nt);
    __syncthreads();
    if (d.mode == TEST_IRFFT) {
        for (int k = tid; k <= M / 2; k += nt) {
            if (k == 0) {
                const T y0 = (T)d.in[0], yM = (T)d.in[2 * M];
                Zc[cpad<T>(0)] = cmk(y0 + yM, y0 - yM);
                continue;
            }
            const cplx<T> Yk = cmk((T)d.in[2 * k], (T)d.in[2 * k + 1]);
            const cplx<T> Ym = cmk((T)d.in[2 * (M - k)], (T)d.in[2 * (M - k) + 1]);
            cplx<T> yk, ym;
            unfold_pair(Yk, Ym, twiddle<T, false>(tw, k), &yk, &ym);
            Zc[cpad<T>(k)] = yk;
            if (M - k != k) Zc[cpad<T>(M - k)] = ym;
        }
        __syncthreads();
        lds_fft<T, E, true>(Zc, M, d.plan, tid, nt, tw);
        for (int p = tid; p < N; p += nt) d.out[p] = (double)Zf[rpad<T>(p)];
        return;
    }
    for (int p = tid; p < N; p += nt) Zf[rpad<T>(p)] = (T)d.in[p];
    __syncthreads();
    if (d.mode == TEST_RFFT) {
        lds_fft<T, E, false>(Zc, M, d.plan, tid, nt, tw);
        for (int k = tid; k <= M / 2; k += nt) {
            const int mk = (k == 0) ? 0 : M - k;
            cplx<T> Xk, Xm;
            fold_spectrum(Zc[cpad<T>(k)], Zc[cpad<T>(mk)], twiddle<T, false>(tw, k), &Xk, &Xm);
            d.out[2 * k] = (double)Xk.re;
            d.out[2 * k + 1] = (double)Xk.im;
            if (M - k != k) {
                d.out[2 * (M - k)] = (double)Xm.re;
                d.out[2 * (M - k) + 1] = (double)Xm.im;
            }
        }
        return;
    }
    lds_rank_series<T, IPT>(Zf, smem, ibuf, scratch, tid, nt);
    for (int k = tid; k < N; k += nt) d.rank_out[ibuf[hpad(k)]] = (uint32_t)k;
}

// Multi-pass path, one curve (descriptor cv[0]).
// y[p] = the real view of the complex buffer in region `sel`.  grid: ceil(n / 256), block 256.
template <typename T>
__global__ __launch_bounds__(256) void k_test_big_real(const BigCurve* __restrict__ cv, int64_t n, int sel,
                                                       double* __restrict__ y) {
    const BigCurve& d = cv[0];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const T* Z = (const T*)(sel ? d.sortB : d.sortA);
    y[p] = (double)Z[p];
}

// Order-preserving keys of y rounded to T, into region A (as the last
// inverse pass writes them).  grid: ceil(n / 256), block 256.
template <typename T>
__global__ __launch_bounds__(256) void k_test_big_keys(const BigCurve* __restrict__ cv, int64_t n,
                                                       const double* __restrict__ y) {
    typedef typename key_of<T>::type K;
    const BigCurve& d = cv[0];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    ((K*)d.sortA)[p] = ord_key((T)y[p]);
}

// LDS read bandwidth probe (the ceiling of the LDS-resident kernels'
// LDS traffic): every thread of a 1024-thread workgroup reads 16-byte words
// of a 64 KB LDS buffer, consecutive lanes consecutive words (no bank
// conflicts), `reps` times over; the sum of what it read goes to out, so
// the loads cannot be removed.  Bytes read per workgroup: reps * 64 KB.
// grid: any, block 1024.
__global__ __launch_bounds__(1024) void k_lds_read_bw(int reps, float* __restrict__ out) {
    __shared__ float4 buf[4096];
    const int t = threadIdx.x;
    for (int i = t; i < 4096; i += 1024) buf[i] = make_float4((float)i, 1.0f, 2.0f, 3.0f);
    __syncthreads();
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int r = 0; r < reps; ++r) {
        const int base = opaque(r & 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float4 v = buf[(t + k * 1024 + base) & 4095];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    }
    out[(size_t)blockIdx.x * 1024 + t] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace agn
