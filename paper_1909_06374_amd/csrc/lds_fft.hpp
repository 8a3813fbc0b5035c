// lds_fft.hpp -- complex FFT of length M = 2^a 3^b held in LDS by one
// workgroup, and the real-to-complex / complex-to-real fold around the
// Fourier-modulus replacement of the light-curve iteration.
//
// Transform: self-sorting (Stockham) passes.  Pass with radix R over the
// current block size Ns: butterfly j (0 <= j < M/R) reads the R inputs
// buf[j + r M/R], multiplies input r by W_{Ns R}^{(j mod Ns) r}, takes a
// length-R DFT and writes output q to buf[(j - j mod Ns) R + j mod Ns + q Ns].
// After the last pass the data are in natural order.  Each thread reads all of
// its butterflies' inputs into registers, meets the workgroup barrier and then
// writes in place: one LDS buffer of M values (plus padding) suffices.
//
// Twiddles W_N^t = exp(-2 pi i t / N) for the real length N = 2M come from a
// two-level double-precision table in LDS (W_M^u = W_N^{2u}); the R - 1
// twiddles of one butterfly are double-precision powers of the first.
#pragma once
#include "common.hpp"

namespace agn {

struct FftPlan {
    int32_t npass;
    uint8_t radix[20];
};

// LDS address of complex element c: one pad element per 256 bytes, so that the
// strided writes of the first Stockham passes and the blocked reads of the
// sort spread over all 64 banks.
template <typename T>
AGN_DEV int cpad(int c) { return c + (c >> (sizeof(T) == 4 ? 5 : 4)); }
// LDS address (in T units) of real element p of the same buffer.
template <typename T>
AGN_DEV int rpad(int p) { return 2 * cpad<T>(p >> 1) + (p & 1); }
template <typename T>
__host__ __device__ inline int cpad_size(int m) { return m + (m >> (sizeof(T) == 4 ? 5 : 4)) + 1; }

// Twiddles W_N^t, 0 <= t < N, from a two-level table held in LDS:
// W_N^t = hi[t >> bits] * lo[t & (2^bits - 1)] with lo[u] = W_N^u and
// hi[v] = W_N^{v 2^bits}, both in double precision; the product is formed in
// double precision and rounded once to T.  Inverse = conjugate.
struct TwLds {
    const cplx<double>* lo;
    const cplx<double>* hi;
    int bits;
};

// bits of the low level for a length-N table (2^bits >= sqrt(N))
__host__ __device__ inline int tw_lds_bits(int N) {
    int lg = 0;
    while ((1 << lg) < N) ++lg;
    return (lg + 1) / 2;
}
// entries of the two levels together
__host__ __device__ inline int tw_lds_entries(int N) {
    const int b = tw_lds_bits(N);
    return (1 << b) + (N + (1 << b) - 1) / (1 << b);
}

template <typename T, bool INV>
AGN_DEV cplx<T> twiddle(const TwLds& tl, int t) {
    const cplx<double> a = tl.hi[t >> tl.bits];
    const cplx<double> b = tl.lo[t & ((1 << tl.bits) - 1)];
    const cplx<double> w = cmul(a, b);
    return cmk((T)w.re, (T)(INV ? -w.im : w.im));
}

// ---- small DFTs in registers; forward uses exp(-2 pi i / R) ----------------
template <typename T, bool INV>
AGN_DEV void dft2(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, bool INV>
AGN_DEV void dft3(cplx<T>* v) {
    const T c = (T)0.86602540378443864676;  // sqrt(3)/2
    cplx<T> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    cplx<T> m = cmk(v[0].re - (T)0.5 * t1.re, v[0].im - (T)0.5 * t1.im);
    // forward: X1 = m - i c t2, X2 = m + i c t2
    cplx<T> u = cmk(c * t2.im, -c * t2.re);  // -i c t2
    v[0] = cadd(v[0], t1);
    if (INV) {
        v[1] = csub(m, u);
        v[2] = cadd(m, u);
    } else {
        v[1] = cadd(m, u);
        v[2] = csub(m, u);
    }
}

template <typename T, bool INV>
AGN_DEV void dft4(cplx<T>* v) {
    cplx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cplx<T> s13 = cadd(v[1], v[3]);
    cplx<T> d13 = cmul_mi<T, INV>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <typename T, bool INV>
AGN_DEV void dft8(cplx<T>* v) {
    const T h = (T)0.70710678118654752440;
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, INV>(e);
    dft4<T, INV>(o);
    cplx<T> o1, o3;
    if (INV) {
        o1 = cmk(h * (o[1].re - o[1].im), h * (o[1].re + o[1].im));
        o3 = cmk(-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im));
    } else {
        o1 = cmk(h * (o[1].re + o[1].im), h * (o[1].im - o[1].re));
        o3 = cmk(h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im));
    }
    cplx<T> o2 = cmul_mi<T, INV>(o[2]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <typename T, int R, bool INV>
AGN_DEV void dftR(cplx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 3) dft3<T, INV>(v);
    else if constexpr (R == 4) dft4<T, INV>(v);
    else if constexpr (R == 8) dft8<T, INV>(v);
}

// One Stockham pass.  The M/R butterflies are dealt round-robin to the nt
// threads (at most BMAX per thread); all threads meet both barriers.  The
// twiddles depend only on the butterfly index, so they are fetched before the
// barrier.
template <typename T, int R, int BMAX, bool INV>
AGN_DEV void lds_pass(cplx<T>* buf, int M, int Ns, int tid, int nt, const TwLds& tw) {
    cplx<T> v[BMAX][R];
    cplx<T> w[BMAX][R];
    tid = opaque(tid);
    const int MR = M / R;
    const bool pow2 = (Ns & (Ns - 1)) == 0;
    const int tstep = 2 * (M / (Ns * R));
    // When a stride is a multiple of the pad period P, cpad(x + r * S) =
    // cpad(x) + r * (S + S / P): one base per butterfly, then fixed steps.
    constexpr int PL = sizeof(T) == 4 ? 5 : 4;
    const bool rd_al = (MR & ((1 << PL) - 1)) == 0, wr_al = (Ns & ((1 << PL) - 1)) == 0;
    const int rd_st = MR + (MR >> PL), wr_st = Ns + (Ns >> PL);
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int j = tid + b * nt;
        if (j < MR) {
            if (rd_al) {
                const int base = cpad<T>(j);
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = buf[base + r * rd_st];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = buf[cpad<T>(j + r * MR)];
            }
            if (Ns > 1) {
                const int jm = pow2 ? (j & (Ns - 1)) : (j % Ns);
                // W^{t r} for r = 1..R-1 as powers of W^t, formed by double-precision
                // products (R - 2 of them) and rounded once to T.  Power r is
                // the product of the powers floor(r / 2) and r - floor(r / 2), so
                // the chain of dependent products is log2(R) deep, not R - 2.
                const int t1 = jm * tstep;
                cplx<double> wp[R];
                wp[1] = cmul(tw.hi[t1 >> tw.bits], tw.lo[t1 & ((1 << tw.bits) - 1)]);
#pragma unroll
                for (int r = 2; r < R; ++r) wp[r] = cmul(wp[r / 2], wp[r - r / 2]);
#pragma unroll
                for (int r = 1; r < R; ++r) w[b][r] = cmk((T)wp[r].re, (T)(INV ? -wp[r].im : wp[r].im));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
        const int j = tid + b * nt;
        if (j < MR) {
            const int jm = pow2 ? (j & (Ns - 1)) : (j % Ns);
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], w[b][r]);
            }
            dftR<T, R, INV>(v[b]);
            const int d = (j - jm) * R + jm;
            if (wr_al) {
                const int base = cpad<T>(d);
#pragma unroll
                for (int r = 0; r < R; ++r) buf[base + r * wr_st] = v[b][r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) buf[cpad<T>(d + r * Ns)] = v[b][r];
            }
        }
    }
    __syncthreads();
}

// Passes p0 .. p1-1 of the plan, starting at stride Ns0; E = M / nt complex
// values per thread (compile-time bound).
template <typename T, int E, bool INV>
AGN_DEV void lds_fft_passes(cplx<T>* buf, int M, const FftPlan& plan, int p0, int p1, int Ns0, int tid, int nt,
                            const TwLds& tw) {
    int Ns = Ns0;
    for (int p = p0; p < p1; ++p) {
        const int R = plan.radix[p];
        if (R == 8) lds_pass<T, 8, (E + 7) / 8, INV>(buf, M, Ns, tid, nt, tw);
        else if (R == 4) lds_pass<T, 4, (E + 3) / 4, INV>(buf, M, Ns, tid, nt, tw);
        else if (R == 3) lds_pass<T, 3, (E + 2) / 3, INV>(buf, M, Ns, tid, nt, tw);
        else lds_pass<T, 2, (E + 1) / 2, INV>(buf, M, Ns, tid, nt, tw);
        Ns *= R;
    }
}

// Full transform.
template <typename T, int E, bool INV>
AGN_DEV void lds_fft(cplx<T>* buf, int M, const FftPlan& plan, int tid, int nt, const TwLds& tw) {
    lds_fft_passes<T, E, INV>(buf, M, plan, 0, plan.npass, 1, tid, nt, tw);
}

// Modulus replacement keeping the phase; zero modulus takes phase 0.  FP64:
// correctly rounded square root and divisions.  FP32 form: the hardware
// reciprocal square root of the squared modulus (about 1 ulp) and two
// products, instead of a square root and two divisions.
template <typename T>
AGN_DEV cplx<T> replace_modulus(cplx<T> X, T a) {
    if constexpr (sizeof(T) == 4) {
        const float m2 = X.re * X.re + X.im * X.im;
        if (m2 == 0.0f) return cmk(a, 0.0f);
        const float s = a * __builtin_amdgcn_rsqf(m2);
        return cmk(s * X.re, s * X.im);
    } else {
        T mod = sqrt(X.re * X.re + X.im * X.im);
        if (mod == (T)0) return cmk(a, (T)0);
        return cmk(a * (X.re / mod), a * (X.im / mod));
    }
}

// Z holds FFT_M(z), z[m] = x[2m] + i x[2m+1].  For every Hermitian pair
// (k, M-k) this forms the real-input spectrum X_k, X_{M-k}, replaces the
// moduli with amp (DC -> 0, Nyquist -> amp sign(Re X)), and writes back the
// length-M spectrum whose inverse FFT is y[2m] + i y[2m+1] with
// y = unnormalised inverse real DFT of Y.
//   X_k     = E_k + W_N^k O_k,          X_{M-k} = conj(E_k - W_N^k O_k)
//   E_k     = (Z_k + conj Z_{M-k}) / 2,  O_k = (Z_k - conj Z_{M-k}) / 2i
//   Z'_k    = A + i conj(W_N^k) B,       Z'_{M-k} = conj(A) + i W_N^k conj(B)
//   A       = Y_k + conj Y_{M-k},        B = Y_k - conj Y_{M-k}
// The two halves of fold_pair: the real-input spectrum of a Hermitian pair
// from the half-length transform (w = W_N^k) ...
template <typename T>
AGN_DEV void fold_spectrum(cplx<T> zk, cplx<T> zm, cplx<T> w, cplx<T>* Xk, cplx<T>* Xm) {
    const cplx<T> Ev = cmk((zk.re + zm.re) * (T)0.5, (zk.im - zm.im) * (T)0.5);
    const cplx<T> Ov = cmk((zk.im + zm.im) * (T)0.5, (zm.re - zk.re) * (T)0.5);
    const cplx<T> wO = cmul(w, Ov);
    *Xk = cadd(Ev, wO);
    *Xm = cconj(csub(Ev, wO));
}

// ... and the half-length spectrum whose inverse transform is the real series
// with half spectrum Y (Y_k, Y_{M-k} of one pair).
template <typename T>
AGN_DEV void unfold_pair(cplx<T> Yk, cplx<T> Ym, cplx<T> w, cplx<T>* yk, cplx<T>* ym) {
    const cplx<T> A = cadd(Yk, cconj(Ym));
    const cplx<T> B = csub(Yk, cconj(Ym));
    const cplx<T> cwB = cmul(cconj(w), B);
    *yk = cmk(A.re - cwB.im, A.im + cwB.re);  // A + i conj(w) B
    const cplx<T> wcB = cmul(w, cconj(B));
    *ym = cmk(A.re - wcB.im, -A.im + wcB.re);  // conj(A) + i w conj(B)
}

template <typename T>
AGN_DEV void fold_pair(cplx<T> zk, cplx<T> zm, cplx<T> w, T amp_k, T amp_m, cplx<T>* yk, cplx<T>* ym) {
    cplx<T> Xk, Xm;
    fold_spectrum(zk, zm, w, &Xk, &Xm);
    unfold_pair(replace_modulus(Xk, amp_k), replace_modulus(Xm, amp_m), w, yk, ym);
}

// DC and Nyquist (k = 0): Y_0 = 0, Y_M = amp_M sign(Re X_M).
template <typename T>
AGN_DEV cplx<T> fold_dc(cplx<T> z0, cplx<T> w0, T amp_n) {
    const cplx<T> Ev = cmk((z0.re + z0.re) * (T)0.5, (z0.im - z0.im) * (T)0.5);
    const cplx<T> Ov = cmk((z0.im + z0.im) * (T)0.5, (z0.re - z0.re) * (T)0.5);
    const cplx<T> wO = cmul(w0, Ov);
    const T xn = Ev.re - wO.re;  // X_M, real for real input
    const T yn = (xn >= (T)0) ? amp_n : -amp_n;
    return cmk(yn, -yn);
}

template <typename T, typename AmpPtr>
AGN_DEV void lds_fold_replace(cplx<T>* Z, int M, AmpPtr __restrict__ amp, const TwLds& tw, int tid,
                              int nthreads) {
    const int half = M / 2;
    for (int k = tid; k <= half; k += nthreads) {
        const int mk = (k == 0) ? 0 : M - k;
        const cplx<T> zk = Z[cpad<T>(k)], zm = Z[cpad<T>(mk)];
        const cplx<T> w = twiddle<T, false>(tw, k);
        if (k == 0) {
            Z[cpad<T>(0)] = fold_dc(zk, w, amp[M]);
        } else {
            cplx<T> yk, ym;
            fold_pair(zk, zm, w, amp[k], amp[M - k], &yk, &ym);
            Z[cpad<T>(k)] = yk;
            if (mk != k) Z[cpad<T>(mk)] = ym;
        }
    }
    __syncthreads();
}

// The forward plan's last pass is radix 2 (stride M/2), here fused with the
// fold / replacement.  On entry Z holds A = Z[0 .. M/2) and B = Z[M/2 .. M)
// of that pass; on return the replaced spectrum, as lds_fold_replace leaves
// it.  For k in [0, M/4] one thread takes the pairs (k, M - k) and
// (M/2 - k, M/2 + k), whose four spectrum values come from A and B at k and
// M/2 - k:  Z_k = A_k + W_M^k B_k,  Z_{M/2+k} = A_k - W_M^k B_k.  It reads and
// writes the same four positions, so no other thread's data is touched and
// no barrier is needed between the reads and the writes.  The operations are
// those of the separate pass and fold (the compiler may fuse multiply-adds
// differently, so results can differ in the last bit).  Needs M >= 16.
template <typename T, typename AmpPtr>
AGN_DEV void lds_fold_replace_r2(cplx<T>* Z, int M, AmpPtr __restrict__ amp, const TwLds& tw, int tid,
                                 int nt) {
    const int h = M / 2, q = M / 4;
    for (int k = tid; k <= q; k += nt) {
        const cplx<T> a0 = Z[cpad<T>(k)], b0 = Z[cpad<T>(k + h)];
        // last forward pass (radix 2): W_M^k = W_N^{2k}
        const cplx<T> t0 = cmul(b0, twiddle<T, false>(tw, 2 * k));
        const cplx<T> zk = cadd(a0, t0), zhk = csub(a0, t0);  // Z_k, Z_{h+k}
        if (k == 0) {
            cplx<T> yh, unused;
            fold_pair(zhk, zhk, twiddle<T, false>(tw, h), amp[h], amp[h], &yh, &unused);  // self pair h
            Z[cpad<T>(0)] = fold_dc(zk, twiddle<T, false>(tw, 0), amp[M]);
            Z[cpad<T>(h)] = yh;
            continue;
        }
        if (k == q) {
            // (q, 3q) is its own partner: Z_{3q} = Z_{h+q}
            cplx<T> yq, y3q;
            fold_pair(zk, zhk, twiddle<T, false>(tw, q), amp[q], amp[M - q], &yq, &y3q);
            Z[cpad<T>(q)] = yq;
            Z[cpad<T>(3 * q)] = y3q;
            continue;
        }
        const cplx<T> a1 = Z[cpad<T>(h - k)], b1 = Z[cpad<T>(M - k)];
        const cplx<T> t1 = cmul(b1, twiddle<T, false>(tw, 2 * (h - k)));  // W_M^{h-k}
        const cplx<T> zh_k = cadd(a1, t1), zm_k = csub(a1, t1);          // Z_{h-k}, Z_{M-k}
        cplx<T> y_k, y_mk, y_hk, y_hpk;
        fold_pair(zk, zm_k, twiddle<T, false>(tw, k), amp[k], amp[M - k], &y_k, &y_mk);
        fold_pair(zh_k, zhk, twiddle<T, false>(tw, h - k), amp[h - k], amp[h + k], &y_hk, &y_hpk);
        Z[cpad<T>(k)] = y_k;
        Z[cpad<T>(M - k)] = y_mk;
        Z[cpad<T>(h - k)] = y_hk;
        Z[cpad<T>(h + k)] = y_hpk;
    }
    __syncthreads();
}

}  // namespace agn
