/*
 * agn_oracle.c -- plain FP64 CPU oracle for the light-curve generator of
 * Sartori et al. (2019), arXiv:1909.06374 (Sec. 2.1, Sec. 3.1, Sec. 3.2.2,
 * Eqs. 3, 4, A1, A2), which runs the Emmanoulopoulos et al. (2013) iteration
 * (a Timmer & Koenig (1995) random spectrum, then repeated amplitude
 * replacement in Fourier space and rank-order substitution of the PDF draw).
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark are the only users.  It shares nothing
 * with the GPU library.
 *
 * Style: each step is the textbook definition, written out with no blocking,
 * fusion or reordering; speed is not a goal.
 *
 * Readings taken where the paper is silent (they are listed in the design
 * notes as well):
 *  - TK95 moduli: only the Fourier moduli of the TK95 spectrum are kept by
 *    the iteration (Sec. 2.1), so each interior bin's modulus is drawn as
 *    sqrt(P_j * E), E ~ Exp(1) = -ln U, which equals |sqrt(P/2)(g1 + i g2)| in
 *    distribution.  The Nyquist bin is real: sqrt(P/2)|g|, g by Box-Muller.
 *    The DC bin is 0.
 *  - Forward DFT uses exp(-2 pi i jk/N) and the inverse exp(+...); Eq. A1
 *    prints the opposite sign, which only conjugates both spectra and leaves
 *    the real output unchanged.
 *  - The inverse DFT is unnormalised (a positive scale does not change ranks).
 *  - A zero-modulus bin takes phase 0; the Nyquist bin keeps the sign of its
 *    real part (sign(0) = +1).
 *  - Eq. 4's log is log10 and rms is over all N samples.
 *  - Ties in the sort break by time index; -0 and +0 are equal.
 */
#include "agn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define E_OK 0
#define E_INVAL (-1)
#define E_SIZE (-2)
#define E_NOMEM (-3)

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 64x64->128 multiplications,   */
/* with a Weyl-sequence key schedule.                                        */
/* ------------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

void agn_oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream layout: key = (seed, stream << 32 | curve_id), counter = (k / 4, 0, 0, 0),
 * uniform #k is word k % 4.  A 64-bit word w maps to ((w >> 12) + 1/2) 2^-52, which
 * is exact in FP64 and lies in [2^-53, 1 - 2^-53]. */
double agn_oracle_uniform(uint64_t seed, uint32_t stream, uint32_t curve_id, uint64_t k)
{
    uint64_t key[2] = {seed, ((uint64_t)stream << 32) | (uint64_t)curve_id};
    uint64_t ctr[4] = {k / 4, 0, 0, 0};
    uint64_t out[4];
    agn_oracle_philox4x64(ctr, key, out);
    uint64_t w = out[k % 4];
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

/* ------------------------------------------------------------------------ */
/* PSD, Eq. 3, on the Fourier grid f_j = j / (N dt) of Appendix A.           */
/* ------------------------------------------------------------------------ */
double agn_oracle_psd_eq3(double f, double A, double f_br, double a_low, double a_high)
{
    double r = f / f_br;
    return A / (pow(r, a_low) + pow(r, a_high));
}

static int valid_n(int64_t n)
{
    if (n < 1) return 0;
    int64_t m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

double agn_oracle_psd_norm(const agn_oracle_psd_params* p, int64_t n, double dt)
{
    if (p->norm > 0.0) return p->norm;
    /* Unit expected variance of the (1/N-normalised) TK95 series:
     * Var = (1/N^2) [ 2 sum_{j=1}^{N/2-1} P_j + P_{N/2} / 2 ]. */
    double s = 0.0;
    for (int64_t j = 1; j < n / 2; ++j)
        s += 2.0 * agn_oracle_psd_eq3((double)j / ((double)n * dt), 1.0, p->f_br, p->a_low, p->a_high);
    s += 0.5 * agn_oracle_psd_eq3(0.5 / dt, 1.0, p->f_br, p->a_low, p->a_high);
    return (double)n * (double)n / s;
}

static int valid_params(const agn_oracle_psd_params* p, double dt)
{
    if (!(dt > 0.0) || !isfinite(dt)) return 0;
    if (!(p->f_br > 0.0) || !isfinite(p->f_br)) return 0;
    if (!isfinite(p->a_low) || !isfinite(p->a_high) || !isfinite(p->norm)) return 0;
    return 1;
}

int agn_oracle_psd_spectrum(const agn_oracle_psd_params* p, int64_t n, double dt,
                            uint64_t seed, uint32_t curve_id, double* amp)
{
    if (!p || !amp) return E_INVAL;
    if (n < 2 || n % 2 != 0 || !valid_n(n)) return E_SIZE;
    if (!valid_params(p, dt)) return E_INVAL;
    double A = agn_oracle_psd_norm(p, n, dt);
    int64_t h = n / 2;
    amp[0] = 0.0;
    for (int64_t j = 1; j < h; ++j) {
        double P = agn_oracle_psd_eq3((double)j / ((double)n * dt), A, p->f_br, p->a_low, p->a_high);
        double U = agn_oracle_uniform(seed, 0, curve_id, (uint64_t)j);
        amp[j] = sqrt(P * (-log(U)));
    }
    {
        double P = agn_oracle_psd_eq3(0.5 / dt, A, p->f_br, p->a_low, p->a_high);
        double Ua = agn_oracle_uniform(seed, 0, curve_id, (uint64_t)h);
        double Ub = agn_oracle_uniform(seed, 0, curve_id, (uint64_t)h + 1);
        double g = sqrt(-2.0 * log(Ua)) * cos(2.0 * M_PI * Ub);
        amp[h] = sqrt(0.5 * P) * fabs(g);
    }
    return E_OK;
}

/* ------------------------------------------------------------------------ */
/* DFT: recursive mixed-radix (2, 3) Cooley-Tukey, decimation in time.       */
/* X[k] = sum_r W_n^{rk} F_r[k mod m], F_r = DFT_m of x[p t + r].            */
/* Each twiddle is cos/sin of 2 pi ((r k) mod n) / n, computed directly.     */
/* ------------------------------------------------------------------------ */
static int dft_rec(const double* x, int64_t stride, int64_t n, int sign, double* X)
{
    if (n == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return E_OK;
    }
    int64_t p = (n % 2 == 0) ? 2 : 3;
    int64_t m = n / p;
    double* F = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!F) return E_NOMEM;
    for (int64_t r = 0; r < p; ++r) {
        int rc = dft_rec(x + 2 * stride * r, stride * p, m, sign, F + 2 * m * r);
        if (rc) { free(F); return rc; }
    }
    for (int64_t k = 0; k < n; ++k) {
        double re = 0.0, im = 0.0;
        for (int64_t r = 0; r < p; ++r) {
            /* W = exp(sign 2 pi i t / n); the quarter turns are exact
             * (1, sign i, -1, -sign i), as the roots of unity they are, so
             * that a bin whose exact value is zero comes out as zero and
             * takes the zero-modulus phase of the replacement */
            const int64_t t = (r * k) % n;
            double wr, wi;
            if ((4 * t) % n == 0) {
                const int64_t q = 4 * t / n;
                wr = q == 0 ? 1.0 : q == 2 ? -1.0 : 0.0;
                wi = q == 1 ? (double)sign : q == 3 ? -(double)sign : 0.0;
            } else {
                double ang = (double)sign * 2.0 * M_PI * (double)t / (double)n;
                wr = cos(ang);
                wi = sin(ang);
            }
            double fr = F[2 * (m * r + k % m)], fi = F[2 * (m * r + k % m) + 1];
            re += wr * fr - wi * fi;
            im += wr * fi + wi * fr;
        }
        X[2 * k] = re;
        X[2 * k + 1] = im;
    }
    free(F);
    return E_OK;
}

int agn_oracle_dft(double* data, int64_t n, int sign)
{
    if (!data) return E_INVAL;
    if (!valid_n(n)) return E_SIZE;
    if (sign != 1 && sign != -1) return E_INVAL;
    double* out = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!out) return E_NOMEM;
    int rc = dft_rec(data, 1, n, sign, out);
    if (!rc) memcpy(data, out, sizeof(double) * 2 * (size_t)n);
    free(out);
    return rc;
}

int agn_oracle_rfft(const double* x, int64_t n, double* X)
{
    if (!x || !X) return E_INVAL;
    if (n < 2 || n % 2 != 0 || !valid_n(n)) return E_SIZE;
    double* z = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!z) return E_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        z[2 * i] = x[i];
        z[2 * i + 1] = 0.0;
    }
    int rc = agn_oracle_dft(z, n, -1);
    if (!rc) memcpy(X, z, sizeof(double) * 2 * (size_t)(n / 2 + 1));
    free(z);
    return rc;
}

/* Real part of the unnormalised inverse DFT of the Hermitian extension
 * Z[k] = Y[k] (k <= n/2), Z[n-k] = conj(Y[k]) (0 < k < n/2). */
int agn_oracle_irfft(const double* Y, int64_t n, double* y)
{
    if (!Y || !y) return E_INVAL;
    if (n < 2 || n % 2 != 0 || !valid_n(n)) return E_SIZE;
    double* z = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!z) return E_NOMEM;
    int64_t h = n / 2;
    for (int64_t k = 0; k <= h; ++k) {
        z[2 * k] = Y[2 * k];
        z[2 * k + 1] = Y[2 * k + 1];
    }
    for (int64_t k = 1; k < h; ++k) {
        z[2 * (n - k)] = Y[2 * k];
        z[2 * (n - k) + 1] = -Y[2 * k + 1];
    }
    int rc = agn_oracle_dft(z, n, +1);
    if (!rc)
        for (int64_t i = 0; i < n; ++i) y[i] = z[2 * i];
    free(z);
    return rc;
}

/* Amplitude replacement (Sec. 2.1, Sec. 3.2.2): keep the phase of X, take the
 * modulus from amp.  DC -> 0; Nyquist -> amp * sign(Re X) with sign(0) = +1;
 * a zero-modulus bin takes phase 0. */
int agn_oracle_replace(const double* X, const double* amp, int64_t n, double* Y)
{
    if (!X || !amp || !Y) return E_INVAL;
    if (n < 2 || n % 2 != 0) return E_SIZE;
    int64_t h = n / 2;
    for (int64_t j = 1; j < h; ++j) {
        double re = X[2 * j], im = X[2 * j + 1];
        double mod = sqrt(re * re + im * im);
        if (mod == 0.0) {
            Y[2 * j] = amp[j];
            Y[2 * j + 1] = 0.0;
        } else {
            Y[2 * j] = amp[j] * (re / mod);
            Y[2 * j + 1] = amp[j] * (im / mod);
        }
    }
    {
        double re = X[2 * h];
        Y[2 * h] = (re >= 0.0) ? amp[h] : -amp[h];
        Y[2 * h + 1] = 0.0;
    }
    Y[0] = 0.0;
    Y[1] = 0.0;
    return E_OK;
}

/* ------------------------------------------------------------------------ */
/* Stable ascending argsort.  The comparator orders (value, index) pairs, a  */
/* total order, so the unstable library sort returns the stable result.      */
/* ------------------------------------------------------------------------ */
static _Thread_local const double* g_sort_keys;

static int cmp_idx(const void* a, const void* b)
{
    uint32_t ia = *(const uint32_t*)a, ib = *(const uint32_t*)b;
    double ya = g_sort_keys[ia], yb = g_sort_keys[ib];
    if (ya < yb) return -1;
    if (ya > yb) return 1;
    return (ia < ib) ? -1 : (ia > ib) ? 1 : 0;
}

int agn_oracle_argsort(const double* y, int64_t n, uint32_t* perm)
{
    if (!y || !perm) return E_INVAL;
    if (n < 0 || n > (int64_t)0xFFFFFFFFLL) return E_SIZE;
    for (int64_t i = 0; i < n; ++i)
        if (isnan(y[i])) return E_INVAL;
    for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    g_sort_keys = y;
    qsort(perm, (size_t)n, sizeof(uint32_t), cmp_idx);
    g_sort_keys = NULL;
    return E_OK;
}

/* ------------------------------------------------------------------------ */
/* The iteration (Sec. 2.1, Sec. 3.2.2):                                     */
/*   s      = PDF draw sorted ascending (values fixed for the whole run)     */
/*   x_0    = PDF draw in draw order                                         */
/*   y      = IDFT(replace(DFT(x_{i-1}), amp))                               */
/*   x_i    = s placed in the rank order of y                                */
/*   delta_i = rms_n log10(x_i[n] / x_{i-1}[n])            (Eq. 4)            */
/* Stopping: tol < 0 runs all iterations; tol >= 0 stops after the first     */
/* iteration that reaches an exact fixed point, or (tol > 0) delta_i <= tol. */
/* ------------------------------------------------------------------------ */
int agn_oracle_iterate(const double* amp, const double* x0, int64_t n, int32_t iters,
                       double tol, double* x_out, double* delta_out, int32_t* iters_done,
                       uint32_t* rank_out)
{
    if (!amp || !x0 || !x_out) return E_INVAL;
    if (n < 2 || n % 2 != 0 || !valid_n(n) || n > ((int64_t)1 << 31)) return E_SIZE;
    if (iters < 0) return E_INVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!(x0[i] > 0.0) || !isfinite(x0[i])) return E_INVAL;

    int64_t h = n / 2;
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double* xp = (double*)malloc(sizeof(double) * (size_t)n);
    double* xn = (double*)malloc(sizeof(double) * (size_t)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    double* X = (double*)malloc(sizeof(double) * 2 * (size_t)(h + 1));
    uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
    int rc = E_OK;
    if (!s || !xp || !xn || !y || !X || !perm) { rc = E_NOMEM; goto done; }

    rc = agn_oracle_argsort(x0, n, perm);
    if (rc) goto done;
    for (int64_t k = 0; k < n; ++k) s[k] = x0[perm[k]];
    if (rank_out)
        for (int64_t k = 0; k < n; ++k) rank_out[perm[k]] = (uint32_t)k;
    memcpy(xp, x0, sizeof(double) * (size_t)n);
    if (delta_out)
        for (int32_t i = 0; i < iters; ++i) delta_out[i] = 0.0;

    int32_t done_count = 0;
    for (int32_t it = 0; it < iters; ++it) {
        if ((rc = agn_oracle_rfft(xp, n, X))) goto done;
        if ((rc = agn_oracle_replace(X, amp, n, X))) goto done;
        if ((rc = agn_oracle_irfft(X, n, y))) goto done;
        if ((rc = agn_oracle_argsort(y, n, perm))) goto done;
        for (int64_t k = 0; k < n; ++k) xn[perm[k]] = s[k];
        if (rank_out)
            for (int64_t k = 0; k < n; ++k) rank_out[perm[k]] = (uint32_t)k;

        double acc = 0.0;
        int same = 1;
        for (int64_t i = 0; i < n; ++i) {
            double l = log10(xn[i] / xp[i]);
            acc += l * l;
            if (xn[i] != xp[i]) same = 0;
        }
        double delta = sqrt(acc / (double)n);
        if (delta_out) delta_out[it] = delta;
        memcpy(xp, xn, sizeof(double) * (size_t)n);
        done_count = it + 1;
        if (tol >= 0.0 && (same || (tol > 0.0 && delta <= tol))) break;
    }
    memcpy(x_out, xp, sizeof(double) * (size_t)n);
    if (iters_done) *iters_done = done_count;

done:
    free(s); free(xp); free(xn); free(y); free(X); free(perm);
    return rc;
}

int agn_oracle_generate(const agn_oracle_psd_params* p, const double* erdf, int64_t n,
                        double dt, int32_t iters, double tol, uint64_t seed,
                        uint32_t curve_id, double* x_out, double* delta_out,
                        int32_t* iters_done, uint32_t* rank_out)
{
    if (!p || !erdf || !x_out) return E_INVAL;
    if (n < 2 || n % 2 != 0 || !valid_n(n)) return E_SIZE;
    double* amp = (double*)malloc(sizeof(double) * (size_t)(n / 2 + 1));
    if (!amp) return E_NOMEM;
    int rc = agn_oracle_psd_spectrum(p, n, dt, seed, curve_id, amp);
    if (!rc)
        rc = agn_oracle_iterate(amp, erdf, n, iters, tol, x_out, delta_out, iters_done, rank_out);
    free(amp);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* PDF draw: inverse CDF of the sharp broken power law in u = log10(lambda). */
/*   M1 = int_{u_min}^{u_br} 10^{-d1 (u - u_br)} du                          */
/*      = (10^{d1 (u_br - u_min)} - 1) / (d1 ln 10)                           */
/*   M2 = int_{u_br}^{u_max} 10^{-d2 (u - u_br)} du                          */
/*      = (1 - 10^{-d2 (u_max - u_br)}) / (d2 ln 10)                          */
/* t = U (M1 + M2); below the break the CDF integral equals t at             */
/*   u = u_br - log10(10^{d1 (u_br - u_min)} - t d1 ln 10) / d1,             */
/* above it at u = u_br - log10(1 - (t - M1) d2 ln 10) / d2.                 */
/* ------------------------------------------------------------------------ */
int agn_oracle_erdf_bpl(const agn_oracle_erdf_params* p, int64_t n, uint64_t seed,
                        uint32_t curve_id, double* out)
{
    if (!p || !out || n < 0) return E_INVAL;
    if (!(p->u_min < p->u_br && p->u_br < p->u_max) || !(p->d1 != 0.0) || !(p->d2 != 0.0)) return E_INVAL;
    const double ln10 = log(10.0);
    const double m1 = (pow(10.0, p->d1 * (p->u_br - p->u_min)) - 1.0) / (p->d1 * ln10);
    const double m2 = (1.0 - pow(10.0, -p->d2 * (p->u_max - p->u_br))) / (p->d2 * ln10);
    for (int64_t k = 0; k < n; ++k) {
        const double U = agn_oracle_uniform(seed, 1, curve_id, (uint64_t)k);
        const double t = U * (m1 + m2);
        double u;
        if (t < m1) {
            u = p->u_br - log10(pow(10.0, p->d1 * (p->u_br - p->u_min)) - t * p->d1 * ln10) / p->d1;
        } else {
            u = p->u_br - log10(1.0 - (t - m1) * p->d2 * ln10) / p->d2;
        }
        if (u < p->u_min) u = p->u_min;
        if (u > p->u_max) u = p->u_max;
        out[k] = pow(10.0, u);
    }
    return E_OK;
}

/* ------------------------------------------------------------------------ */
/* General PDF draw (Sec. 2.1 step ii; Eq. 1, Eq. 2).                         */
/* ------------------------------------------------------------------------ */
static const double LN10 = 2.302585092994045684;

/* Shape of the density in u = log10(lambda), up to a constant. */
static double pdf_shape_u(const agn_oracle_pdf_params* p, double u)
{
    const double x = u - p->u_star;
    double f;
    if (p->kind == 0) f = pow(10.0, -(x < 0.0 ? p->d1 : p->d2) * x);
    else if (p->kind == 1) f = 1.0 / (pow(10.0, p->d1 * x) + pow(10.0, p->d2 * x));
    else f = exp(-x * x / (2.0 * p->sigma * p->sigma));
    if (p->measure == 1) f *= pow(10.0, x);  /* dN/du = dN/dlambda * lambda ln10 */
    return f;
}

/* 20-point Gauss-Legendre integral of the shape over [a, b]. */
static double pdf_gl(const agn_oracle_pdf_params* p, double a, double b)
{
    static const double xg[10] = {0.0765265211334973338, 0.2277858511416450781, 0.3737060887154195607,
                                  0.5108670019508270980, 0.6360536807265150254, 0.7463319064601507926,
                                  0.8391169718222188234, 0.9122344282513259059, 0.9639719272779137912,
                                  0.9931285991850949248};
    static const double wg[10] = {0.1527533871307258507, 0.1491729864726037467, 0.1420961093183820514,
                                  0.1316886384491766269, 0.1181945319615184174, 0.1019301198172404351,
                                  0.0832767415767047487, 0.0626720483341090636, 0.0406014298003869413,
                                  0.0176140071391521183};
    const double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double s = 0.0;
    for (int i = 0; i < 10; ++i) s += wg[i] * (pdf_shape_u(p, c - h * xg[i]) + pdf_shape_u(p, c + h * xg[i]));
    return s * h;
}

/* Standard normal CDF and its complement. */
static double phi_lo(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

/* Inverse CDF of one uniform for kinds 0 and 2 (closed form / bisection on erfc). */
static double pdf_invert_analytic(const agn_oracle_pdf_params* p, double U)
{
    if (p->kind == 0) {
        /* closed form: the density in u is 10^(-e1 (u - u*)) below and 10^(-e2 (u - u*)) above */
        const double e1 = p->d1 - (p->measure == 1 ? 1.0 : 0.0), e2 = p->d2 - (p->measure == 1 ? 1.0 : 0.0);
        const double a = p->u_star - p->u_min, b = p->u_max - p->u_star;
        const double m1 = (e1 == 0.0) ? a : (pow(10.0, e1 * a) - 1.0) / (e1 * LN10);
        const double m2 = (e2 == 0.0) ? b : (1.0 - pow(10.0, -e2 * b)) / (e2 * LN10);
        const double t = U * (m1 + m2);
        double u;
        if (t < m1) u = (e1 == 0.0) ? p->u_min + t : p->u_star - log10(pow(10.0, e1 * a) - t * e1 * LN10) / e1;
        else u = (e2 == 0.0) ? p->u_star + (t - m1) : p->u_star - log10(1.0 - (t - m1) * e2 * LN10) / e2;
        if (u < p->u_min) u = p->u_min;
        if (u > p->u_max) u = p->u_max;
        return u;
    }
    /* kind 2: normal in u truncated to [u_min, u_max]; for the linear measure the
     * extra factor 10^(u - u*) completes the square to a mean of u* + sigma^2 ln10 */
    const double mu = p->u_star + (p->measure == 1 ? p->sigma * p->sigma * LN10 : 0.0);
    /* a support above the mean is reflected about it, so that the normal CDF is
     * always taken in its lower half, where it keeps full relative precision;
     * the reflected draw uses the exact complement 1 - U */
    const int mirror = 0.5 * (p->u_min + p->u_max) > mu;
    const double a = mirror ? 2.0 * mu - p->u_max : p->u_min;
    const double b = mirror ? 2.0 * mu - p->u_min : p->u_max;
    const double fa = phi_lo((a - mu) / p->sigma), fb = phi_lo((b - mu) / p->sigma);
    const double target = fa + (mirror ? 1.0 - U : U) * (fb - fa);
    double lo = a, hi = b;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * (1.0 + fabs(lo)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (phi_lo((mid - mu) / p->sigma) < target) lo = mid;
        else hi = mid;
    }
    const double v = 0.5 * (lo + hi);
    return mirror ? 2.0 * mu - v : v;
}

int agn_oracle_pdf_draw_at(const agn_oracle_pdf_params* p, uint64_t seed, uint32_t curve_id,
                           const int64_t* idx, int64_t m, double* out)
{
    if (!p || m < 0 || (m > 0 && (!idx || !out))) return E_INVAL;
    if (!(p->u_min < p->u_max) || !isfinite(p->u_min) || !isfinite(p->u_max) || !isfinite(p->u_star))
        return E_INVAL;
    if (p->kind < 0 || p->kind > 2 || (p->measure != 0 && p->measure != 1)) return E_INVAL;
    if (p->kind == 0 && !(p->u_min < p->u_star && p->u_star < p->u_max)) return E_INVAL;
    if (p->kind != 2 && (!isfinite(p->d1) || !isfinite(p->d2))) return E_INVAL;
    if (p->kind == 2 && !(p->sigma > 0.0 && isfinite(p->sigma))) return E_INVAL;
    for (int64_t i = 0; i < m; ++i)
        if (idx[i] < 0) return E_INVAL;
    if (p->kind != 1) {
        for (int64_t i = 0; i < m; ++i)
            out[i] = pow(10.0, pdf_invert_analytic(p, agn_oracle_uniform(seed, 1, curve_id, (uint64_t)idx[i])));
        return E_OK;
    }
    /* kind 1 (Eq. 1): CDF from Gauss-Legendre panels, summed in extended precision;
     * the draw is found by search over the panels, then bisection inside one */
    enum { NP = 2048 };
    long double* cum = (long double*)malloc(sizeof(long double) * (NP + 1));
    if (!cum) return E_NOMEM;
    const double w = (p->u_max - p->u_min) / NP;
    cum[0] = 0.0L;
    for (int i = 0; i < NP; ++i) cum[i + 1] = cum[i] + pdf_gl(p, p->u_min + i * w, p->u_min + (i + 1) * w);
    const long double total = cum[NP];
    for (int64_t i = 0; i < m; ++i) {
        const long double target = (long double)agn_oracle_uniform(seed, 1, curve_id, (uint64_t)idx[i]) * total;
        int lo_i = 0, hi_i = NP;  /* cum[lo_i] <= target < cum[hi_i] */
        while (hi_i - lo_i > 1) {
            const int mid = (lo_i + hi_i) / 2;
            if (cum[mid] <= target) lo_i = mid;
            else hi_i = mid;
        }
        const double a = p->u_min + lo_i * w;
        const double rest = (double)(target - cum[lo_i]);
        double lo = a, hi = (lo_i == NP - 1) ? p->u_max : a + w;
        for (int it = 0; it < 200 && hi - lo > 1e-15 * (1.0 + fabs(lo)); ++it) {
            const double mid = 0.5 * (lo + hi);
            if (pdf_gl(p, a, mid) < rest) lo = mid;
            else hi = mid;
        }
        out[i] = pow(10.0, 0.5 * (lo + hi));
    }
    free(cum);
    return E_OK;
}

int agn_oracle_pdf_draw(const agn_oracle_pdf_params* p, int64_t n, uint64_t seed, uint32_t curve_id,
                        double* out)
{
    if (n < 0 || (n > 0 && !out)) return E_INVAL;
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!idx) return E_NOMEM;
    for (int64_t k = 0; k < n; ++k) idx[k] = k;
    const int rc = agn_oracle_pdf_draw_at(p, seed, curve_id, idx, n, out);
    free(idx);
    return rc;
}

/* Periodogram, Eq. A2 (Appendix A): P(f_j) = 2 / N^2 |DFT(f_j)|^2, j = 0..N/2. */
int agn_oracle_periodogram(const double* x, int64_t n, double* P)
{
    if (!x || !P) return E_INVAL;
    if (n < 2 || n % 2 != 0 || !valid_n(n)) return E_SIZE;
    int64_t h = n / 2;
    double* X = (double*)malloc(sizeof(double) * 2 * (size_t)(h + 1));
    if (!X) return E_NOMEM;
    int rc = agn_oracle_rfft(x, n, X);
    if (!rc)
        for (int64_t j = 0; j <= h; ++j)
            P[j] = 2.0 / ((double)n * (double)n) * (X[2 * j] * X[2 * j] + X[2 * j + 1] * X[2 * j + 1]);
    free(X);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Lag statistics of a series (App. A, Eq. A6; Sec. 3.2.10; Sec. 4.2).        */
/* ------------------------------------------------------------------------ */
int agn_oracle_lag_stats(const double* x, int64_t n, const int64_t* lags, int32_t n_lags, int32_t units,
                         const double* dm_ref, int32_t n_thr, double lam_cut, double* sf2_out,
                         uint64_t* exceed_out, uint64_t* pairs_out)
{
    if (!x || n < 2 || !lags || n_lags < 0 || n_thr < 0 || (units != 0 && units != 1)) return E_INVAL;
    if (n_thr > 0 && (!dm_ref || !exceed_out)) return E_INVAL;
    if (n_thr > 64) return E_INVAL;
    for (int32_t j = 0; j < n_thr; ++j)
        if (!(dm_ref[j] >= 0.0) || !isfinite(dm_ref[j])) return E_INVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!(x[i] > 0.0) || !isfinite(x[i])) return E_INVAL;
    for (int32_t l = 0; l < n_lags; ++l)
        if (lags[l] < 1 || lags[l] >= n) return E_INVAL;
    for (int32_t l = 0; l < n_lags; ++l) {
        const int64_t k = lags[l];
        /* Eq. A6: mean over the n - k pairs separated by k samples of the squared
         * difference, of x itself or of the magnitude -2.5 log10 x (Sec. 3.2.10) */
        long double acc = 0.0L;
        for (int64_t i = 0; i + k < n; ++i) {
            const double a = x[i], b = x[i + k];
            const double d = units ? -2.5 * (log10(b) - log10(a)) : b - a;
            acc += (long double)d * d;
        }
        if (sf2_out) sf2_out[l] = (double)(acc / (long double)(n - k));
        /* Fig. 16 / Fig. 17: pairs whose |dm| exceeds each threshold.  A point
         * fainter than the cut is replaced by the cut (an upper limit) and only
         * pairs with at least one point at or above the cut count.  |dm| > D is
         * taken as hi > lo * 10^(D / 2.5), the factor rounded once to double. */
        uint64_t pairs = 0;
        double fac[64];
        for (int32_t j = 0; j < n_thr; ++j) {
            exceed_out[(int64_t)l * n_thr + j] = 0;
            fac[j] = pow(10.0, dm_ref[j] / 2.5);
        }
        for (int64_t i = 0; i + k < n; ++i) {
            double a = x[i], b = x[i + k];
            if (lam_cut > 0.0) {
                if (a < lam_cut && b < lam_cut) continue;
                if (a < lam_cut) a = lam_cut;
                if (b < lam_cut) b = lam_cut;
            }
            ++pairs;
            const double hi = a > b ? a : b, lo = a > b ? b : a;
            for (int32_t j = 0; j < n_thr; ++j)
                if (hi > lo * fac[j]) ++exceed_out[(int64_t)l * n_thr + j];
        }
        if (pairs_out) pairs_out[l] = pairs;
    }
    return E_OK;
}

/* ------------------------------------------------------------------------ */
/* Fit of Eq. 3 to a binned periodogram (the convergence test of Sec. 3.2.2). */
/* ------------------------------------------------------------------------ */
/* Least squares in log10 P over the bins with pbar > 0:
 *   model(f) = a - log10((f / f_br)^a_low + (f / f_br)^a_high),
 * with f_br held at the input value and (a, a_low, a_high) free; Gauss-Newton
 * in extended precision with step halving, from a_low0 / a_high0 and the best
 * a for them, until the step is below 1e-14 of the parameters. */
static long double fit_sse(const double* f, const double* pbar, int64_t nb, double f_br, const long double th[3])
{
    long double sse = 0.0L;
    for (int64_t b = 0; b < nb; ++b) {
        if (!(pbar[b] > 0.0)) continue;
        const long double lu = logl((long double)f[b] / (long double)f_br);
        const long double m = th[0] - log10l(expl(th[1] * lu) + expl(th[2] * lu));
        const long double r = log10l((long double)pbar[b]) - m;
        sse += r * r;
    }
    return sse;
}

int agn_oracle_psd_fit(const double* f, const double* pbar, int64_t nb, double f_br, double a_low0, double a_high0,
                       double out[4])
{
    if (!f || !pbar || !out || nb < 0 || !(f_br > 0.0)) return E_INVAL;
    int64_t used = 0, below = 0, above = 0;
    for (int64_t b = 0; b < nb; ++b) {
        if (!(pbar[b] > 0.0)) continue;
        if (!(f[b] > 0.0)) return E_INVAL;
        ++used;
        below += f[b] < f_br;
        above += f[b] > f_br;
    }
    if (used < 3 || below < 1 || above < 1) return E_INVAL;
    long double th[3] = {0.0L, a_low0, a_high0};
    {
        long double s = 0.0L;
        for (int64_t b = 0; b < nb; ++b) {
            if (!(pbar[b] > 0.0)) continue;
            const long double lu = logl((long double)f[b] / (long double)f_br);
            s += log10l((long double)pbar[b]) + log10l(expl(th[1] * lu) + expl(th[2] * lu));
        }
        th[0] = s / used;
    }
    long double sse = fit_sse(f, pbar, nb, f_br, th);
    for (int it = 0; it < 500; ++it) {
        long double A[3][3] = {{0}}, g[3] = {0};
        for (int64_t b = 0; b < nb; ++b) {
            if (!(pbar[b] > 0.0)) continue;
            const long double lu = logl((long double)f[b] / (long double)f_br), L = lu / logl(10.0L);
            const long double tl = expl(th[1] * lu), thh = expl(th[2] * lu), S = tl + thh;
            const long double r = log10l((long double)pbar[b]) - (th[0] - log10l(S));
            const long double J[3] = {1.0L, -tl / S * L, -thh / S * L};  /* d model / d theta */
            for (int i = 0; i < 3; ++i) {
                g[i] += J[i] * r;
                for (int k = 0; k < 3; ++k) A[i][k] += J[i] * J[k];
            }
        }
        /* minimum-norm solution of A d = g: A = V diag(w) V^T by Jacobi
         * rotations, directions with w below 1e-15 of the largest dropped (with
         * equal slopes the two slope columns of the Jacobian coincide) */
        long double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int sweep = 0; sweep < 60; ++sweep) {
            long double off = 0.0L;
            for (int p = 0; p < 3; ++p)
                for (int q = p + 1; q < 3; ++q) off += A[p][q] * A[p][q];
            if (off < 1e-60L) break;
            for (int p = 0; p < 3; ++p)
                for (int q = p + 1; q < 3; ++q) {
                    if (A[p][q] == 0.0L) continue;
                    const long double tau = (A[q][q] - A[p][p]) / (2.0L * A[p][q]);
                    const long double t = (tau >= 0.0L ? 1.0L : -1.0L) / (fabsl(tau) + sqrtl(1.0L + tau * tau));
                    const long double c = 1.0L / sqrtl(1.0L + t * t), sn = t * c;
                    for (int k = 0; k < 3; ++k) {  /* A <- A J */
                        const long double akp = A[k][p], akq = A[k][q];
                        A[k][p] = c * akp - sn * akq;
                        A[k][q] = sn * akp + c * akq;
                    }
                    for (int k = 0; k < 3; ++k) {  /* A <- J^T A */
                        const long double apk = A[p][k], aqk = A[q][k];
                        A[p][k] = c * apk - sn * aqk;
                        A[q][k] = sn * apk + c * aqk;
                    }
                    for (int k = 0; k < 3; ++k) {  /* V <- V J */
                        const long double vkp = V[k][p], vkq = V[k][q];
                        V[k][p] = c * vkp - sn * vkq;
                        V[k][q] = sn * vkp + c * vkq;
                    }
                }
        }
        long double wmax = 0.0L;
        for (int i = 0; i < 3; ++i)
            if (A[i][i] > wmax) wmax = A[i][i];
        if (!(wmax > 0.0L)) return E_INVAL;
        long double d[3] = {0.0L, 0.0L, 0.0L};
        for (int i = 0; i < 3; ++i) {
            if (!(A[i][i] > 1e-15L * wmax)) continue;
            long double vg = 0.0L;
            for (int k = 0; k < 3; ++k) vg += V[k][i] * g[k];
            for (int k = 0; k < 3; ++k) d[k] += V[k][i] * vg / A[i][i];
        }
        long double step = 1.0L, nt[3], nsse = 0.0L;
        for (int h = 0; h < 60; ++h) {
            for (int i = 0; i < 3; ++i) nt[i] = th[i] + step * d[i];
            nsse = fit_sse(f, pbar, nb, f_br, nt);
            if (nsse <= sse) break;
            step *= 0.5L;
        }
        if (!(nsse <= sse)) break;  /* no descent left: at the minimum to working precision */
        long double mx = 0.0L;
        for (int i = 0; i < 3; ++i) {
            const long double rel = fabsl(nt[i] - th[i]) / (1.0L + fabsl(th[i]));
            if (rel > mx) mx = rel;
            th[i] = nt[i];
        }
        sse = nsse;
        if (mx < 1e-14L) break;
    }
    /* Eq. 3 is symmetric in its two slopes; the smaller one is the
     * low-frequency slope */
    out[0] = (double)th[0];
    out[1] = (double)(th[1] < th[2] ? th[1] : th[2]);
    out[2] = (double)(th[1] < th[2] ? th[2] : th[1]);
    out[3] = (double)sqrtl(sse / used);
    return E_OK;
}

/* ------------------------------------------------------------------------ */
/* Slice sampling of the PDF in linear lambda (Sec. 3.1; Neal 2003).          */
/* ------------------------------------------------------------------------ */
/* Uniform #k of chain `chain`: counter (k / 4, chain, 0, 0), word k % 4. */
double agn_oracle_uniform_chain(uint64_t seed, uint32_t stream, uint32_t curve_id, uint64_t chain, uint64_t k)
{
    uint64_t key[2] = {seed, ((uint64_t)stream << 32) | (uint64_t)curve_id};
    uint64_t ctr[4] = {k / 4, chain, 0, 0};
    uint64_t out[4];
    agn_oracle_philox4x64(ctr, key, out);
    return ((double)(out[k % 4] >> 12) + 0.5) * 0x1.0p-52;
}

/* ln of the density of lambda (per unit lambda), up to a constant. */
static double slice_log_density(const agn_oracle_pdf_params* p, double lam)
{
    const double u = log10(lam), x = u - p->u_star;
    double l10;  /* log10 of the shape in u */
    if (p->kind == 0) l10 = -(x < 0.0 ? p->d1 : p->d2) * x;
    else if (p->kind == 1) l10 = -log10(pow(10.0, p->d1 * x) + pow(10.0, p->d2 * x));
    else l10 = -x * x / (2.0 * p->sigma * p->sigma) / LN10;
    /* per dex (measure 0) -> per unit lambda: divide by lambda ln 10 */
    if (p->measure == 0) l10 -= u;
    return l10 * LN10;
}

int agn_oracle_pdf_slice(const agn_oracle_pdf_params* p, int64_t n, int32_t n_chains, int32_t burn,
                         uint64_t seed, uint32_t curve_id, double* out)
{
    if (!p || n < 0 || (n > 0 && !out) || n_chains < 1 || burn < 0) return E_INVAL;
    if (!(p->u_min < p->u_max) || !isfinite(p->u_min) || !isfinite(p->u_max) || !isfinite(p->u_star))
        return E_INVAL;
    if (p->kind < 0 || p->kind > 2 || (p->measure != 0 && p->measure != 1)) return E_INVAL;
    if (p->kind != 2 && (!isfinite(p->d1) || !isfinite(p->d2))) return E_INVAL;
    if (p->kind == 2 && !(p->sigma > 0.0 && isfinite(p->sigma))) return E_INVAL;
    const double lo = pow(10.0, p->u_min), hi = pow(10.0, p->u_max);
    double start = pow(10.0, p->u_star);
    if (!(start > lo && start < hi)) start = 0.5 * (lo + hi);
    for (int64_t c = 0; c < n_chains && c < (n > 0 ? n : 0); ++c) {
        double lam = start, lf = slice_log_density(p, lam);
        uint64_t k = 0;
        for (int64_t step = 0; ; ++step) {
            const int64_t j = (step - burn) * (int64_t)n_chains + c;  /* output slot */
            if (step >= burn && j >= n) break;
            /* the slice: ln f > ln f(lam) + ln U; then shrink [lo, hi] toward lam */
            const double level = lf + log(agn_oracle_uniform_chain(seed, 6, curve_id, (uint64_t)c, k++));
            double L = lo, R = hi, next = lam, lnext = lf;
            for (int t = 0; t < 200; ++t) {
                const double cand = L + agn_oracle_uniform_chain(seed, 6, curve_id, (uint64_t)c, k++) * (R - L);
                const double lc = slice_log_density(p, cand);
                if (lc > level) { next = cand; lnext = lc; break; }
                if (cand < lam) L = cand;
                else R = cand;
            }
            lam = next;
            lf = lnext;
            if (step >= burn) out[j] = lam;
        }
    }
    return E_OK;
}
