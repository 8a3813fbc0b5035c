/*
 * agn_oracle.h -- plain FP64 CPU oracle for the Emmanoulopoulos-style
 * light-curve iteration of Sartori et al. (2019), arXiv:1909.06374.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * statement of what the GPU path computes.  It shares no code, header,
 * table or constant generator with the HIP library.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * Everything is host memory, double precision, single threaded.
 * Every function returns 0 on success and a negative code on bad input.
 */
#ifndef AGN_ORACLE_H
#define AGN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Eq. 3 parameters.  norm <= 0 selects the unit-variance normalisation. */
typedef struct {
    double norm;
    double f_br;
    double a_low;
    double a_high;
} agn_oracle_psd_params;

/* Philox4x64-10 block function (Salmon et al., SC'11). */
void agn_oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Uniform number #k of stream `stream` for (seed, curve_id); value in (0, 1). */
double agn_oracle_uniform(uint64_t seed, uint32_t stream, uint32_t curve_id, uint64_t k);

/* Eq. 3 at frequency f with the given amplitude A. */
double agn_oracle_psd_eq3(double f, double A, double f_br, double a_low, double a_high);

/* Amplitude A actually used for a length-n grid (norm, or the unit-variance value). */
double agn_oracle_psd_norm(const agn_oracle_psd_params* p, int64_t n, double dt);

/* Timmer-Koenig Fourier moduli, amp[0..n/2]. */
int agn_oracle_psd_spectrum(const agn_oracle_psd_params* p, int64_t n, double dt,
                            uint64_t seed, uint32_t curve_id, double* amp);

/* Complex DFT of length n (n = 2^a 3^b), unnormalised.  sign = -1 forward, +1 inverse.
 * data is interleaved (re, im), in place. */
int agn_oracle_dft(double* data, int64_t n, int sign);

/* Real forward DFT: x[n] -> X[n/2+1] interleaved complex. */
int agn_oracle_rfft(const double* x, int64_t n, double* X);

/* Unnormalised inverse real DFT of a Hermitian half spectrum: Y[n/2+1] -> y[n]. */
int agn_oracle_irfft(const double* Y, int64_t n, double* y);

/* Fourier amplitude replacement keeping phases (in: X, amp; out: Y; may alias X). */
int agn_oracle_replace(const double* X, const double* amp, int64_t n, double* Y);

/* Stable ascending argsort of y (ties by index; -0 equals +0).  perm[k] = index of
 * the k-th smallest. */
int agn_oracle_argsort(const double* y, int64_t n, uint32_t* perm);

/* Iterate from x0 (the PDF draw, in draw order) with target moduli amp.
 * x_out[n]: final series; delta_out[iters] (nullable); iters_done (nullable);
 * rank_out[n] (nullable): rank of each time sample in the sorted draw. */
int agn_oracle_iterate(const double* amp, const double* x0, int64_t n, int32_t iters,
                       double tol, double* x_out, double* delta_out, int32_t* iters_done,
                       uint32_t* rank_out);

/* Spectrum + iterate. */
int agn_oracle_generate(const agn_oracle_psd_params* p, const double* erdf, int64_t n,
                        double dt, int32_t iters, double tol, uint64_t seed,
                        uint32_t curve_id, double* x_out, double* delta_out,
                        int32_t* iters_done, uint32_t* rank_out);

/* PDF draw (Sec. 2.1 step ii) from a sharp broken power law in dN/dlog10(lambda)
 * with Eq. 1's slope convention: density 10^(-d1 (u - u_br)) below the break and
 * 10^(-d2 (u - u_br)) above it, u = log10(lambda) in [u_min, u_max].  Inverse CDF
 * of uniform #k of Philox stream 1 (key (seed, 1 << 32 | curve_id)); out[k] = 10^u. */
typedef struct {
    double u_min;
    double u_max;
    double u_br;
    double d1;
    double d2;
} agn_oracle_erdf_params;

int agn_oracle_erdf_bpl(const agn_oracle_erdf_params* p, int64_t n, uint64_t seed,
                        uint32_t curve_id, double* out);

/* General PDF draw (Sec. 2.1 step ii), u = log10(lambda) in [u_min, u_max]:
 *   kind 0: sharp broken power law, shape 10^(-d1 (u - u_star)) below u_star and
 *           10^(-d2 (u - u_star)) above;
 *   kind 1: Eq. 1, shape 1 / ((lambda/lambda*)^d1 + (lambda/lambda*)^d2);
 *   kind 2: Eq. 2, shape exp(-(u - u_star)^2 / (2 sigma^2)).
 * measure 0: the shape is dN/dlog10(lambda); measure 1: the shape is dN/dlambda
 * (the density in u then carries an extra factor lambda).  Draw k is the exact
 * inverse CDF (closed form, or bisection on the CDF computed by quadrature) of
 * uniform #k of Philox stream 1; out[k] = 10^u. */
typedef struct {
    int32_t kind;
    int32_t measure;
    double u_min;
    double u_max;
    double u_star;
    double d1;
    double d2;
    double sigma;
} agn_oracle_pdf_params;

int agn_oracle_pdf_draw(const agn_oracle_pdf_params* p, int64_t n, uint64_t seed, uint32_t curve_id,
                        double* out);
/* The same draws at the m indices idx[0..m-1] only (out[i] is draw #idx[i]). */
int agn_oracle_pdf_draw_at(const agn_oracle_pdf_params* p, uint64_t seed, uint32_t curve_id,
                           const int64_t* idx, int64_t m, double* out);

/* Uniform #k of chain `chain` of a stream: Philox counter (k / 4, chain, 0, 0). */
double agn_oracle_uniform_chain(uint64_t seed, uint32_t stream, uint32_t curve_id, uint64_t chain, uint64_t k);

/* Slice sampling (Sec. 3.1; Neal 2003) of the PDF above in linear lambda on
 * [10^u_min, 10^u_max], target density per unit lambda (measure 0: the shape
 * per dex divided by lambda; measure 1: the shape itself).  n_chains chains
 * start at lambda* (the middle of the support if lambda* lies outside); each
 * step draws a level ln f(lambda) + ln U, then proposals uniform on the
 * support interval, shrunk toward the current point after each rejection (at
 * most 200; the point is kept if none is accepted).  Chain c takes uniforms
 * #0, 1, ... of Philox stream 6, counter (k / 4, c, 0, 0); after `burn`
 * steps, its step t fills out[t * n_chains + c]. */
int agn_oracle_pdf_slice(const agn_oracle_pdf_params* p, int64_t n, int32_t n_chains, int32_t burn,
                         uint64_t seed, uint32_t curve_id, double* out);

/* Periodogram, Eq. A2: P[j] = 2/n^2 |DFT_j|^2 for j = 0..n/2. */
int agn_oracle_periodogram(const double* x, int64_t n, double* P);

/* Lag statistics of one positive series x[n] at lags[n_lags] (1 <= lag < n):
 *   sf2_out[l] (nullable): Eq. A6, the mean over the n - lag pairs of the squared
 *     difference of x (units 0) or of the magnitude -2.5 log10 x (units 1);
 *   exceed_out[l * n_thr + j]: pairs with |dm| > dm_ref[j] (Fig. 16), taken as
 *     hi > lo * 10^(dm_ref[j] / 2.5); with lam_cut > 0 values below lam_cut are
 *     replaced by it and only pairs with a value >= lam_cut count (Fig. 17);
 *   pairs_out[l] (nullable): the pairs counted.  At most 64 thresholds. */
int agn_oracle_lag_stats(const double* x, int64_t n, const int64_t* lags, int32_t n_lags, int32_t units,
                         const double* dm_ref, int32_t n_thr, double lam_cut, double* sf2_out,
                         uint64_t* exceed_out, uint64_t* pairs_out);

/* Fit of Eq. 3 to a binned periodogram (f[b], pbar[b], bins with pbar <= 0
 * skipped): least squares in log10 P with the break held at f_br, free
 * (a = log10 A, a_low, a_high), started from a_low0 / a_high0.  Needs >= 3 used
 * bins with at least one below and one above f_br.  out = {a, a_low, a_high,
 * rms of the log10 residuals}; the model is symmetric in the two slopes, and
 * a_low is reported as the smaller. */
int agn_oracle_psd_fit(const double* f, const double* pbar, int64_t nb, double f_br, double a_low0, double a_high0,
                       double out[4]);

#ifdef __cplusplus
}
#endif
#endif
