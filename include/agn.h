/*
 * agn.h -- C ABI of the MI355X (gfx950) light-curve generator.
 *
 * The library generates light curves with a prescribed power spectral density
 * (Eq. 3 of Sartori et al. 2019, arXiv:1909.06374) and a prescribed
 * distribution of values (a sample of the Eddington-ratio distribution, the
 * PDF draw of Sec. 2.1), using the Emmanoulopoulos et al. (2013) iteration
 * that the paper adopts (Sec. 2.1, Sec. 3.1, Sec. 3.2.2):
 *
 *   1. draw a Timmer & Koenig (1995) random spectrum for the PSD; only its
 *      Fourier moduli are kept (agn_psd_spectrum);
 *   2. start from the PDF draw in draw order;
 *   3. repeat: forward real FFT, replace the Fourier moduli by the target
 *      moduli keeping the phases, inverse real FFT, rank the result, and put
 *      the sorted PDF draw into that rank order (agn_lc_iterate);
 *   4. record the convergence distance of Eq. 4 after every iteration.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Device pointers are HIP device memory owned by the caller (for example
 *    torch tensors' data_ptr()).  The library never frees or retains them
 *    after the enqueued work completes.  Host pointers are read before the
 *    call returns.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *    call is stream ordered and returns without synchronising the host;
 *    outputs are valid once the stream has completed the work.
 *  - `ws` is a caller-owned device workspace of at least the size reported
 *    by the matching *_workspace_size call; its contents on entry do not
 *    matter.  Calls that overlap in time must not share a workspace.
 *  - Return value: AGN_OK or a negative agn_status.  All argument checks
 *    happen on the host before anything is enqueued; on error nothing is
 *    enqueued and agn_last_error() describes the problem.
 *  - Supported lengths: n even, n = 2^a or 3 * 2^a, 2 <= n <= 2^27.
 *  - PDF draw values must be finite and > 0 (Eq. 4 takes logarithms).  This
 *    is checked on the device: an invalid draw sets *iters_done = -1 and the
 *    outputs of that curve are unspecified.
 *  - Determinism: identical inputs give bit-identical outputs; the kernels
 *    chosen depend only on (n, precision), never on batch composition.
 *
 * Precision
 * ---------
 *  AGN_FP64: every step in double precision (the plain method).
 *  AGN_FP32: FFTs, moduli and sort keys in single precision, twiddle tables
 *            generated in double and rounded once, convergence sums in
 *            double.  The output values are always the caller's double
 *            precision PDF draw, only reordered.
 */
#ifndef AGN_H
#define AGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct agn_ctx agn_ctx;

/* PSD parameters of Eq. 3: PSD(f) = norm / ((f/f_br)^a_low + (f/f_br)^a_high).
 * f and f_br are in cycles per unit of dt.  norm <= 0 selects the value of
 * norm that gives the Timmer-Koenig series unit expected variance:
 * norm = N^2 / (2 sum_{j=1}^{N/2-1} P~_j + P~_{N/2} / 2), P~ = Eq. 3 with norm 1.
 * The normalisation does not change the output ordering, only the moduli. */
typedef struct {
    double norm;
    double f_br;
    double a_low;
    double a_high;
} agn_psd_params;

typedef enum { AGN_FP64 = 0, AGN_FP32 = 1 } agn_precision;

typedef enum {
    AGN_OK = 0,
    AGN_EINVAL = -1,          /* bad pointer, parameter or workspace size */
    AGN_EUNSUPPORTED_N = -2,  /* n not of the supported form */
    AGN_ENOMEM = -3,          /* library-owned table allocation failed */
    AGN_EDEVICE = -4          /* HIP runtime error */
} agn_status;

/* Context: holds per-(n, precision) twiddle tables on one device.
 * Created once; the tables are allocated on the first call that needs them. */
int agn_ctx_create(int device, agn_ctx** out);
int agn_ctx_destroy(agn_ctx* ctx);

/* Thread-local description of the last error (never NULL). */
const char* agn_last_error(void);

/* 1 if n is a supported length, else 0. */
int agn_supported_n(int64_t n);

/* Bytes of workspace for agn_psd_spectrum on one curve of length n. */
int agn_spectrum_workspace_size(int64_t n, size_t* bytes);

/* Bytes of workspace for agn_lc_iterate / agn_lc_generate on one curve. */
int agn_workspace_size(int64_t n, agn_precision prec, size_t* bytes);

/* Bytes of workspace for agn_lc_generate_batch; n is a host array. */
int agn_batch_workspace_size(int32_t n_curves, const int64_t* n, agn_precision prec,
                             size_t* bytes);

/*
 * agn_psd_spectrum -- Timmer-Koenig Fourier moduli (Sec. 2.1 step i; Eq. 3 on
 * the Fourier grid f_j = j / (n dt) of Appendix A).
 *   amp_out[0]       = 0 (the DC bin; the series has zero mean)
 *   amp_out[j]       = sqrt(PSD(f_j) * E_j),  E_j = -ln U_j,   0 < j < n/2
 *   amp_out[n/2]     = sqrt(PSD(f_{n/2}) / 2) * |g|,  g = sqrt(-2 ln U_a) cos(2 pi U_b)
 * E_j is the squared modulus of a complex Gaussian with variance PSD/2 per
 * component, divided by PSD; only the moduli matter to the iteration.
 * Random numbers: Philox4x64-10 with key (seed, 0 << 32 | curve_id),
 * counter (k / 4, 0, 0, 0); uniform #k = word k % 4 mapped to
 * ((w >> 12) + 1/2) 2^-52.  Bin j uses uniform #j; the Nyquist bin uses
 * #(n/2) and #(n/2 + 1).
 *   p        host, PSD parameters.
 *   amp_out  device, n/2 + 1 values of float (AGN_FP32) or double (AGN_FP64).
 *   ws       device workspace of agn_spectrum_workspace_size(n) bytes.
 */
int agn_psd_spectrum(agn_ctx* ctx, const agn_psd_params* p, int64_t n, double dt,
                     uint64_t seed, uint32_t curve_id, agn_precision prec,
                     void* amp_out, void* ws, size_t ws_bytes, void* stream);

/*
 * agn_psd_spectrum_noalloc -- agn_psd_spectrum for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and bit-identical
 * moduli, but the workspace is a library-owned device array of 512 KiB
 * (enough for every supported n; each device holds its own copy until the
 * process ends) instead of a caller's ws, and the descriptor is written by a
 * kernel instead of through a pinned staging buffer.  The call allocates
 * nothing, host or device, and records no kernel timing.
 *   Arguments, layout and errors as agn_psd_spectrum (no ws); AGN_EDEVICE if
 *   the array's device address could not be resolved when ctx was created.
 *   All calls on one device share the array: calls that overlap in time on
 *   one device (different streams, or different contexts) race and give
 *   undefined moduli; serialise them.  Nothing in the array needs to start
 *   at zero: each call writes what it reads.
 */
int agn_psd_spectrum_noalloc(agn_ctx* ctx, const agn_psd_params* p, int64_t n, double dt,
                             uint64_t seed, uint32_t curve_id, agn_precision prec,
                             void* amp_out, void* stream);

/*
 * agn_lc_iterate -- the iteration of Sec. 2.1 / Sec. 3.2.2 from a given start.
 *   amp        device, n/2 + 1 target moduli (float for AGN_FP32, double for
 *              AGN_FP64), as produced by agn_psd_spectrum.
 *   x0         device, n doubles: the PDF draw in draw order (it is also the
 *              starting series x_0).  s = x0 sorted ascending is the fixed set
 *              of values; every output is a permutation of it.
 *   iters      number of iterations (>= 0).
 *   tol        < 0: run exactly `iters` iterations.  >= 0: stop after the first
 *              iteration i with x_i == x_{i-1} (an exact fixed point), or, if
 *              tol > 0, with delta_i <= tol.
 *   x_out      device, n doubles: x_iters_done.
 *   delta_out  device, `iters` doubles or NULL: delta_i of Eq. 4,
 *              sqrt(mean_n (log10 x_i[n] - log10 x_{i-1}[n])^2); entries past
 *              iters_done are 0.
 *   iters_done device, one int32 or NULL: iterations performed, -1 if x0 holds
 *              a value that is not finite and > 0, -2 if a multi-pass sort
 *              step gave up waiting for another workgroup (a device fault
 *              that should not occur; x_out is then not valid).
 *   rank_out   device, n uint32 or NULL: rank_out[t] = index into s of x_out[t].
 * Each iteration: X = rFFT(x_{i-1}); Y_j = amp_j X_j / |X_j| (Y_0 = 0,
 * Y_{n/2} = amp_{n/2} sign(Re X_{n/2}) with sign(0) = +1, phase 0 where
 * |X_j| = 0); y = unnormalised inverse rFFT(Y); perm = stable ascending
 * argsort of y (ties by index, -0 == +0); x_i[perm[k]] = s[k].
 */
int agn_lc_iterate(agn_ctx* ctx, const void* amp, const double* x0, int64_t n, int32_t iters,
                   double tol, agn_precision prec, double* x_out, double* delta_out,
                   int32_t* iters_done, uint32_t* rank_out, void* ws, size_t ws_bytes,
                   void* stream);

/*
 * agn_lc_generate -- agn_psd_spectrum followed by agn_lc_iterate for one curve
 * (the whole method of Sec. 2.1 for a given PDF draw).  Arguments as above;
 * erdf is the PDF draw (device, n doubles, draw order).
 */
int agn_lc_generate(agn_ctx* ctx, const agn_psd_params* p, const double* erdf, int64_t n,
                    double dt, int32_t iters, double tol, uint64_t seed, uint32_t curve_id,
                    agn_precision prec, double* x_out, double* delta_out, int32_t* iters_done,
                    void* ws, size_t ws_bytes, void* stream);

/*
 * agn_lc_generate_batch -- agn_lc_generate for n_curves independent curves of
 * possibly different lengths in one call.  Per-curve arrays are HOST arrays
 * of n_curves entries: n, offset (element offset of the curve in erdf and
 * x_out), p, dt, iters, seed, curve_id.  erdf and x_out are device arrays
 * holding all curves at their offsets (curves must not overlap).  delta_out
 * (device, nullable) holds max(iters) doubles per curve, curve c at
 * c * max(iters); iters_done (device, nullable) one int32 per curve.
 * Results are bit-identical to n_curves separate agn_lc_generate calls.
 */
int agn_lc_generate_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n,
                          const int64_t* offset, const agn_psd_params* p, const double* dt,
                          const int32_t* iters, const uint64_t* seed, const uint32_t* curve_id,
                          const double* erdf, double tol, agn_precision prec, double* x_out,
                          double* delta_out, int32_t* iters_done, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * Batch plans -- agn_lc_generate_batch split into a set-up call and a launch
 * call, for callers that run the same batch layout (same lengths, same device
 * buffers) many times.  The method is the same as agn_lc_generate_batch (Sec.
 * 2.1, Eq. 3-4): results of every launch are bit-identical to it.
 *
 * agn_batch_plan_create takes the arguments of agn_lc_generate_batch (same
 * meaning, layout and ownership; the host arrays are read during the call
 * only; the device buffers erdf, x_out, delta_out, iters_done and ws must
 * stay allocated, and are read or written by every launch, until the plan is
 * destroyed) plus:
 *   flags      AGN_PLAN_GRAPH: the first launch captures the plan's kernels
 *              into a HIP graph on a private stream; every launch replays it
 *              with hipGraphLaunch (no per-kernel host work).
 *              AGN_PLAN_AUTOTUNE: choose the number of concurrent launch
 *              chains (1, 2 or 4; the lengths are dealt to chains longest
 *              first) and, in the FP32 form, the tile of the multi-pass
 *              radix sort (8192 or 16384 keys, the latter for lengths it
 *              divides), by timing each pair on the batch cut to two
 *              iterations per curve; the choice is cached in ctx per batch
 *              layout.  This synchronises `stream` and runs kernels that
 *              write x_out.  Neither choice changes any arithmetic: chains
 *              only reorder independent curves, and the sort is exact.
 *              AGN_PLAN_LARGE_SORT_TILE: use the 16384-key sort tile
 *              for every length it divides, without tuning (not with
 *              AGN_PLAN_AUTOTUNE).  Without either flag the tile is chosen
 *              by length: 16384 keys for FP32 multi-pass curves of at least
 *              2^20 samples that it divides, 8192 otherwise.
 *              AGN_PLAN_NARROW_FFT: 16 butterflies per multi-pass FFT
 *              workgroup instead of up to 64, without tuning.  With
 *              AGN_PLAN_AUTOTUNE this width (64, 32 or 16) is also tuned,
 *              after the chains and the sort tile.  The width changes no
 *              arithmetic: results are bit-identical for every width.  The FFT
 *              decomposition is fixed per length, because it sets the
 *              rounding of the transforms.
 *   branches   chain count when AGN_PLAN_AUTOTUNE is not set (0 or 1: one
 *              chain; at most 8).  Chains run on plan-owned streams of
 *              default priority that fork from and join back into the
 *              launch stream.
 *   out        receives the plan (destroy with agn_batch_plan_destroy).
 * The descriptors are uploaded into ws on `stream` during create.
 * agn_batch_plan_launch enqueues one complete run of the batch on `stream`;
 * launches of one plan must not overlap in time (they share ws).
 */
typedef struct agn_batch_plan agn_batch_plan;
enum { AGN_PLAN_GRAPH = 1, AGN_PLAN_AUTOTUNE = 2, AGN_PLAN_LARGE_SORT_TILE = 4, AGN_PLAN_NARROW_FFT = 8 };

int agn_batch_plan_create(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const int64_t* offset,
                          const agn_psd_params* p, const double* dt, const int32_t* iters,
                          const uint64_t* seed, const uint32_t* curve_id, const double* erdf, double tol,
                          agn_precision prec, double* x_out, double* delta_out, int32_t* iters_done,
                          int flags, int branches, void* ws, size_t ws_bytes, void* stream,
                          agn_batch_plan** out);
int agn_batch_plan_launch(agn_batch_plan* plan, void* stream);
/* Chain count in use, number of launch groups, 1 if graph mode.  A launch
 * group is one length on one path, except that when two or more LDS-resident
 * lengths run whole waves per curve they share one persistent pack launch,
 * which counts once. */
int agn_batch_plan_info(const agn_batch_plan* plan, int32_t* branches, int32_t* groups, int32_t* uses_graph);
/* The tuned (or requested) choices: chain count, sort tile (8192 or 16384;
 * 16384 applies to FP32 multi-pass curves whose length it divides; 0: chosen
 * by length, as described for AGN_PLAN_LARGE_SORT_TILE) and the most
 * butterflies per multi-pass FFT workgroup (64, 32 or 16).  Any output
 * pointer may be NULL. */
int agn_batch_plan_tuning(const agn_batch_plan* plan, int32_t* branches, int32_t* sort_tile,
                          int32_t* fft_cols);
int agn_batch_plan_destroy(agn_batch_plan* plan);

/* Parameters of the PDF draw: a sharp broken power law in dN/dlog10(lambda)
 * with the slope convention of Eq. 1 -- density 10^(-d1 (u - u_br)) below the
 * break and 10^(-d2 (u - u_br)) above it, u = log10(lambda) in [u_min, u_max].
 * Requires u_min < u_br < u_max and d1, d2 != 0. */
typedef struct {
    double u_min;
    double u_max;
    double u_br;
    double d1;
    double d2;
} agn_erdf_params;

/*
 * agn_erdf_draw -- the PDF draw of Sec. 2.1 step (ii): n i.i.d. values of
 * L/L_Edd, lambda = 10^u, by the closed-form inverse CDF of the broken power
 * law applied to uniform #k of Philox stream 1 (key (seed, 1 << 32 |
 * curve_id), same counter layout and uniform mapping as agn_psd_spectrum).
 *   p    host parameters; out: device, n doubles, in draw order.
 */
int agn_erdf_draw(agn_ctx* ctx, const agn_erdf_params* p, int64_t n, uint64_t seed,
                  uint32_t curve_id, double* out, void* stream);

/* General PDF of the draw (Sec. 2.1 step (ii), shapes of Sec. 2.1.1), in
 * u = log10(lambda) on [u_min, u_max], x = u - u_star:
 *   AGN_PDF_SHARP_BPL  10^(-d1 x) for x < 0, 10^(-d2 x) for x >= 0 (needs
 *                      u_min < u_star < u_max);
 *   AGN_PDF_EQ1        Eq. 1: 1 / (10^(d1 x) + 10^(d2 x));
 *   AGN_PDF_LOGNORMAL  Eq. 2: exp(-x^2 / (2 sigma^2)) (needs sigma > 0).
 * measure AGN_PDF_PER_LOG reads the shape as dN/dlog10(lambda); measure
 * AGN_PDF_PER_LINEAR reads it as dN/dlambda (the paper samples in linear
 * lambda), so that the density in u carries an extra factor 10^x.  Slopes are
 * limited so that the shape spans under 10^260 over the support, and for
 * Eq. 1 so that (u_max - u_min) |d2 - d1| ln 10 <= 512 (the break spans at
 * least two cells of the 1024-cell CDF table). */
enum { AGN_PDF_SHARP_BPL = 0, AGN_PDF_EQ1 = 1, AGN_PDF_LOGNORMAL = 2 };
enum { AGN_PDF_PER_LOG = 0, AGN_PDF_PER_LINEAR = 1 };
typedef struct {
    int32_t kind;
    int32_t measure;
    double u_min;
    double u_max;
    double u_star;
    double d1;      /* slopes (kinds 0 and 1) */
    double d2;
    double sigma;   /* dex (kind 2) */
} agn_pdf_params;

/*
 * agn_pdf_draw -- n i.i.d. draws lambda = 10^u of the PDF above, draw k the
 * inverse CDF of uniform #k of Philox stream 1 (key (seed, 1 << 32 |
 * curve_id); same stream as agn_erdf_draw, which equals kind 0, measure 0).
 * Kind 0 inverts in closed form, kind 2 with erfcinv, kind 1 on a CDF table
 * that each block builds in LDS followed by Newton steps on the exact integral.
 *   p    host parameters; out: device, n doubles, in draw order.
 * Errors: AGN_EINVAL for NULL pointers, n < 0 or parameters outside the ranges
 * above (nothing is launched).  Stream-ordered; no allocation.
 */
int agn_pdf_draw(agn_ctx* ctx, const agn_pdf_params* p, int64_t n, uint64_t seed, uint32_t curve_id,
                 double* out, void* stream);

/*
 * agn_pdf_slice -- the PDF draw as the paper makes it (Sec. 3.1): slice
 * sampling (Neal 2003) in linear lambda of the PDF above, with n_chains
 * independent chains.  Target density per unit lambda: the shape per dex
 * divided by lambda (AGN_PDF_PER_LOG) or the shape itself (AGN_PDF_PER_LINEAR).
 * Each chain starts at lambda* (the middle of the support if lambda* lies
 * outside it); a step draws the level ln f(lambda) + ln U, then proposals
 * uniform on [10^u_min, 10^u_max] shrunk toward the current point after each
 * rejection (at most 200; the point is kept if none is accepted).  Chain c
 * draws uniforms 0, 1, ... of Philox stream 6 with counter (k / 4, c, 0, 0)
 * (key (seed, 6 << 32 | curve_id)); after `burn` steps its step t fills
 * out[t * n_chains + c].  Successive steps of one chain are correlated (over
 * several decades the lag-one correlation is 0.6-0.8); n_chains = n gives
 * one draw per chain.
 *   p: host; out: device, n doubles.  n_chains >= 1, 0 <= burn <= 2^24.
 * Errors: AGN_EINVAL (nothing launched).  Stream-ordered; no allocation.
 */
int agn_pdf_slice(agn_ctx* ctx, const agn_pdf_params* p, int64_t n, int32_t n_chains, int32_t burn, uint64_t seed,
                  uint32_t curve_id, double* out, void* stream);

/*
 * Observables after the path (App. A).
 *
 * agn_periodogram_batch -- the periodogram of Eq. A2 of n_curves real series
 * (for example the generator's output), in double precision:
 *   P_c[j] = 2 / N^2 |sum_t x_c[t] exp(-2 pi i j t / N)|^2,  j = 0 .. N/2,
 * and, if bins_out is not NULL, its arithmetic means over logarithmic
 * frequency bins: j >= 1 falls in bin floor(log10(j) / dex + 1e-9) (bins of
 * `dex` in log10 frequency starting at the first Fourier frequency); empty
 * bins are dropped and the others are written in increasing frequency.
 *   n, offset  host, n_curves entries: length (2^a or 3*2^a, >= 4) and EVEN
 *              element offset of each curve in x (device)
 *   p_offset   host: element offset of curve c's N/2+1 values in P_out (device)
 *   b_offset   host (with bins_out): offset of curve c's bins in bins_out
 *              (device); agn_log_bin_count gives their number
 *   ws         device workspace of agn_periodogram_workspace_size bytes
 *              (the same dex, or dex <= 0 without bins)
 * Errors: AGN_EINVAL (NULL, negative or odd offset, bad dex, small
 * workspace), AGN_EUNSUPPORTED_N.  Stream-ordered; nothing is enqueued on error.
 */
int agn_log_bin_count(int64_t n, double dex, int32_t* count);
int agn_periodogram_workspace_size(int32_t n_curves, const int64_t* n, double dex, size_t* bytes);
int agn_periodogram_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const int64_t* offset,
                          const double* x, const int64_t* p_offset, double* P_out, double dex,
                          const int64_t* b_offset, double* bins_out, void* ws, size_t ws_bytes,
                          void* stream);

/* ---- instrumentation ----------------------------------------------------- */

/* Turns per-kernel timing on (1) or off (0) for calls made with this context.
 * While on, every kernel launch is bracketed by two HIP events recorded on
 * the launch stream. */
int agn_ctx_set_profiling(agn_ctx* ctx, int on);

/* For failure-handling tests of the multi-pass sort.  Each scatter workgroup
 * of that sort waits, by polling, for the digit counts of the tiles before it
 * (a decoupled look-back; those tiles are always running, so the wait ends
 * within microseconds).  A wait that exceeds `polls` polls gives up: the
 * curve's iters_done reads -2 and its x_out is not valid, but every store
 * stays in bounds.  polls > 0 sets the limit, 0 restores the default
 * (2^18), polls < 0 makes every wait give up at once.  Applies to calls and
 * plans made with this context afterwards. */
int agn_ctx_set_lookback_polls(agn_ctx* ctx, int32_t polls);

/* Synchronises the recorded events and returns, for kernel `name` (one of the
 * names listed by agn_ctx_kernel_names), the summed duration in milliseconds
 * and the number of launches since the last reset; reset = 1 clears all
 * records afterwards.  Unknown name: *total_ms = 0, *launches = 0. */
int agn_ctx_kernel_time(agn_ctx* ctx, const char* name, double* total_ms, int64_t* launches,
                        int reset);

/* Comma-separated kernel names the library times.  On the multi-pass path:
 * fft_pass and fft_mid (the transform passes), sort_hist (the digit count of
 * a sort, one launch per sort), sort_scan (the digit starts), sort_scatter
 * (one launch per 8-bit pass), delta (Eq. 4 reductions), big_prep (the
 * draw's keys and their one-time sort), big_output. */
const char* agn_ctx_kernel_names(void);

/* ---- test-only exports (same conventions) ------------------------------- */

/* Philox4x64-10 blocks: out[4 b + w] = word w of block (ctr0 + b) under key
 * (key0, key1), counter (ctr0 + b, 0, 0, 0), for b < n_blocks.  out: device. */
int agn_test_philox(uint64_t key0, uint64_t key1, uint64_t ctr0, int64_t n_blocks,
                    uint64_t* out, void* stream);

/*
 * The iteration's transforms and ranking on their own, run by the same
 * kernels as agn_lc_iterate (the Stockham passes, the real-spectrum fold of
 * the replacement step, the radix sorts), so that each step can be checked
 * against its definition.  path selects the kernels:
 *   AGN_TEST_PATH_LDS  the LDS-resident kernels: one workgroup, the block
 *                      shape and LDS layout of the iteration; n must be a
 *                      length that agn_lc_iterate runs there (FP32:
 *                      n <= 2^14, or 3 * 2^a <= 12288; FP64: n <= 2^13, or
 *                      3 * 2^a <= 12288).
 *   AGN_TEST_PATH_HBM  the multi-pass kernels with the iteration's pass plan
 *                      for n (any supported n that is a multiple of 8192).
 * Arithmetic is in the working precision of prec: inputs are rounded to it
 * on load (as the iteration rounds x_i), outputs widened to double.  All
 * arrays are device memory; ws is a device workspace of
 * agn_test_workspace_size(n, prec, path) bytes.  Errors: AGN_EINVAL (NULL
 * pointers, small workspace, unknown path or precision, an x that is not
 * 16-byte aligned for the multi-pass transform), AGN_EUNSUPPORTED_N (n not of
 * the supported form or not on the chosen path); nothing is enqueued on
 * error.  Stream-ordered.
 *
 * agn_test_rfft   X_out[j] = sum_t x[t] exp(-2 pi i j t / n), j = 0 .. n/2, as
 *                 interleaved (re, im) doubles: the real DFT of App. A (Eq. A1,
 *                 taken with the negative exponent forward; the sign does not
 *                 change the iteration's output).
 * agn_test_irfft  y_out[t] = sum_j Y_j exp(+2 pi i j t / n) over the full
 *                 Hermitian spectrum built from the n/2 + 1 values Y
 *                 (interleaved re, im), unnormalised; the imaginary parts of
 *                 Y_0 and Y_{n/2} are ignored (the iteration's are zero).
 * agn_test_argsort  rank_out[t] = position of sample t in the stable ascending
 *                 order of y (ties by index, -0 == +0): the ranking of Sec.
 *                 2.1.  Keys: the order-preserving integer image of y rounded
 *                 to the working precision, except in the FP32 form on the
 *                 LDS path, where y (rounded to float) is mapped in double
 *                 precision onto 2^30 levels over [min y, max y],
 *                 key = trunc((y - min) * ((2^30 - 1) / (max - min))), so that
 *                 values closer than (max - min) 2^-30 can share a key and
 *                 are then ordered by index.
 */
/*
 * agn_test_lds_bandwidth -- measured LDS read bandwidth, the ceiling against
 * which the LDS-resident kernels' LDS traffic is rated: `blocks` workgroups
 * of 1024 threads each read a 64 KB LDS buffer `reps` times in 16-byte words
 * (consecutive lanes, consecutive words: no bank conflicts).  Bytes read:
 * blocks * reps * 65536.  *seconds = device time of the timed launch (after
 * one untimed launch); out: device, blocks * 1024 floats (the sums read, so
 * the loads cannot be elided).  Synchronises the stream.  Errors: AGN_EINVAL,
 * AGN_EDEVICE.
 */
int agn_test_lds_bandwidth(int32_t blocks, int32_t reps, float* out, double* seconds, void* stream);

enum { AGN_TEST_PATH_LDS = 0, AGN_TEST_PATH_HBM = 1 };
int agn_test_workspace_size(int64_t n, agn_precision prec, int32_t path, size_t* bytes);
int agn_test_rfft(agn_ctx* ctx, const double* x, int64_t n, agn_precision prec, int32_t path,
                  double* X_out, void* ws, size_t ws_bytes, void* stream);
int agn_test_irfft(agn_ctx* ctx, const double* Y, int64_t n, agn_precision prec, int32_t path,
                   double* y_out, void* ws, size_t ws_bytes, void* stream);
int agn_test_argsort(agn_ctx* ctx, const double* y, int64_t n, agn_precision prec, int32_t path,
                     uint32_t* rank_out, void* ws, size_t ws_bytes, void* stream);

/*
 * agn_psd_fit_batch -- the convergence test of Sec. 3.2.2: Eq. 3 fitted to
 * each curve's log-binned periodogram, as written by agn_periodogram_batch
 * with the same dex (bins_out at b_offset[c], agn_log_bin_count(n[c], dex)
 * bins).  Least squares in log10 P over the bins with a positive mean; each
 * bin sits at the mean frequency of the f_j = j / (n dt) it holds; the break
 * is held at p[c].f_br and (log10 A, a_low, a_high) are free, started from
 * p[c].a_low / p[c].a_high (Levenberg-Marquardt, FP64, one wave per curve).
 *   fit_out[4 c + {0,1,2,3}] = log10 A, a_low, a_high, rms of the log10
 *   residuals; Eq. 3 is symmetric in its slopes, so a_low is the smaller.
 *   NaN if fewer than 3 bins are positive or none lies on one side of f_br.
 * n, dt, p, b_offset: host; bins, fit_out: device.  Workspace:
 * agn_psd_fit_workspace_size.  Errors: AGN_EINVAL / AGN_EUNSUPPORTED_N,
 * including an f_br outside the binned frequency range (nothing launched).
 */
int agn_psd_fit_workspace_size(int32_t n_curves, const int64_t* n, double dex, size_t* bytes);
int agn_psd_fit_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const double* dt, const agn_psd_params* p,
                      double dex, const int64_t* b_offset, const double* bins, double* fit_out, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * Lag statistics of the output series (Eq. A6; Sec. 3.2.10; Sec. 4.2,
 * Figs. 16-17), for n_curves positive series at the same n_lags lags
 * (in samples; 1 <= lags[l] < n[c] for every curve):
 *   sf2_out[c * n_lags + l]  Eq. A6: the mean over the n - k pairs (x_i,
 *                            x_{i+k}) of (x_{i+k} - x_i)^2 with
 *                            units AGN_SF_LINEAR, or of dm^2 with
 *                            dm = -2.5 log10(x_{i+k} / x_i) (AGN_SF_MAGNITUDE;
 *                            Sec. 3.2.10);
 *   rep_out[l]               Eq. 6: the mean of sf2 over the curves (lag by lag);
 *   exceed_out[(c * n_lags + l) * n_thr + j]
 *                            pairs with |dm| > dm_ref[j] (Fig. 16), decided as
 *                            hi > lo * 10^(dm_ref[j] / 2.5) with the factor
 *                            rounded once to double; with lam_cut > 0 a value
 *                            below lam_cut is replaced by lam_cut (an upper
 *                            limit) and only pairs with a value >= lam_cut are
 *                            counted (Fig. 17);
 *   pairs_out[c * n_lags + l] the pairs counted (n - k without a cut).
 * n, offset, lags, dm_ref: host arrays; x and all outputs: device (every output
 * nullable; exceed_out required when n_thr > 0).  dm_ref ascending, >= 0, at
 * most 16 values.  x must be positive (not checked on the device).  Each
 * (curve, lag) is summed in a fixed order: results are deterministic.
 * Workspace: agn_lag_stats_workspace_size (in magnitudes it holds -2.5 log10 x,
 * 8 bytes per sample); no allocation.  Errors: AGN_EINVAL
 * (nothing is launched).
 */
enum { AGN_SF_LINEAR = 0, AGN_SF_MAGNITUDE = 1 };
int agn_lag_stats_workspace_size(int32_t n_curves, const int64_t* n, int32_t n_lags, const int64_t* lags,
                                 int32_t n_thr, int32_t units, size_t* bytes);
int agn_lag_stats_batch(agn_ctx* ctx, int32_t n_curves, const int64_t* n, const int64_t* offset, const double* x,
                        int32_t n_lags, const int64_t* lags, int32_t units, double* sf2_out, double* rep_out,
                        int32_t n_thr, const double* dm_ref, double lam_cut, uint64_t* exceed_out,
                        uint64_t* pairs_out, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* AGN_H */
