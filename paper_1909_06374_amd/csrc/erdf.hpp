// erdf.hpp -- the PDF draw of Sec. 2.1 step (ii) on the device: N values of
// L/L_Edd = 10^u, u = log10 lambda in [u_min, u_max], each the inverse CDF of
// uniform #k of Philox stream 1.  Three shapes (Sec. 2.1.1):
//   sharp broken power law (slopes as in Eq. 1, kink at u*): closed form;
//   log-normal, Eq. 2: a normal in u truncated to the support, inverted with
//     erfcinv on whichever tail keeps the argument small;
//   smooth broken power law, Eq. 1: CDF tabulated per block in LDS
//     (Gauss-Legendre per cell), search over the cells, then Newton inside
//     the cell on the exact integral until the step is below the ulp of u.
// With the dN/dlambda measure the density in u gains a factor 10^(u - u*):
// the power-law slopes drop by one and the log-normal mean moves up by
// sigma^2 ln 10; the host folds that into the parameters below.
#pragma once
#include "common.hpp"
#include "philox.hpp"

namespace agn {

// Closed forms (sharp broken power law, log-normal).
struct PdfClosed {
    int kind;              // 0 sharp broken power law, 2 log-normal
    double u_min, u_max;
    // kind 0: density 10^(-e1 (u - u*)) below u*, 10^(-e2 (u - u*)) above
    double u_star, e1, e2;
    double m1, m2;         // masses below / above u*
    double a1;             // 10^(e1 (u* - u_min))
    // kind 2: normal of mean mu and standard deviation s / sqrt(2) in u
    double mu, s;
    double c_lo, c_hi;     // normal mass below u_min, above u_max
    double tot;            // normal mass inside the support
    int64_t n;
    uint64_t seed;
    uint32_t curve_id;
    double* out;
};

__global__ __launch_bounds__(256) void k_pdf_closed(PdfClosed P) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const double ln10 = 2.30258509299404568402;
    const double U = philox_uniform(P.seed, 1, P.curve_id, (uint64_t)k);
    double u;
    if (P.kind == 0) {
        const double t = U * (P.m1 + P.m2);
        if (t < P.m1) u = (P.e1 == 0.0) ? P.u_min + t : P.u_star - log10(P.a1 - t * P.e1 * ln10) / P.e1;
        else u = (P.e2 == 0.0) ? P.u_star + (t - P.m1) : P.u_star - log10(1.0 - (t - P.m1) * P.e2 * ln10) / P.e2;
    } else {
        // mass below the draw, lo; above it, hi = c_hi + (1 - U) tot (1 - U is exact)
        const double lo = P.c_lo + U * P.tot;
        double z;
        if (lo <= 0.5) z = -erfcinv(2.0 * lo);
        else z = erfcinv(2.0 * (P.c_hi + (1.0 - U) * P.tot));
        u = P.mu + P.s * z;
    }
    u = fmin(fmax(u, P.u_min), P.u_max);
    P.out[k] = pow(10.0, u);
}

// Eq. 1: density 1 / (exp(c1 x) + exp(c2 x)) in x = u - u*, c = slope * ln 10.
constexpr int PDF_CELLS = 1024;
constexpr int PDF_THREADS = 256;
constexpr int PDF_MAX_BLOCKS = 2048;

struct PdfTable {
    double u_min, u_max, u_star, c1, c2, h;  // h = (u_max - u_min) / PDF_CELLS
    int64_t n;
    uint64_t seed;
    uint32_t curve_id;
    double* out;
};

AGN_DEV double eq1_density(const PdfTable& P, double u) {
    const double x = u - P.u_star;
    return 1.0 / (exp(P.c1 * x) + exp(P.c2 * x));
}

// Eight-point Gauss-Legendre integral of the density over [a, a + w].  The
// host keeps the break's width at two cells or more (h |c2 - c1| <= 0.5), so
// the density's complex poles lie over six cell widths from the real axis
// and the rule is exact to rounding.
AGN_DEV double eq1_integral(const PdfTable& P, double a, double w) {
    const double c = a + 0.5 * w, hw = 0.5 * w;
    const double x0 = 0.1834346424956498049, x1 = 0.5255324099163289858, x2 = 0.7966664774136267396,
                 x3 = 0.9602898564975362317;
    double s = 0.3626837833783619830 * (eq1_density(P, c - hw * x0) + eq1_density(P, c + hw * x0));
    s += 0.3137066458778872873 * (eq1_density(P, c - hw * x1) + eq1_density(P, c + hw * x1));
    s += 0.2223810344533744706 * (eq1_density(P, c - hw * x2) + eq1_density(P, c + hw * x2));
    s += 0.1012285362903762591 * (eq1_density(P, c - hw * x3) + eq1_density(P, c + hw * x3));
    return s * hw;
}

__global__ __launch_bounds__(PDF_THREADS) void k_pdf_eq1(PdfTable P) {
    constexpr int CPT = PDF_CELLS / PDF_THREADS;  // cells per thread
    constexpr int W = PDF_THREADS / 64;
    __shared__ double cum[PDF_CELLS + 1];         // CDF at the cell edges (unnormalised)
    __shared__ double fe[PDF_CELLS + 1];          // density at the cell edges
    __shared__ double wtot[W];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    // 1. table: every block builds the same one, in the same order of operations
    double pre[CPT];
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int i = tid * CPT + j;
        const double a = P.u_min + i * P.h;
        acc += eq1_integral(P, a, P.h);
        pre[j] = acc;
        fe[i] = eq1_density(P, a);
    }
    if (tid == 0) fe[PDF_CELLS] = eq1_density(P, P.u_max);
    double inc = acc;  // wave inclusive scan of the per-thread sums
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const double o = __shfl_up(inc, s, 64);
        if (lane >= s) inc += o;
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    double base = inc - acc;
    for (int v = 0; v < wv; ++v) base += wtot[v];
#pragma unroll
    for (int j = 0; j < CPT; ++j) cum[tid * CPT + j + 1] = base + pre[j];
    if (tid == 0) cum[0] = 0.0;
    __syncthreads();
    const double total = cum[PDF_CELLS];

    // 2. draws, grid-stride
    for (int64_t k = (int64_t)blockIdx.x * PDF_THREADS + tid; k < P.n; k += (int64_t)gridDim.x * PDF_THREADS) {
        const double t = philox_uniform(P.seed, 1, P.curve_id, (uint64_t)k) * total;
        int lo = 0, hi = PDF_CELLS;  // cum[lo] <= t < cum[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cum[mid] <= t) lo = mid;
            else hi = mid;
        }
        const double a = P.u_min + lo * P.h;
        const double r = t - cum[lo];
        // start: root of the integral of the linear interpolant of the density
        const double f0 = fe[lo], g = (fe[lo + 1] - f0) / P.h;
        double s = 2.0 * r / (f0 + sqrt(fmax(f0 * f0 + 2.0 * g * r, 0.0)));
        s = fmin(fmax(s, 0.0), P.h);
        // Newton on the exact integral: quadratic convergence from the start
        // above, to the ulp of u (two or three steps for moderate slopes,
        // more for cells as wide as the host allows)
        const double tol = 0x1.0p-52 * (fabs(a) + P.h);
        for (int it = 0; it < 8; ++it) {
            const double ds = (eq1_integral(P, a, s) - r) / eq1_density(P, a + s);
            s = fmin(fmax(s - ds, 0.0), P.h);
            if (fabs(ds) <= tol) break;
        }
        const double u = fmin(fmax(a + s, P.u_min), P.u_max);
        P.out[k] = pow(10.0, u);
    }
}

// Slice sampling (Neal 2003) of the same PDFs in linear lambda, as the paper
// draws them: the chain state is lambda, the target density per unit lambda
// is the shape per dex divided by lambda (measure 0) or the shape itself
// (measure 1).  One thread per chain; each step draws the level
// ln f(lambda) + ln U, then proposals uniform on [lambda_min, lambda_max],
// the interval shrunk toward the current point after each rejection (at most
// SLICE_MAX_SHRINK; the point is kept if none is accepted).  Chain c uses
// uniforms 0, 1, ... of Philox stream 6 on counter word 1 = c; after `burn`
// steps its step t writes out[t * n_chains + c] (coalesced over chains).
// Multiply-adds are not fused here (contract off), so that every proposal
// and log-density is rounded operation by operation, as in a plain C build.
constexpr int SLICE_MAX_SHRINK = 200;
constexpr uint32_t SLICE_STREAM = 6;

struct PdfSlice {
    int kind, measure;
    double u_star, d1, d2, gauss;  // gauss = 1 / (2 sigma^2 ln 10)
    double lo, hi, start;          // support and starting point in lambda
    int64_t n;
    int32_t n_chains, burn;
    uint64_t seed;
    uint32_t curve_id;
    double* out;
};

AGN_DEV double slice_lnf(const PdfSlice& P, double lam) {
#pragma clang fp contract(off)
    const double ln10 = 2.30258509299404568402;
    const double u = log10(lam), x = u - P.u_star;
    double l10;
    if (P.kind == 0) l10 = -(x < 0.0 ? P.d1 : P.d2) * x;
    else if (P.kind == 1) l10 = -log10(pow(10.0, P.d1 * x) + pow(10.0, P.d2 * x));
    else l10 = -x * x * P.gauss;
    if (P.measure == 0) l10 -= u;
    return l10 * ln10;
}

__global__ __launch_bounds__(256) void k_pdf_slice(PdfSlice P) {
#pragma clang fp contract(off)
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.n_chains || c >= P.n) return;
    double lam = P.start, lf = slice_lnf(P, lam);
    uint64_t k = 0;
    for (int64_t step = 0;; ++step) {
        const int64_t j = (step - P.burn) * (int64_t)P.n_chains + c;
        if (step >= P.burn && j >= P.n) break;
        const double level = lf + log(philox_uniform_chain(P.seed, SLICE_STREAM, P.curve_id, (uint64_t)c, k++));
        double L = P.lo, R = P.hi, next = lam, lnext = lf;
        for (int t = 0; t < SLICE_MAX_SHRINK; ++t) {
            const double U = philox_uniform_chain(P.seed, SLICE_STREAM, P.curve_id, (uint64_t)c, k++);
            const double cand = L + U * (R - L);
            const double lc = slice_lnf(P, cand);
            if (lc > level) {
                next = cand;
                lnext = lc;
                break;
            }
            if (cand < lam) L = cand;
            else R = cand;
        }
        lam = next;
        lf = lnext;
        if (step >= P.burn) P.out[j] = lam;
    }
}

}  // namespace agn
