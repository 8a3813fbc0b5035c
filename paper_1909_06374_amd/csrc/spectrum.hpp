// spectrum.hpp -- Timmer & Koenig Fourier moduli for the PSD of Eq. 3 on the
// Fourier grid f_j = j / (N dt) (Appendix A), with Philox4x64-10 uniforms.
//
// Only the moduli of the TK95 spectrum are used by the iteration (Sec. 2.1):
// for an interior bin, |sqrt(P/2)(g1 + i g2)|^2 = P E with E ~ Exp(1) = -ln U,
// so one uniform per bin suffices; the Nyquist bin is real,
// sqrt(P/2)|g| with g = sqrt(-2 ln Ua) cos(2 pi Ub); the DC bin is 0.
// With norm <= 0 the amplitude A of Eq. 3 is chosen so that the TK95 series
// has unit expected variance: A = N^2 / (2 sum_{0<j<N/2} P~_j + P~_{N/2}/2).
//
// Three launches: per-chunk partial sums of the weighted P~, one block per
// curve to total them (fixed order: bit-reproducible), then the moduli.
#pragma once
#include "common.hpp"
#include "philox.hpp"

namespace agn {

constexpr int SPEC_THREADS = 256;
constexpr int SPEC_CHUNK = 2048;  // bins per block

struct SpecDesc {
    int64_t n;
    double dt;
    double norm, f_br, a_low, a_high;
    uint64_t seed;
    uint32_t curve_id;
    int32_t is_f32;        // 1: amp is float, 0: double
    int64_t chunk0;        // first global chunk of this curve
    int64_t nchunk;        // chunks of N/2 + 1 bins
    void* amp;             // N/2 + 1 outputs
    double* partial;       // [nchunk]
    double* A;             // [1]
};

// Denominator of Eq. 3: (f/f_br)^a_low + (f/f_br)^a_high.
AGN_DEV double psd_den(double f, double f_br, double a_low, double a_high) {
    const double r = f / f_br;
    return pow(r, a_low) + pow(r, a_high);
}

AGN_DEV int find_curve(const SpecDesc* __restrict__ d, int nd, int64_t b) {
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].chunk0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

AGN_DEV double block_sum_f64_256(double v, double* sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    const double t = ((sh[0] + sh[1]) + (sh[2] + sh[3]));
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(SPEC_THREADS) void k_spec_partial(const SpecDesc* __restrict__ descs, int nd) {
    __shared__ double sh[4];
    const int c = find_curve(descs, nd, blockIdx.x);
    const SpecDesc& d = descs[c];
    const int64_t q = (int64_t)blockIdx.x - d.chunk0;
    const int64_t M = d.n / 2;
    const double ndt = (double)d.n * d.dt;
    double s = 0.0;
    for (int u = 0; u < SPEC_CHUNK / SPEC_THREADS; ++u) {
        const int64_t j = q * SPEC_CHUNK + (int64_t)u * SPEC_THREADS + threadIdx.x;
        if (j >= 1 && j < M) s += 2.0 * (1.0 / psd_den((double)j / ndt, d.f_br, d.a_low, d.a_high));
        else if (j == M) s += 0.5 * (1.0 / psd_den(0.5 / d.dt, d.f_br, d.a_low, d.a_high));
    }
    s = block_sum_f64_256(s, sh);
    if (threadIdx.x == 0) d.partial[q] = s;
}

__global__ __launch_bounds__(SPEC_THREADS) void k_spec_norm(const SpecDesc* __restrict__ descs) {
    __shared__ double sh[4];
    const SpecDesc& d = descs[blockIdx.x];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < d.nchunk; q += SPEC_THREADS) s += d.partial[q];
    s = block_sum_f64_256(s, sh);
    if (threadIdx.x == 0) *d.A = (d.norm > 0.0) ? d.norm : (double)d.n * (double)d.n / s;
}

__global__ __launch_bounds__(SPEC_THREADS) void k_spec_amp(const SpecDesc* __restrict__ descs, int nd) {
    const int c = find_curve(descs, nd, blockIdx.x);
    const SpecDesc& d = descs[c];
    const int64_t q = (int64_t)blockIdx.x - d.chunk0;
    const int64_t M = d.n / 2;
    const double ndt = (double)d.n * d.dt;
    const double A = *d.A;
    for (int u = 0; u < SPEC_CHUNK / SPEC_THREADS; ++u) {
        const int64_t j = q * SPEC_CHUNK + (int64_t)u * SPEC_THREADS + threadIdx.x;
        if (j > M) break;
        double a;
        if (j == 0) {
            a = 0.0;
        } else if (j < M) {
            const double P = A / psd_den((double)j / ndt, d.f_br, d.a_low, d.a_high);
            const double U = philox_uniform(d.seed, 0, d.curve_id, (uint64_t)j);
            a = sqrt(P * (-log(U)));
        } else {
            const double P = A / psd_den(0.5 / d.dt, d.f_br, d.a_low, d.a_high);
            const double Ua = philox_uniform(d.seed, 0, d.curve_id, (uint64_t)M);
            const double Ub = philox_uniform(d.seed, 0, d.curve_id, (uint64_t)M + 1);
            const double g = sqrt(-2.0 * log(Ua)) * cos(2.0 * 3.14159265358979323846 * Ub);
            a = sqrt(0.5 * P) * fabs(g);
        }
        if (d.is_f32) ((float*)d.amp)[j] = (float)a;
        else ((double*)d.amp)[j] = a;
    }
}

// Test export: raw Philox blocks.
__global__ void k_philox_blocks(uint64_t k0, uint64_t k1, uint64_t c0, int64_t nb, uint64_t* out) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    u64x4 o = philox4x64_10(c0 + (uint64_t)b, 0, 0, 0, k0, k1);
    for (int w = 0; w < 4; ++w) out[4 * b + w] = o.v[w];
}

}  // namespace agn
