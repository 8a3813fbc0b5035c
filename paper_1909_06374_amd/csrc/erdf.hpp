// erdf.hpp -- the PDF draw of Sec. 2.1 step (ii) on the device: N values of
// L/L_Edd from a sharp broken power law in dN/dlog10(lambda) with the slope
// convention of Eq. 1 (density 10^(-d1 (u - u_br)) below the break, 10^(-d2
// (u - u_br)) above, u = log10 lambda in [u_min, u_max]), by its closed-form
// inverse CDF applied to uniform #k of Philox stream 1.
#pragma once
#include "common.hpp"
#include "philox.hpp"

namespace agn {

struct ErdfDraw {
    double u_min, u_max, u_br, d1, d2;
    double m1, m2;         // masses below / above the break (host-computed)
    double a1;             // 10^(d1 (u_br - u_min))
    int64_t n;
    uint64_t seed;
    uint32_t curve_id;
    double* out;
};

__global__ __launch_bounds__(256) void k_erdf_draw(ErdfDraw P) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const double ln10 = 2.30258509299404568402;
    const double U = philox_uniform(P.seed, 1, P.curve_id, (uint64_t)k);
    const double t = U * (P.m1 + P.m2);
    double u;
    if (t < P.m1) u = P.u_br - log10(P.a1 - t * P.d1 * ln10) / P.d1;
    else u = P.u_br - log10(1.0 - (t - P.m1) * P.d2 * ln10) / P.d2;
    u = fmin(fmax(u, P.u_min), P.u_max);
    P.out[k] = pow(10.0, u);
}

}  // namespace agn
